// philox.hpp -- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) for gfx950,
// and the geometric-gap search of the draw contract.
// Ten rounds of two 32x32->64 multiplies with the published multipliers and
// Weyl key increments.  Used by the draw contract: key = (seed lo, seed hi),
// counter top byte = draw domain (1 gap, 2 branch, 3 random measurement,
// 4 active-measurement uniform).
#pragma once

#include <hip/hip_runtime.h>

#include "device_program.hpp"

namespace symft {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one v_mad_u64_u32 per product gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// G = max { g in [0, 4096] : v < Q[g] }.  Q[g] ~ 2^32 q^g, so g ~ log2(v/2^32) / log2(q);
// the guess is then moved until the exact table brackets v.
__device__ __forceinline__ int gap_of(const uint64_t *__restrict__ Q, float invlog2q, uint32_t v) {
    const float x = ((float)v + 0.5f) * 2.3283064365386963e-10f;
    int g = (int)fminf(__log2f(x) * invlog2q, 4096.0f);
    g = g < 0 ? 0 : g;
#pragma unroll 1
    for (int it = 0; it < 6; ++it) {
        if ((uint64_t)v >= Q[g]) { --g; continue; }
        if (g < 4096 && (uint64_t)v < Q[g + 1]) { ++g; continue; }
        return g;
    }
    if ((uint64_t)v < Q[4096]) return 4096;
    int lo = 0, hi = 4096;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((uint64_t)v < Q[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

// The same decision without branches (every lane evaluates every term, so a
// wave decides its 4 x 64 draws in straight-line code): G is the gap and the
// result says whether the margins decided it; lanes it does not decide take
// the table search.
__device__ __forceinline__ bool gap_fast_select(const GapFast &F, uint32_t v, int &G) {
    const float vf = (float)v;
    const float t = __log2f(vf * 2.3283064365386963e-10f) * F.invlog2q;
    const int g0 = (int)t;
    const float fr = t - (float)g0;
    const bool margin = fr >= F.A * __builtin_amdgcn_rcpf(vf) + F.eps && fr < 1.0f - F.eps;
    const bool below = (uint64_t)v < F.qW;
    const bool ok = (uint64_t)v >= F.vmin && g0 < 4096 && margin;
    G = below ? 4096 : g0;
    return below || ok;
}

// The decision the walks take: gap_fast_select with the margin test
// frac(t) >= A / v + eps rewritten as frac(t) v >= A + eps v (no reciprocal;
// the rounding of the two products is far inside the 1.25 inflation of A).
// Draws of 0 fail it (0 >= A), which the table then decides.
__device__ __forceinline__ bool gap_fast_lean(const GapFast &F, uint32_t v, int &G) {
    const float vf = (float)v;
    const float t = __log2f(vf * 2.3283064365386963e-10f) * F.invlog2q;
    const int g0 = (int)t;
    const float fr = t - (float)g0;
    const bool margin = fr * vf >= __builtin_fmaf(F.eps, vf, F.A) && fr < 1.0f - F.eps;
    const bool below = (uint64_t)v < F.qW;
    const bool ok = (uint64_t)v >= F.vmin && g0 < 4096 && margin;
    G = below ? 4096 : g0;
    return below || ok;
}

// G from the computed g0 = floor(t) by the window rule of GapFast (v >= vwin):
// Q[k] for k < 0 counts as above every draw, for k > 4096 as 0.
__device__ __forceinline__ int gap_window(const uint64_t *__restrict__ Q, uint32_t v, int g0) {
    int G = g0 - 2;
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
        const int k = g0 + d;
        const uint64_t q = k < 0 ? ~0ull : k > 4096 ? 0ull : Q[k];
        G += (uint64_t)v < q ? 1 : 0;
    }
    return G;
}

__device__ __forceinline__ bool gap_fast(const GapFast &F, uint32_t v, int &G) {
    if ((uint64_t)v < F.qW) {
        G = 4096;
        return true;
    }
    if ((uint64_t)v < F.vmin) return false;
    const float vf = (float)v;
    const float t = __log2f(vf * 2.3283064365386963e-10f) * F.invlog2q;
    const int g0 = (int)t;
    const float fr = t - (float)g0;
    G = g0;
    return g0 < 4096 && fr >= F.A * __builtin_amdgcn_rcpf(vf) + F.eps && fr < 1.0f - F.eps;
}

}  // namespace symft
