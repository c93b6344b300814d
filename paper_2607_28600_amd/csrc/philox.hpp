// philox.hpp -- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) for gfx950.
// Ten rounds of two 32x32->64 multiplies with the published multipliers and
// Weyl key increments.  Used by the draw contract: key = (seed lo, seed hi),
// counter top byte = draw domain (1 gap, 2 branch, 3 random measurement,
// 4 active-measurement uniform).
#pragma once

#include <hip/hip_runtime.h>

namespace symft {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
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

}  // namespace symft
