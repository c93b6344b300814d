// frame_device.hpp -- device helpers shared by the two pure-frame kernels
// (sample_frame.hip, sample_frame_wave.hip): constant-address-space reads of
// wave-uniform program data, the noise draw contract's per-class constants,
// channel branch decisions, wave prefix sums and the RandomMeas column.
#pragma once

#include <hip/hip_runtime.h>

#include "device_program.hpp"
#include "philox.hpp"

namespace symft {

// Program data read with wave-uniform indices goes through the constant
// address space, so it is fetched by scalar loads: those are counted apart
// from vector memory, and never wait behind the row stores in flight.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> uniform(const T *p) {
    return (cptr<T>)p;
}

__device__ __forceinline__ GapFast load_fast(const GapFast *p, uint32_t c) {
    const cptr<uint32_t> q = uniform((const uint32_t *)(p + c));
    GapFast f;
    f.invlog2q = __uint_as_float(q[0]);
    f.A = __uint_as_float(q[1]);
    f.eps = __uint_as_float(q[2]);
    f.pad = 0;
    f.qW = (uint64_t)q[4] | ((uint64_t)q[5] << 32);
    f.vmin = (uint64_t)q[6] | ((uint64_t)q[7] << 32);
    return f;
}

struct FrWord {
    uint32_t pos, j, e, pad;  // class stream state: next position, draw, event index
};

__device__ __forceinline__ uint32_t pick4(uint4 r, uint32_t i) {
    return i == 0 ? r.x : i == 1 ? r.y : i == 2 ? r.z : r.w;
}

// Channel record: flip-table offset | J << 26 | uniform << 32 | step << 33 | thr_off << 41.
__device__ __forceinline__ uint32_t branch_of(const uint64_t *thr, uint64_t info, uint32_t bv) {
    const uint32_t J = (uint32_t)(info >> 26) & 0x3Fu;
    if ((info >> 32) & 1u) return (uint32_t)(((uint64_t)bv * J) >> 32);
    const uint64_t t0 = info >> 41;
    for (uint32_t t = 0; t < J; ++t)
        if ((uint64_t)bv < thr[t0 + t]) return t;
    return J - 1;
}

struct Walk {
    uint32_t pos, j, e;
};

// Flip-table word of a (channel, branch): its single flip entry (slot count
// in bits 6..7, nonzero), or entry count (bits 0..5) | first entry << 8.
__device__ __forceinline__ bool flip_inline(uint64_t fw) { return ((fw >> 6) & 3u) != 0; }
__device__ __forceinline__ uint32_t flip_count(uint64_t fw) { return flip_inline(fw) ? 1u : (uint32_t)(fw & 63u); }

// Inclusive prefix sum over the 64 lanes of a wave by DPP: a 4-lane window
// inside each row of 16 (row shifts 1..3), then banks (row shifts 4 and 8
// into the upper banks), then rows (broadcasts of lanes 15 and 31).
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    const int xi = (int)x;
    uint32_t s = x;
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0x111, 0xf, 0xf, true);  // row_shr:1
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0x112, 0xf, 0xf, true);  // row_shr:2
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, xi, 0x113, 0xf, 0xf, true);  // row_shr:3
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x114, 0xf, 0xe, false);  // row_shr:4, banks 1-3
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x118, 0xf, 0xc, false);  // row_shr:8, banks 2-3
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x142, 0xa, 0xf, false);  // row_bcast:15, rows 1, 3
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x143, 0xc, 0xf, false);  // row_bcast:31, rows 2, 3
    return s;
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ unsigned long long word_mask(uint64_t wi, uint64_t shots) {
    const uint64_t s0 = wi * 64;
    if (s0 + 64 <= shots) return ~0ull;
    if (s0 >= shots) return 0ull;
    return (1ull << (shots - s0)) - 1ull;
}

__device__ __forceinline__ unsigned long long rm_word(uint32_t t, uint64_t w, uint32_t k0, uint32_t k1) {
    const uint4 o = philox4x32_10(make_uint4(t >> 1, (uint32_t)w, 0u, (3u << 24) | (uint32_t)(w >> 32)), k0, k1);
    return (t & 1) ? ((uint64_t)o.z | ((uint64_t)o.w << 32)) : ((uint64_t)o.x | ((uint64_t)o.y << 32));
}


// One walk of the noise stream (class c, word w) under the draw contract: the
// 256 gap draws from st.j (aligned down to a Philox block, earlier draws of
// the block ignored), decided table-free except near a boundary, turned into
// positions by a wave prefix sum, and cut before the first event at a position
// >= R or with an index past the 64 branch blocks that start at st.e & ~3.
// Lane l then holds events eb + 4l .. eb + 4l + 3 (eb = st.e & ~3): ok[i]
// marks the ones this walk made, at[i] is the position (channel rank * 64 +
// shot lane) and bv[i] the branch draw.  tmp (256 words, private to the wave)
// carries positions between the lanes.  Advances st; returns whether the walk
// stopped at R.
__device__ __forceinline__ bool walk_events(const GapFast &F, const uint64_t *Q, uint32_t c, uint32_t wlo, uint32_t whi,
                                            Walk &st, uint32_t R, uint32_t *tmp, uint32_t k0, uint32_t k1,
                                            bool ok[4], uint32_t at[4], uint32_t bv[4]) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t jal = st.j & ~3u;
    const uint4 rr = philox4x32_10(make_uint4((jal >> 2) + lane, wlo, c, (1u << 24) | whi), k0, k1);
    int G[4];
    {
        bool n[4];
        const uint32_t v[4] = {rr.x, rr.y, rr.z, rr.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool a = jal + 4 * lane + i >= st.j;
            int g = 0;
            n[i] = a && !gap_fast(F, v[i], g);
            G[i] = a ? g : -1;
        }
        // exact table search for the draws that fell outside the margins
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (n[i]) G[i] = gap_of(Q, F.invlog2q, v[i]);
    }
    uint32_t inc = 0, nev = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (G[i] >= 0) {
            inc += G[i] == 4096 ? 4096u : (uint32_t)G[i] + 1u;
            nev += G[i] < 4096 ? 1u : 0u;
        }
    }
    // (events << 23 | advance): a walk advances at most 2^20 positions and finds at most 256 events
    const uint32_t mine = (nev << 23) | inc;
    const uint32_t x = wave_incl_sum(mine);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
    const uint32_t ex = x - mine;
    const uint32_t p = st.pos + (ex & 0x7FFFFFu), e = st.e + (ex >> 23);
    const uint32_t eb = st.e & ~3u, elim = eb + 256u;
    int cut_i = 4;
    uint32_t cut_p = 0, cut_e = 0, cut_r = 0;
    {
        uint32_t pp = p, ee = e;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (G[i] >= 0) {
                if (G[i] < 4096 && cut_i == 4 && (pp + (uint32_t)G[i] >= R || ee >= elim)) {
                    cut_i = i;
                    cut_p = pp;
                    cut_e = ee;
                    cut_r = pp + (uint32_t)G[i] >= R ? 1u : 0u;
                }
                if (G[i] < 4096) ++ee;
                pp += G[i] == 4096 ? 4096u : (uint32_t)G[i] + 1u;
            }
        }
    }
    const uint64_t bal = __ballot(cut_i < 4);
    const uint32_t cut_lane = bal ? (uint32_t)(__ffsll((long long)bal) - 1) : 64u;
    uint32_t n_pos, n_e, n_j;
    bool cutR;
    if (cut_lane < 64) {
        n_pos = (uint32_t)__builtin_amdgcn_readlane((int)cut_p, (int)cut_lane);
        n_e = (uint32_t)__builtin_amdgcn_readlane((int)cut_e, (int)cut_lane);
        n_j = jal + 4 * cut_lane + (uint32_t)__builtin_amdgcn_readlane(cut_i, (int)cut_lane);
        cutR = __builtin_amdgcn_readlane((int)cut_r, (int)cut_lane) != 0;
    } else {
        n_pos = st.pos + (total & 0x7FFFFFu);
        n_e = st.e + (total >> 23);
        n_j = jal + 256;
        cutR = false;
    }
    // positions of the kept events, by event index
    {
        uint32_t pp = p, ee = e;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (G[i] >= 0) {
                const bool before = lane < cut_lane || (lane == cut_lane && i < cut_i);
                if (before && G[i] < 4096) tmp[ee - eb] = pp + (uint32_t)G[i];
                if (G[i] < 4096) ++ee;
                pp += G[i] == 4096 ? 4096u : (uint32_t)G[i] + 1u;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // branch draws: lane l owns events eb + 4l .. eb + 4l + 3, one Philox block
    const uint4 bb = philox4x32_10(make_uint4((eb >> 2) + lane, wlo, c, (2u << 24) | whi), k0, k1);
    const uint32_t bw[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        const uint32_t ev = eb + 4 * lane + i;
        ok[i] = ev >= st.e && ev < n_e;
        at[i] = ok[i] ? tmp[4 * lane + i] : 0u;
        bv[i] = bw[i];
    }
    // every lane has read tmp before the next walk writes it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    st.pos = n_pos;
    st.e = n_e;
    st.j = n_j;
    return cutR;
}

}  // namespace symft
