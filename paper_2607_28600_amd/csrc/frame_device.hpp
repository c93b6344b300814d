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
    f.vwin = q[3];
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
        const uint32_t v[4] = {rr.x, rr.y, rr.z, rr.w};
        bool need[4], act[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            act[i] = jal + 4 * lane + i >= st.j;
            need[i] = act[i] && !gap_fast_select(F, v[i], G[i]);
        }
        // draws the margins leave: three table reads around the computed gap, or (draws smaller than
        // the window covers) the table search
        if (__ballot(need[0] || need[1] || need[2] || need[3])) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (need[i]) G[i] = v[i] >= F.vwin ? gap_window(Q, v[i], G[i]) : gap_of(Q, F.invlog2q, v[i]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) G[i] = act[i] ? G[i] : -1;
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

// Slot-flip entry of the frame kernels' scratch: shot lane | step index within
// the class << 6 | slot << 14.
__device__ __forceinline__ uint32_t flip_entry(uint32_t lane, uint32_t step, uint32_t slot) {
    return lane | (step << 6) | (slot << 14);
}

// One walk of the (class c, word w) stream with every event resolved through
// its channel record (flip-table offset | J << 26 | uniform << 32 | step << 33
// | threshold offset << 41) and its branch's slot flips (wv_fl: n | slots, or a
// list in wv_sl).  Every lane loads a channel record (inactive lanes the
// class's first), so the loads need no branch; non-uniform channels take
// their threshold search only when some lane has one.
// GEN: the flips become entries appended at out[*n_out ..] (those past cap
// are dropped, *n_out still counts them).  Otherwise apply(slot, lane bit) is
// called for each flip.  Returns whether the walk stopped at R.
template <bool GEN, typename Apply>
__device__ __forceinline__ bool walk_resolved(const DevProg &P, const GapFast &F, uint32_t c, uint32_t coff, uint64_t w,
                                              Walk &st, uint32_t R, uint32_t *tmp, uint32_t *out, uint32_t cap,
                                              uint32_t *n_out, uint32_t k0, uint32_t k1, Apply apply) {
    bool ok[4];
    uint32_t at[4], bv[4];
    const bool cut = walk_events(F, P.cls_Q + (size_t)c * 4097, c, (uint32_t)w, (uint32_t)(w >> 32), st, R, tmp, k0,
                                 k1, ok, at, bv);
    uint64_t info[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) info[i] = P.fr_chinfo[coff + (ok[i] ? at[i] >> 6 : 0u)];
    uint32_t br[4];
    bool nonuni = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t J = (uint32_t)(info[i] >> 26) & 0x3Fu;
        br[i] = (uint32_t)(((uint64_t)bv[i] * J) >> 32);
        nonuni |= ok[i] && !((info[i] >> 32) & 1u);
    }
    if (__ballot(nonuni)) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (ok[i] && !((info[i] >> 32) & 1u)) br[i] = branch_of(P.thr, info[i], bv[i]);
    }
    uint64_t fw[4];
    uint32_t nfl[4], k_lane = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        fw[i] = P.wv_fl[(uint32_t)(info[i] & 0x3FFFFFFu) + br[i]];
        const uint32_t n = (fw[i] & 3u) ? (uint32_t)(fw[i] & 3u) : (uint32_t)(fw[i] >> 8) & 0xFFFFFFu;
        nfl[i] = ok[i] ? n : 0u;
        k_lane += nfl[i];
    }
    if (GEN) {
        // flips of this lane's events go after those of the lanes below it
        const uint32_t xs = wave_incl_sum(k_lane);
        const uint32_t ktot = (uint32_t)__builtin_amdgcn_readlane((int)xs, 63);
        uint32_t o = *n_out + xs - k_lane;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t sh = at[i] & 63u, stp = (uint32_t)(info[i] >> 33) & 0xFFu;
            if (fw[i] & 3u) {
#pragma unroll
                for (uint32_t q = 0; q < 3; ++q)
                    if (q < nfl[i] && o + q < cap)
                        out[o + q] = flip_entry(sh, stp, (uint32_t)(fw[i] >> (16 + 16 * q)) & 0xFFFFu);
            } else if (nfl[i]) {
                const uint16_t *sl = P.wv_sl + (fw[i] >> 32);
                for (uint32_t q = 0; q < nfl[i]; ++q)
                    if (o + q < cap) out[o + q] = flip_entry(sh, stp, sl[q]);
            }
            o += nfl[i];
        }
        *n_out += ktot;
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const unsigned long long bit = 1ull << (at[i] & 63u);
            if (fw[i] & 3u) {
#pragma unroll
                for (uint32_t q = 0; q < 3; ++q)
                    if (q < nfl[i]) apply((uint32_t)(fw[i] >> (16 + 16 * q)) & 0xFFFFu, bit);
            } else if (nfl[i]) {
                const uint16_t *sl = P.wv_sl + (fw[i] >> 32);
                for (uint32_t q = 0; q < nfl[i]; ++q) apply((uint32_t)sl[q], bit);
            }
        }
    }
    return cut;
}

// Tables of the walk.  LT: LDS copies (compact channel records ci32 =
// flip-table offset | J << 20 of uniform channels, step bytes st8, and the
// gap table as 32-bit words q32), which phase G keeps in the slot region;
// otherwise the device program's global tables.
struct WalkLds {
    const uint32_t *ci32;
    const uint8_t *st8;
    const uint32_t *q32;
};

// Step-kernel flip entry: shot lane | (k - 1) << 6 | step << 8 | k slots of
// 12 bits from bit 16 (k = 1..4).
__device__ __forceinline__ uint32_t entry_slots(uint64_t e) { return ((uint32_t)(e >> 6) & 3u) + 1u; }
__device__ __forceinline__ uint32_t entry_slot(uint64_t e, uint32_t q) { return (uint32_t)(e >> (16 + 12 * q)) & 0xFFFu; }

// Lean walk of the (class c, word w) stream: the draws, gaps and positions of
// walk_events, each event resolved through its channel record and branch into
// its 16-byte flip record (the first two pre-packed entries, the count in the
// first one's lane bits), the four records of a lane loaded together; a lane
// whose event has more entries loads the next two from the extension, and
// past four (rare) one at a time.  Straight-line code except where some lane
// takes the table search or more than two entries.  GEN: the entries, tagged
// with shot lane and step, appended at out[n_out ..] (those past cap
// dropped, n_out still counts them); otherwise apply(entry) per entry.
// Returns whether the walk stopped at R.
template <bool GEN, bool LT, typename Apply>
__device__ __forceinline__ bool walk_entries(const DevProg &P, const WalkLds &T, const GapFast &F, uint32_t c,
                                             uint32_t coff, uint64_t w, Walk &st, uint32_t R, uint32_t *tmp,
                                             uint64_t *out, uint32_t cap, uint32_t &n_out, uint32_t k0, uint32_t k1,
                                             Apply apply) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wlo = (uint32_t)w, whi = (uint32_t)(w >> 32);
    const uint64_t *Q = P.cls_Q + (size_t)c * 4097;
    const uint32_t jal = st.j & ~3u;
    const uint4 rr = philox4x32_10(make_uint4((jal >> 2) + lane, wlo, c, (1u << 24) | whi), k0, k1);
    const uint32_t v[4] = {rr.x, rr.y, rr.z, rr.w};
    // G[i] = -1: a draw before the stream's position (only lane 0's first draws can be)
    int G[4];
    bool need[4], act[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        act[i] = lane != 0 || (uint32_t)i >= st.j - jal;
        const bool fast = gap_fast_lean(F, v[i], G[i]);
        need[i] = act[i] & !fast;
    }
    if (__ballot(need[0] | need[1] | need[2] | need[3])) {
        // the window's three table reads for every draw, issued together (indices clamped into the
        // table), then the draws the window does not cover take the table search
        uint64_t q[4][3];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int k = min(max(G[i] - 1 + d, 0), 4096);
                q[i][d] = LT ? (uint64_t)T.q32[(size_t)c * 4097 + k] : Q[k];
            }
        bool slow = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int g = G[i] - 2;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int k = G[i] - 1 + d;
                g += (k <= 0 || (k <= 4096 && (uint64_t)v[i] < q[i][d])) ? 1 : 0;
            }
            const bool win = v[i] >= F.vwin;
            G[i] = need[i] && win ? g : G[i];
            need[i] = need[i] && !win;
            slow |= need[i];
        }
        if (__ballot(slow)) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (need[i]) G[i] = gap_of(Q, F.invlog2q, v[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) G[i] = act[i] ? G[i] : -1;
    // advance of each draw (0 for inactive ones) and whether it is an event
    uint32_t adv[4], isev[4], inc = 0, nev = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        isev[i] = (G[i] >= 0 && G[i] < 4096) ? 1u : 0u;
        adv[i] = G[i] < 0 ? 0u : (G[i] == 4096 ? 4096u : (uint32_t)G[i] + 1u);
        inc += adv[i];
        nev += isev[i];
    }
    // (events << 23 | advance): a walk advances at most 2^20 positions and finds at most 256 events
    const uint32_t mine = (nev << 23) | inc;
    const uint32_t x = wave_incl_sum(mine);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
    const uint32_t ex = x - mine;
    const uint32_t eb = st.e & ~3u, elim = eb + 256u;
    // per draw: the stream position before it, its event position and its event index
    uint32_t base[4], evi[4], cutm = 0;
    {
        uint32_t pp = st.pos + (ex & 0x7FFFFFu), ee = st.e + (ex >> 23);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            base[i] = pp;
            evi[i] = ee;
            const uint32_t at = pp + (uint32_t)(G[i] < 0 ? 0 : G[i]);
            cutm |= (isev[i] && (at >= R || ee >= elim)) ? (1u << i) : 0u;
            ee += isev[i];
            pp += adv[i];
        }
    }
    const uint32_t ci = cutm ? (uint32_t)__ffs(cutm) - 1u : 0u;  // this lane's first cut draw
    const uint64_t bal = __ballot(cutm != 0);
    uint32_t n_pos, n_e, n_j;
    bool cutR;
    if (bal) {
        const uint32_t cl = (uint32_t)(__ffsll((long long)bal) - 1);
        const uint32_t cp = ci == 0 ? base[0] : ci == 1 ? base[1] : ci == 2 ? base[2] : base[3];
        const uint32_t ce = ci == 0 ? evi[0] : ci == 1 ? evi[1] : ci == 2 ? evi[2] : evi[3];
        const int cg = ci == 0 ? G[0] : ci == 1 ? G[1] : ci == 2 ? G[2] : G[3];
        n_pos = (uint32_t)__builtin_amdgcn_readlane((int)cp, (int)cl);
        n_e = (uint32_t)__builtin_amdgcn_readlane((int)ce, (int)cl);
        n_j = jal + 4 * cl + (uint32_t)__builtin_amdgcn_readlane((int)ci, (int)cl);
        cutR = n_pos + (uint32_t)__builtin_amdgcn_readlane(cg, (int)cl) >= R;
    } else {
        n_pos = st.pos + (total & 0x7FFFFFu);
        n_e = st.e + (total >> 23);
        n_j = jal + 256;
        cutR = false;
    }
    // positions of the kept events (before the cut), by event index
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (isev[i] && evi[i] < n_e) tmp[evi[i] - eb] = base[i] + (uint32_t)G[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // branch draws: lane l owns events eb + 4l .. eb + 4l + 3, one Philox block
    const uint4 bb = philox4x32_10(make_uint4((eb >> 2) + lane, wlo, c, (2u << 24) | whi), k0, k1);
    const uint32_t bw[4] = {bb.x, bb.y, bb.z, bb.w};
    bool ok[4];
    uint32_t at[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t ev = eb + 4 * lane + i;
        ok[i] = ev >= st.e && ev < n_e;
        at[i] = tmp[4 * lane + i];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    st.pos = n_pos;
    st.e = n_e;
    st.j = n_j;
    // resolve: channel record (inactive lanes read the class's first), branch, flip record index
    uint32_t fi[4], stp[4];
    if (LT) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t rk = coff + (ok[i] ? at[i] >> 6 : 0u);
            const uint32_t ci32 = T.ci32[rk];
            stp[i] = T.st8[rk];
            fi[i] = (ci32 & 0xFFFFFu) + (uint32_t)(((uint64_t)bw[i] * (ci32 >> 20)) >> 32);
        }
    } else {
        uint64_t info[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) info[i] = P.fr_chinfo[coff + (ok[i] ? at[i] >> 6 : 0u)];
        uint32_t br[4];
        bool nonuni = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            br[i] = (uint32_t)(((uint64_t)bw[i] * ((uint32_t)(info[i] >> 26) & 0x3Fu)) >> 32);
            nonuni |= ok[i] && !((info[i] >> 32) & 1u);
        }
        if (__ballot(nonuni)) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (ok[i] && !((info[i] >> 32) & 1u)) br[i] = branch_of(P.thr, info[i], bw[i]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            fi[i] = (uint32_t)(info[i] & 0x3FFFFFFu) + br[i];
            stp[i] = (uint32_t)(info[i] >> 33) & 0xFFu;
        }
    }
    // the four flip records of the lane, 16 bytes each, loaded together
    uint4 ra[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[i] = ((const uint4 *)P.fr_frec)[fi[i]];
    // entries per event; past two, the extension offset (in 16-byte units) held in the records' idle bits
    uint32_t m[4], k_lane = 0, xm = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        m[i] = ok[i] ? (ra[i].x & 63u) : 0u;
        xm |= m[i] > 2 ? (1u << i) : 0u;
        k_lane += m[i];
    }
    uint4 rb[4];
    const bool more = __ballot(xm != 0) != 0;
    if (more) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            rb[i] = make_uint4(0, 0, 0, 0);
            if ((xm >> i) & 1u) {
                const uint32_t x = ((ra[i].x >> 8) & 0xFFu) | ((ra[i].z & 63u) << 8) | (((ra[i].z >> 8) & 0xFFu) << 14);
                rb[i] = ((const uint4 *)P.fr_fl3)[x];
            }
        }
    }
    uint32_t o = 0;
    if (GEN) {
        const uint32_t xs = wave_incl_sum(k_lane);
        const uint32_t ktot = (uint32_t)__builtin_amdgcn_readlane((int)xs, 63);
        o = n_out + xs - k_lane;
        n_out += ktot;
    }
    // bits 0..5 and 8..15 of a stored entry (count, extension offset) give way to the tag
    const uint64_t keep = ~0xFF3Full;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t tag = (uint64_t)(at[i] & 63u) | ((uint64_t)stp[i] << 8);
        uint64_t e[4] = {((((uint64_t)ra[i].y << 32) | ra[i].x) & keep) | tag,
                         ((((uint64_t)ra[i].w << 32) | ra[i].z) & keep) | tag, 0, 0};
        if (more) {
            e[2] = (((uint64_t)rb[i].y << 32) | rb[i].x) | tag;
            e[3] = (((uint64_t)rb[i].w << 32) | rb[i].z) | tag;
        }
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            if (q < m[i]) {
                if (GEN) {
                    if (o + q < cap) out[o + q] = e[q];
                } else {
                    apply(e[q]);
                }
            }
        }
        if (more && m[i] > 4) {
            const uint32_t x = ((ra[i].x >> 8) & 0xFFu) | ((ra[i].z & 63u) << 8) | (((ra[i].z >> 8) & 0xFFu) << 14);
            const uint64_t *l = P.fr_fl3 + 2 * (size_t)x;
            for (uint32_t q = 4; q < m[i]; ++q) {
                if (GEN) {
                    if (o + q < cap) out[o + q] = l[q - 2] | tag;
                } else {
                    apply(l[q - 2] | tag);
                }
            }
        }
        o += m[i];
    }
    return cutR;
}

}  // namespace symft
