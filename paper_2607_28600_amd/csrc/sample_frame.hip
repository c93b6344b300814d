// sample_frame.hip -- pure-frame sampling (peak active width 0) for gfx950.
//
// A workgroup owns a tile of TW = 16 or 32 consecutive 64-shot words.  One
// uint64 holds one row of one word's 64 shots, so a row of a tile is one or two
// aligned 128-byte lines of the record-major output.  32-word tiles (16 waves,
// one workgroup per CU) spend each barrier step on twice the words; they are
// taken when the schedule's slots fit LDS at that width.  Per tile:
//  * phase G (no barriers): the waves share out the tile's words and draw
//    every noise event of each (word, probability class) stream under the
//    draw contract -- walks of 64 lanes x 4 gap draws decided without the
//    table except near a boundary, a 32-bit wave scan turning gaps into
//    positions, one branch-draw Philox block per lane -- and turn each event
//    into its pre-packed flip entries (shot lane, NOISE step, up to three
//    slots), written in stream order to the workgroup's scratch, which stays
//    in L2 / the Infinity Cache;
//  * phase S: the push-based schedule (launch_args.hpp), a barrier after
//    every step.  NOISE: each wave streams its words' entries of the step and
//    XORs the lane bits into the slots.  EMIT: lanes take (node, 4 words),
//    read and clear the node's four slot words, add its constant or
//    RandomMeas words, store 32 bytes of its row and XOR the values into its
//    successors' slots.
// A (word, class) stream with more entries than its capacity (8 standard
// deviations above the mean) is instead walked afresh at every NOISE step
// and applied at once, so records never depend on the capacity.
// Aggregate-count mode (paper Sec. 6) writes no rows: EMIT ORs postselected
// detectors and (expected-value-corrected) observables into per-word flag
// words, and each tile ends by writing its discarded / logical-error flags.
// A word's 64 shots run bit-parallel, so a discarded shot cannot stop early.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "frame_device.hpp"
#include "launch_args.hpp"
#include "philox.hpp"

namespace symft {

// Tile shape, by tile width TW (16 or 32 words): TW / 2 waves, each walking
// two words in phase G and streaming two words' entries in NOISE steps; an
// EMIT step gives each thread one (node, 4 words) of up to FR_LEVEL_MAX nodes.
template <uint32_t TW>
struct Tile {
    static_assert(TW == 16 || TW == 32, "tile of 16 or 32 words");
    static constexpr uint32_t NWC = TW / 2;                    // waves
    static constexpr uint32_t WPW = TW / NWC;                  // words per wave in NOISE steps
    static constexpr uint32_t QPN = TW / 4;                    // word quads per node
    static constexpr uint32_t STG_WORDS = FR_LEVEL_MAX * TW;   // staged u64
    static_assert(FR_LEVEL_MAX * QPN == NWC * 64, "one (node, 4 words) per thread");
};

// Slot array: slot s holds the tile's TW words at s * TW + (w ^ (s & (TW - 1))).
// The swizzle spreads one word column over the LDS banks (an unswizzled column
// sits in one bank pair, so 64 lanes XOR-ing random slots of one word would
// serialise); the four words wl .. wl + 3 of an aligned quad stay one 32-byte
// block, word wl + i at element i ^ (s & 3).
template <uint32_t TW>
__device__ __forceinline__ unsigned long long *slot_word(unsigned long long *slots, uint32_t s, uint32_t w) {
    return &slots[(size_t)s * TW + (w ^ (s & (TW - 1)))];
}
template <uint32_t TW>
__device__ __forceinline__ unsigned long long *slot_quad(unsigned long long *slots, uint32_t s, uint32_t wl) {
    return &slots[(size_t)s * TW + (wl ^ (s & (TW - 4)))];
}

// Flip entry: lane | cnt << 6 | step << 8 | s0 << 16 | s1 << 32 | s2 << 48,
// applied to word wl of the tile.
template <uint32_t TW>
__device__ __forceinline__ void apply_entry(uint64_t e, unsigned long long *slots, uint32_t wl) {
    const unsigned long long bit = 1ull << (e & 63u);
    const uint32_t cnt = (uint32_t)(e >> 6) & 3u;
    atomicXor(slot_word<TW>(slots, (uint32_t)(e >> 16) & 0xFFFFu, wl), bit);
    if (cnt > 1) atomicXor(slot_word<TW>(slots, (uint32_t)(e >> 32) & 0xFFFFu, wl), bit);
    if (cnt > 2) atomicXor(slot_word<TW>(slots, (uint32_t)(e >> 48), wl), bit);
}

// XOR v[0 .. 3] into words wl .. wl + 3 of slot s.
template <uint32_t TW>
__device__ __forceinline__ void push_quad(unsigned long long *slots, uint32_t s, uint32_t wl, const unsigned long long *v) {
    unsigned long long *d = slot_quad<TW>(slots, s, wl);
    const uint32_t x = s & 3u;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) atomicXor(d + (i ^ x), v[i]);
}

// The program tables a walk reads (passed by value, so an out-of-line walk
// needs no copy of the whole program descriptor).
struct WalkTabs {
    const uint64_t *chinfo, *fltab, *fl3, *thr;
};

__device__ __forceinline__ WalkTabs walk_tabs(const DevProg &P) { return WalkTabs{P.fr_chinfo, P.fr_fltab, P.fr_fl3, P.thr}; }

// One walk of the stream (class c, word w): the 256 gap draws from st.j
// (aligned down to a Philox block), cut before the first event at a position
// >= R or with an index past the 64 branch blocks that start at st.e & ~3.
// tmp (256 words, private to the wave) carries event positions between the
// two phases.  Each event becomes its flip entries: GEN appends them to
// out[*n_out ...] (those past `cap` are dropped, *n_out still counts them);
// otherwise they are applied to the word's slot column.  Returns whether the
// walk stopped at R.
template <uint32_t TW, bool GEN>
__device__ __forceinline__ bool walk(const WalkTabs &T, const GapFast &F, const uint64_t *Q, uint32_t c, uint32_t coff, uint32_t wlo,
                     uint32_t whi, Walk &st, uint32_t R, uint32_t *tmp, uint64_t *out, uint32_t cap,
                     uint32_t *n_out, unsigned long long *slots, uint32_t wl, uint32_t k0, uint32_t k1) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t jal = st.j & ~3u;
    const uint4 rr = philox4x32_10(make_uint4((jal >> 2) + lane, wlo, c, (1u << 24) | whi), k0, k1);
    int G0, G1, G2, G3;
    bool n0, n1, n2, n3;
    {
        const uint32_t jl = jal + 4 * lane;
        const bool a0 = jl + 0 >= st.j, a1 = jl + 1 >= st.j, a2 = jl + 2 >= st.j, a3 = jl + 3 >= st.j;
        int g0 = 0, g1 = 0, g2 = 0, g3 = 0;
        n0 = a0 && !gap_fast(F, rr.x, g0);
        n1 = a1 && !gap_fast(F, rr.y, g1);
        n2 = a2 && !gap_fast(F, rr.z, g2);
        n3 = a3 && !gap_fast(F, rr.w, g3);
        G0 = a0 ? g0 : -1;
        G1 = a1 ? g1 : -1;
        G2 = a2 ? g2 : -1;
        G3 = a3 ? g3 : -1;
    }
    // exact table search for the draws that fell outside the margins
    while (n0 || n1 || n2 || n3) {
        const uint32_t v = n0 ? rr.x : n1 ? rr.y : n2 ? rr.z : rr.w;
        const int g = gap_of(Q, F.invlog2q, v);
        if (n0) {
            G0 = g;
            n0 = false;
        } else if (n1) {
            G1 = g;
            n1 = false;
        } else if (n2) {
            G2 = g;
            n2 = false;
        } else {
            G3 = g;
            n3 = false;
        }
    }
    const int G[4] = {G0, G1, G2, G3};
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
    uint64_t fw[4], tag[4];
    uint32_t k_lane = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        const uint32_t ev = eb + 4 * lane + i;
        fw[i] = 0;
        tag[i] = 0;
        if (ev >= st.e && ev < n_e) {
            const uint32_t at = tmp[4 * lane + i];
            const uint64_t info = T.chinfo[coff + (at >> 6)];
            const uint32_t fi = (uint32_t)(info & 0x3FFFFFFu) + branch_of(T.thr, info, pick4(bb, i));
            fw[i] = T.fltab[fi];
            tag[i] = (uint64_t)(at & 63u) | (((info >> 33) & 0xFFu) << 8);
            k_lane += flip_count(fw[i]);
        }
    }
    if (GEN) {
        // entries of this lane's events go after those of the lanes below it
        const uint32_t xs = wave_incl_sum(k_lane);
        const uint32_t ktot = (uint32_t)__builtin_amdgcn_readlane((int)xs, 63);
        uint32_t o = *n_out + xs - k_lane;
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            if (flip_inline(fw[i])) {
                if (o < cap) out[o] = fw[i] | tag[i];
                ++o;
                continue;
            }
            const uint32_t k = flip_count(fw[i]);
            const uint64_t f0 = fw[i] >> 8;
            for (uint32_t q = 0; q < k; ++q, ++o)
                if (o < cap) out[o] = T.fl3[f0 + q] | tag[i];
        }
        *n_out += ktot;
    } else {
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            if (flip_inline(fw[i])) {
                apply_entry<TW>(fw[i] | tag[i], slots, wl);
                continue;
            }
            const uint32_t k = flip_count(fw[i]);
            const uint64_t f0 = fw[i] >> 8;
            for (uint32_t q = 0; q < k; ++q) apply_entry<TW>(T.fl3[f0 + q] | tag[i], slots, wl);
        }
    }
    st.pos = n_pos;
    st.e = n_e;
    st.j = n_j;
    return cutR;
}


// Walk the word's class stream up to the end R of this step, applying events at once.
template <uint32_t TW>
__device__ __forceinline__ void noise_direct(WalkTabs T, GapFast F, const uint64_t *Q, uint32_t c, uint32_t coff,
                                          uint32_t R, uint64_t w, FrWord *S, uint32_t *tmp, unsigned long long *slots,
                                          uint32_t wl,
                                          uint32_t k0, uint32_t k1) {
    Walk st = {rfl(S->pos), rfl(S->j), rfl(S->e)};
    if (st.pos >= R) return;
    while (!walk<TW, false>(T, F, Q, c, coff, (uint32_t)w, (uint32_t)(w >> 32), st, R, tmp, nullptr, 0, nullptr, slots, wl,
                        k0, k1) &&
           st.pos < R) {
    }
    if ((threadIdx.x & 63u) == 0) {
        S->pos = st.pos;
        S->j = st.j;
        S->e = st.e;
    }
}

// One (node, 4 words) of an EMIT step: the four slot words are read and
// cleared, the node's constant and RandomMeas words added, the values staged
// for the next step's stores (with the node's row, or FR_NO_ROW when the row
// is not written) and XOR-ed into the successors' slots.  Thread q always
// stages at the same place, so it stores the previous step's chunk and
// stages the next one in program order without a second buffer.
template <uint32_t TW>
__device__ __forceinline__ void emit_quad(const DevProg &P, const FrameArgs &A, uint4 ra, uint4 rb, uint32_t q,
                                          uint64_t wt, unsigned long long *slots, unsigned long long *stg,
                                          uint32_t *rows, unsigned long long *fl, uint32_t k0, uint32_t k1) {
    const uint32_t vi = q / Tile<TW>::QPN, wl = 4 * (q % Tile<TW>::QPN);
    const uint32_t flags = ra.x >> 24;
    const unsigned long long c = (flags & 1u) ? ~0ull : 0ull;
    unsigned long long v[4] = {c, c, c, c};
    {
        // a node with no contributions reads the extra slot past the schedule's, which stays zero
        const uint32_t sl = ra.x & 0xFFFFFFu, x = sl & 3u;
        unsigned long long *sp = slot_quad<TW>(slots, sl, wl);
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) v[i] ^= sp[i ^ x];
        ((ulonglong2 *)sp)[0] = make_ulonglong2(0ull, 0ull);
        ((ulonglong2 *)sp)[1] = make_ulonglong2(0ull, 0ull);
    }
    if (flags & 4u) {
        // one word at a time (four Philox blocks in flight would spill registers):
        // each pass adds the word to v[0] and rotates, which after four passes
        // leaves every word back in place
        const uint64_t w = A.word_begin + wt + wl;
#pragma unroll 1
        for (uint32_t i = 0; i < 4; ++i) {
            const unsigned long long t = v[0] ^ rm_word(ra.z, w + i, k0, k1);
            v[0] = v[1];
            v[1] = v[2];
            v[2] = v[3];
            v[3] = t;
        }
    }
    if (A.cnt.on) {
        // aggregate counts: a postselected detector ORs into the discarded
        // flags, an observable (XOR its expected value) into the logical ones
        const uint32_t sec = (flags >> 4) & 3u;
        if (sec == 2u) {
            const uint32_t d = ra.y - P.n_rec;
            if ((A.cnt.post[d >> 5] >> (d & 31u)) & 1u) {
#pragma unroll
                for (uint32_t i = 0; i < 4; ++i) atomicOr(&fl[wl + i], v[i]);
            }
        } else if (sec == 3u) {
            const uint32_t o = ra.y - P.n_rec - P.n_det;
            const unsigned long long x = ((A.cnt.obs_exp[o >> 5] >> (o & 31u)) & 1u) ? ~0ull : 0ull;
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) atomicOr(&fl[TW + wl + i], v[i] ^ x);
        }
    }
    ((ulonglong2 *)&stg[vi * TW + wl])[0] = make_ulonglong2(v[0], v[1]);
    ((ulonglong2 *)&stg[vi * TW + wl])[1] = make_ulonglong2(v[2], v[3]);
    {
        // every lane of the node writes the same row index
        const uint32_t sec = (flags >> 4) & 3u;
        rows[vi] = (ra.y != FR_NO_ROW && sec && ((A.sections >> (sec - 1)) & 1u)) ? ra.y : FR_NO_ROW;
    }
    const uint32_t np = ra.w;
    if (np > 0) push_quad<TW>(slots, rb.x, wl, v);
    if (np > 1) push_quad<TW>(slots, rb.y, wl, v);
    for (uint32_t k = 2; k < np; ++k) push_quad<TW>(slots, P.fr_push[rb.z + k - 2], wl, v);
}

// One 32-byte chunk (node q / 4, words 4 (q % 4) .. + 3) of the rows staged
// by an EMIT step.
template <uint32_t TW>
__device__ __forceinline__ void store_chunk(const FrameArgs &A, const unsigned long long *stg, const uint32_t *rows,
                                            uint32_t q, uint64_t wt, bool full) {
    const uint32_t v = q / Tile<TW>::QPN, pw = 4 * (q % Tile<TW>::QPN);
    const uint32_t row = rows[v];
    const uint64_t wi = wt + pw;
    const ulonglong2 *src = (const ulonglong2 *)&stg[v * TW + pw];
    if (full) {
        // every word of the tile is whole and 16-byte stores are allowed
        if (row == FR_NO_ROW) return;
        ulonglong2 *dst = (ulonglong2 *)((unsigned long long *)A.out + (uint64_t)row * A.row_stride + wi);
        const ulonglong2 a = src[0], b = src[1];
        dst[0] = a;
        dst[1] = b;
        return;
    }
    if (row == FR_NO_ROW) return;
#pragma unroll
    for (uint32_t h = 0; h < 2; ++h) {
        const uint64_t wh = wi + 2 * h;
        if (wh >= A.n_words) return;
        const ulonglong2 val = src[h];
        const unsigned long long m0 = word_mask(wh, A.shots), m1 = word_mask(wh + 1, A.shots);
        unsigned long long *dst = (unsigned long long *)A.out + (uint64_t)row * A.row_stride + wh;
        if (A.store16 && wh + 1 < A.n_words) {
            *(ulonglong2 *)dst = make_ulonglong2(val.x & m0, val.y & m1);
        } else {
            dst[0] = val.x & m0;
            if (wh + 1 < A.n_words) dst[1] = val.y & m1;
        }
    }
}

// Workgroup: TW / 2 waves.  LDS: slots [NS][TW] u64 | stream states [TW][NC] |
// entry cursors and counts [TW][NC] | overflow flags [TW] | aggregate-count
// flags [2][TW] u64 (discarded, logical error) | one region used by
// phase G as walk positions [NWC][256] and by phase S as the staging buffer
// ([FR_LEVEL_MAX][TW] u64 + [FR_LEVEL_MAX] rows).
// Phase S orders each step so that nothing it waits for was issued in the
// same step: the rows staged by the previous EMIT step are stored first (one
// 32-byte chunk per thread), node records were fetched one EMIT step ahead
// and the first flip entries of a NOISE step right after the previous NOISE
// step; a step record (one scalar load) names what the next steps need.  (Vector loads and stores share one completion counter, so a load
// issued behind fresh stores would wait for them.)  Every slot is zero
// between tiles: each one that receives a contribution is read and cleared by
// the node that owns it, and every node is emitted.
template <uint32_t TW>
__global__ void __launch_bounds__(TW * 32) __attribute__((amdgpu_waves_per_eu(4))) frame_kernel(FrameArgs A) {
    constexpr uint32_t NWC = Tile<TW>::NWC, WPW = Tile<TW>::WPW, QPN = Tile<TW>::QPN, STG_WORDS = Tile<TW>::STG_WORDS;
    extern __shared__ __align__(16) unsigned char smem[];
    const DevProg &P = A.P;
    const uint32_t NC = P.n_cls, NS = P.fr_n_slots, n_steps = P.fr_n_steps;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    unsigned long long *slots = (unsigned long long *)smem;
    FrWord *wst = (FrWord *)(slots + (size_t)(NS + 1) * TW);
    uint32_t *cur = (uint32_t *)(wst + (size_t)TW * NC);
    uint32_t *cnt = cur + (size_t)TW * NC;
    uint32_t *ovf = cnt + (size_t)TW * NC;
    // offsets from smem itself keep the pointers in the LDS address space (an
    // integer round trip would turn every access into a flat one, which also
    // waits on vector-memory counters)
    unsigned long long *fl = (unsigned long long *)(smem + ((((unsigned char *)(ovf + TW) - smem) + 15) & ~(ptrdiff_t)15));
    unsigned char *region = (unsigned char *)(fl + 2 * TW);
    uint32_t *tmp = (uint32_t *)region + (size_t)wave * 256;
    unsigned long long *stg = (unsigned long long *)region;         // [STG_WORDS]
    uint32_t *rows = (uint32_t *)(stg + STG_WORDS);                  // [FR_LEVEL_MAX]
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    const uint64_t n_tiles = (A.n_words + TW - 1) / TW;
    uint64_t *scr = A.scratch + (size_t)blockIdx.x * (TW * A.word_entries + NWC * 128);
    uint32_t *gtmp = (uint32_t *)(scr + (size_t)TW * A.word_entries) + (size_t)wave * 256;  // fallback walks
    for (uint32_t i = tid; i < (NS + 1) * TW; i += NWC * 64) slots[i] = 0ull;
    if (tid < 2 * TW) fl[tid] = 0ull;
    unsigned long long n_disc = 0, n_logic = 0;  // aggregate counts of this workgroup (threads < TW)
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint64_t wt = tile * TW;
        const bool full = A.store16 && (wt + TW) * 64 <= A.shots;
        for (uint32_t i = tid; i < TW * NC; i += NWC * 64) {
            wst[i] = FrWord{0, 0, 0, 0};
            cur[i] = 0;
        }
        if (tid < TW) ovf[tid] = 0;
        __syncthreads();
        // phase G: every event of every (word, class) stream of the tile
        for (uint32_t wl = wave; wl < TW && wt + wl < A.n_words; wl += NWC) {
            const uint64_t w = A.word_begin + wt + wl;
            bool over = false;
            for (uint32_t c = 0; c < NC && !over; ++c) {
                const uint32_t coff = uniform(P.cls_off)[c], cend = (uniform(P.cls_off)[c + 1] - coff) * 64u;
                const GapFast F = load_fast(P.cls_fast, c);
                const uint32_t cap = A.cap_override ? A.cap_override : uniform(A.cap)[c];
                uint64_t *out =
                    scr + (size_t)wl * A.word_entries + (A.cap_override ? c * A.cap_override : uniform(A.cap_off)[c]);
                Walk st = {0, 0, 0};
                uint32_t n = 0;
                while (!walk<TW, true>(walk_tabs(P), F, P.cls_Q + (size_t)c * 4097, c, coff, (uint32_t)w, (uint32_t)(w >> 32), st,
                                   cend, tmp, out, cap, &n, nullptr, 0, k0, k1) &&
                       st.pos < cend && n <= cap) {
                }
                over = n > cap;
                if (lane == 0) cnt[wl * NC + c] = n;
            }
            if (lane == 0 && over) ovf[wl] = 1;
        }
        // each wave reads back only the entries it wrote (through other lanes); a
        // workgroup-scope fence orders them, all waves of a workgroup sharing one L1
        __threadfence_block();
        __syncthreads();
        // phase S
        const cptr<uint32_t> stp = uniform(P.fr_step);
        uint32_t pend_n = 0;
        uint4 pa = make_uint4(0, 0, 0, 0), pb = pa;
        uint64_t pe[WPW];
        uint32_t pk[WPW];
        auto fetch_records = [&](uint32_t first, uint32_t n) {
            if (tid < n * QPN) {
                const uint4 *rec = (const uint4 *)(P.fr_nodes + 8 * (size_t)(first + tid / QPN));
                pa = rec[0];
                pb = rec[1];
            }
        };
        auto fetch_entries = [&](uint32_t c) {
#pragma unroll
            for (uint32_t i = 0; i < WPW; ++i) {
                pe[i] = 0;
                pk[i] = FR_NONE;
            }
            if (c == FR_NONE) return;
            const uint32_t coff = A.cap_override ? c * A.cap_override : uniform(A.cap_off)[c];
#pragma unroll
            for (uint32_t i = 0; i < WPW; ++i) {
                const uint32_t wl = wave + i * NWC;
                if (wt + wl >= A.n_words || rfl(ovf[wl])) continue;
                const uint32_t k = rfl(cur[wl * NC + c]), kend = rfl(cnt[wl * NC + c]);
                pk[i] = k;
                if (k + lane < kend) pe[i] = scr[(size_t)wl * A.word_entries + coff + k + lane];
            }
        };
        fetch_records(P.fr_first_emit, P.fr_first_emit_n);
        fetch_entries(P.fr_first_noise_cls);
        auto noise_step = [&](cptr<uint32_t> r) {
            const uint32_t c = r[1], r1 = r[2], sl = r[3];
            const uint32_t coff = A.cap_override ? c * A.cap_override : uniform(A.cap_off)[c];
#pragma unroll
            for (uint32_t i = 0; i < WPW; ++i) {
                const uint32_t wl = wave + i * NWC;
                if (wt + wl >= A.n_words) continue;
                if (rfl(ovf[wl])) {
                    noise_direct<TW>(walk_tabs(P), load_fast(P.cls_fast, c), P.cls_Q + (size_t)c * 4097, c,
                                 uniform(P.cls_off)[c], r1 * 64u, A.word_begin + wt + wl, &wst[wl * NC + c], gtmp,
                                 slots, wl, k0, k1);
                    continue;
                }
                const uint64_t *src = scr + (size_t)wl * A.word_entries + coff;
                uint32_t k = rfl(cur[wl * NC + c]);
                const uint32_t kend = rfl(cnt[wl * NC + c]);
                bool first = pk[i] == k;
                while (k < kend) {
                    const uint32_t idx = k + lane;
                    const uint64_t e = first ? pe[i] : (idx < kend ? src[idx] : 0ull);
                    first = false;
                    const bool take = idx < kend && ((uint32_t)(e >> 8) & 0xFFu) == sl;
                    if (take) apply_entry<TW>(e, slots, wl);
                    const uint32_t nd = (uint32_t)__popcll(__ballot(take));
                    k += nd;
                    if (nd < 64) break;
                }
                if (lane == 0) cur[wl * NC + c] = k;
            }
            fetch_entries(r[7]);
        };
        for (uint32_t step = 0; step < n_steps; ++step) {
            const cptr<uint32_t> r = stp + (size_t)step * FR_STEP_WORDS;
            const bool is_emit = r[0] == FR_EMIT;
            // Take the data fetched for this step before issuing any store: a wait
            // on vector memory covers every operation issued before it, so a load
            // consumed behind fresh stores would wait for the stores as well.
            const uint4 ra = pa, rb = pb;
            if (is_emit) {
                asm volatile("" : : "v"(ra.x), "v"(ra.y), "v"(ra.z), "v"(ra.w), "v"(rb.x), "v"(rb.y), "v"(rb.z));
            } else {
#pragma unroll
                for (uint32_t i = 0; i < WPW; ++i) asm volatile("" : : "v"(pe[i]));
            }
            // rows staged by the previous step (if it was an EMIT step)
            if (tid < pend_n * QPN) store_chunk<TW>(A, stg, rows, tid, wt, full);
            pend_n = 0;
            if (is_emit) {
                const uint32_t n = r[2];
                fetch_records(r[5], r[6]);
                if (tid < n * QPN) emit_quad<TW>(P, A, ra, rb, tid, wt, slots, stg, rows, fl, k0, k1);
                pend_n = n;
            } else {
                noise_step(r);
            }
            __syncthreads();
        }
        if (tid < pend_n * QPN) store_chunk<TW>(A, stg, rows, tid, wt, full);
        __syncthreads();
        if (A.cnt.on && tid < TW) {
            // the tile's flags: kept shots only can have a logical error; bits past the shot count are 0
            const uint64_t wi = wt + tid;
            if (wi < A.n_words) {
                const unsigned long long m = word_mask(wi, A.shots);
                const unsigned long long d = fl[tid] & m, l = fl[TW + tid] & ~d & m;
                if (A.cnt.flags) {
                    A.cnt.flags[wi] = d;
                    A.cnt.flags[A.n_words + wi] = l;
                }
                n_disc += (unsigned long long)__popcll(d);
                n_logic += (unsigned long long)__popcll(l);
            }
            fl[tid] = 0ull;
            fl[TW + tid] = 0ull;
        }
    }
    if (A.cnt.on && A.cnt.counts && wave == 0) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            n_disc += __shfl_xor(n_disc, off, 64);
            n_logic += __shfl_xor(n_logic, off, 64);
        }
        if (lane == 0) {
            if (n_disc) atomicAdd(&A.cnt.counts[0], n_disc);
            if (n_logic) atomicAdd(&A.cnt.counts[1], n_logic);
        }
    }
}

// Gap decisions exactly as the walk takes them (fast margins, else the table).
__global__ void gap_check_kernel(GapFast F, const uint64_t *Q, const uint32_t *v, int32_t *g, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int G = 0;
    if (!gap_fast(F, v[i], G)) G = gap_of(Q, F.invlog2q, v[i]);
    g[i] = G;
}

template <uint32_t TW>
static size_t lds_bytes_of(const DevProg &P) {
    // slots | stream states | cursors and counts | overflow flags | count flags | (walk positions or staging)
    const size_t head = (size_t)(P.fr_n_slots + 1) * TW * 8 + (size_t)TW * P.n_cls * (sizeof(FrWord) + 8) + TW * 4;
    const size_t flags = 2 * TW * 8;
    const size_t region =
        std::max<size_t>((size_t)Tile<TW>::NWC * 256 * 4, Tile<TW>::STG_WORDS * 8 + FR_LEVEL_MAX * 4);
    return ((head + 15) & ~(size_t)15) + flags + region;
}

// Tile width tw is 16 or 32 in all of these.
size_t frame_lds_bytes(const DevProg &P, uint32_t tw) { return tw == 32 ? lds_bytes_of<32>(P) : lds_bytes_of<16>(P); }

// Scratch per workgroup, in u64: flip entries of the tile's words plus the fallback walks' positions.
size_t frame_scratch_words(uint32_t word_entries, uint32_t tw) { return (size_t)tw * word_entries + (tw / 2) * 128; }

uint32_t frame_threads(uint32_t tw) { return tw * 32; }

int frame_max_blocks_per_cu(size_t lds, uint32_t tw) {
    int nb = 0;
    const void *k = tw == 32 ? (const void *)frame_kernel<32> : (const void *)frame_kernel<16>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)frame_threads(tw), lds) != hipSuccess) return 1;
    return nb;
}

hipError_t launch_frame(const FrameArgs &A, uint32_t grid, hipStream_t st, uint32_t tw) {
    const void *k = tw == 32 ? (const void *)frame_kernel<32> : (const void *)frame_kernel<16>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)A.lds_bytes);
    if (e != hipSuccess) return e;
    if (tw == 32)
        hipLaunchKernelGGL(frame_kernel<32>, dim3(grid), dim3(frame_threads(32)), A.lds_bytes, st, A);
    else
        hipLaunchKernelGGL(frame_kernel<16>, dim3(grid), dim3(frame_threads(16)), A.lds_bytes, st, A);
    return hipGetLastError();
}

hipError_t launch_gap_check(const GapFast &F, const uint64_t *Q, const uint32_t *v, int32_t *g, uint64_t n,
                            hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(gap_check_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, F, Q, v, g, n);
    return hipGetLastError();
}

}  // namespace symft
