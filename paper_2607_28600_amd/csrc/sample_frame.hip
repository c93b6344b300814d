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
//    into its pre-packed flip entries (shot lane, NOISE step, up to four
//    12-bit slots each; a branch's entries sit in one 32-byte flip record, so
//    a lane loads the records of its four events together), written in
//    stream order to the workgroup's scratch, which stays in L2 / the
//    Infinity Cache.  The slot region is free in this phase: when they fit,
//    it holds LDS copies of the walk's tables (32-bit gap table, compact
//    channel records, step bytes), which leaves the flip records as the
//    walk's only global loads, and is cleared again before phase S;
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
#include <type_traits>

#include "frame_device.hpp"
#include "launch_args.hpp"
#include "philox.hpp"

namespace symft {

// Tile shape, by tile width TW (16 or 32 words): TW / 2 waves, each walking
// two words in phase G and streaming two words' entries in NOISE steps; an
// EMIT step of up to FR_LEVEL_MAX nodes gives each thread two (node, 4 words)
// tasks, q and q + the thread count.
template <uint32_t TW>
struct Tile {
    static_assert(TW == 16 || TW == 32, "tile of 16 or 32 words");
    static constexpr uint32_t NWC = TW / 2;                    // waves
    static constexpr uint32_t NT = NWC * 64;                   // threads
    static constexpr uint32_t WPW = TW / NWC;                  // words per wave in NOISE steps
    static constexpr uint32_t QPN = TW / 4;                    // word quads per node
    static_assert(FR_LEVEL_MAX * QPN == 2 * NT, "two (node, 4 words) tasks per thread");
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

// Flip entry (lane | (k - 1) << 6 | step << 8 | k 12-bit slots from bit 16)
// applied to word wl of the tile.
template <uint32_t TW>
__device__ __forceinline__ void apply_entry(uint64_t e, unsigned long long *slots, uint32_t wl) {
    const unsigned long long bit = 1ull << (e & 63u);
    const uint32_t k = entry_slots(e);
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q)
        if (q < k) atomicXor(slot_word<TW>(slots, entry_slot(e, q), wl), bit);
}

// XOR v[0 .. 3] into words wl .. wl + 3 of slot s.
template <uint32_t TW>
__device__ __forceinline__ void push_quad(unsigned long long *slots, uint32_t s, uint32_t wl, const unsigned long long *v) {
    unsigned long long *d = slot_quad<TW>(slots, s, wl);
    const uint32_t x = s & 3u;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) atomicXor(d + (i ^ x), v[i]);
}

// Walk the word's class stream up to the end R of this step, applying events at once.
template <uint32_t TW>
__device__ __forceinline__ void noise_direct(const DevProg &P, uint32_t c, uint32_t R, uint64_t w, FrWord *S,
                                             uint32_t *tmp, unsigned long long *slots, uint32_t wl, uint32_t k0,
                                             uint32_t k1) {
    Walk st = {rfl(S->pos), rfl(S->j), rfl(S->e)};
    if (st.pos >= R) return;
    const GapFast F = load_fast(P.cls_fast, c);
    const uint32_t coff = uniform(P.cls_off)[c];
    auto flip = [slots, wl](uint64_t e) { apply_entry<TW>(e, slots, wl); };
    uint32_t none = 0;
    const WalkLds T = {nullptr, nullptr, nullptr};
    while (!walk_entries<false, false>(P, T, F, c, coff, w, st, R, tmp, nullptr, 0, none, k0, k1, flip) && st.pos < R) {
    }
    if ((threadIdx.x & 63u) == 0) {
        S->pos = st.pos;
        S->j = st.j;
        S->e = st.e;
    }
}

// One (node, 4 words) task of an EMIT step: the four slot words are read and
// cleared, the node's constant and RandomMeas words added, the 32 bytes of its
// row stored (the node's QPN tasks are adjacent threads, so a row of the tile
// goes out as whole lines) and the values XOR-ed into the successors' slots.
template <uint32_t TW>
__device__ __forceinline__ void emit_quad(const DevProg &P, const FrameArgs &A, uint4 ra, uint32_t q,
                                          uint64_t wt, bool full, unsigned long long *slots, unsigned long long *fl,
                                          uint32_t k0, uint32_t k1) {
    const uint32_t wl = 4 * (q % Tile<TW>::QPN);
    const uint32_t flags = (ra.x >> 12) & 0xFFu;
    const unsigned long long c = (flags & 1u) ? ~0ull : 0ull;
    unsigned long long v[4] = {c, c, c, c};
    {
        // a node with no contributions reads the extra slot past the schedule's, which stays zero
        const uint32_t sl = ra.x & 0xFFFu, x = sl & 3u;
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
        const uint32_t rm_t = P.fr_push16[ra.w];
#pragma unroll 1
        for (uint32_t i = 0; i < 4; ++i) {
            const unsigned long long t = v[0] ^ rm_word(rm_t, w + i, k0, k1);
            v[0] = v[1];
            v[1] = v[2];
            v[2] = v[3];
            v[3] = t;
        }
    }
    const uint32_t sec = (flags >> 4) & 3u;
    if (A.cnt.on) {
        // aggregate counts: a postselected detector ORs into the discarded
        // flags, an observable (XOR its expected value) into the logical ones
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
    } else if (ra.y != FR_NO_ROW && sec && ((A.sections >> (sec - 1)) & 1u)) {
        const uint64_t wi = wt + wl;
        unsigned long long *dst = (unsigned long long *)A.out + (uint64_t)ra.y * A.row_stride + wi;
        if (full) {
            // every word of the tile is whole and 16-byte stores are allowed; the rows are not read again,
            // so they are stored non-temporally and leave the L2 to the flip records and entries (C2: 5.48
            // against 5.61 ms)
            typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
            __builtin_nontemporal_store((u64x2){v[0], v[1]}, (u64x2 *)dst);
            __builtin_nontemporal_store((u64x2){v[2], v[3]}, (u64x2 *)dst + 1);
        } else {
#pragma unroll
            for (uint32_t h = 0; h < 2; ++h) {
                const uint64_t wh = wi + 2 * h;
                if (wh < A.n_words) {
                    const unsigned long long m0 = word_mask(wh, A.shots), m1 = word_mask(wh + 1, A.shots);
                    unsigned long long *d = dst + 2 * h;
                    if (A.store16 && wh + 1 < A.n_words) {
                        *(ulonglong2 *)d = make_ulonglong2(v[2 * h] & m0, v[2 * h + 1] & m1);
                    } else {
                        d[0] = v[2 * h] & m0;
                        if (wh + 1 < A.n_words) d[1] = v[2 * h + 1] & m1;
                    }
                }
            }
        }
    }
    const uint32_t np = ra.x >> 20;
    if (np > 0) push_quad<TW>(slots, ra.z & 0xFFFu, wl, v);
    if (np > 1) push_quad<TW>(slots, (ra.z >> 12) & 0xFFFu, wl, v);
    const uint32_t lb = ra.w + ((flags >> 2) & 1u);  // past a RandomMeas node's measurement
    for (uint32_t k = 2; k < np; ++k) push_quad<TW>(slots, P.fr_push16[lb + k - 2], wl, v);
}

// Phase G of one tile: each wave walks the streams of its words, class by
// class, into the workgroup's scratch; a stream past its capacity marks its
// word for the fallback.  LT: the walk tables are in LDS (T).
template <uint32_t TW, bool LT>
__device__ __forceinline__ void phase_g(const DevProg &P, const FrameArgs &A, const WalkLds &T, uint64_t wt,
                                        uint64_t *scr, uint32_t *tmp, uint32_t *cnt, uint32_t *ovf, uint32_t k0,
                                        uint32_t k1) {
    constexpr uint32_t NWC = Tile<TW>::NWC;
    const uint32_t NC = P.n_cls, wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    for (uint32_t wl = wave; wl < TW && wt + wl < A.n_words; wl += NWC) {
        const uint64_t w = A.word_begin + wt + wl;
        bool over = false;
        for (uint32_t c = 0; c < NC && !over; ++c) {
            const uint32_t coff = uniform(P.cls_off)[c], cend = (uniform(P.cls_off)[c + 1] - coff) * 64u;
            const GapFast F = load_fast(P.cls_fast, c);
            const uint32_t cap = A.cap_override ? A.cap_override : uniform(P.fr_cap)[c];
            uint64_t *out =
                scr + (size_t)wl * A.word_entries + (A.cap_override ? c * A.cap_override : uniform(P.fr_capoff)[c]);
            Walk st = {0, 0, 0};
            uint32_t n = 0;
            auto none = [](uint64_t) {};
            while (!walk_entries<true, LT>(P, T, F, c, coff, w, st, cend, tmp, out, cap, n, k0, k1, none) &&
                   st.pos < cend && n <= cap) {
            }
            over = n > cap;
            if (lane == 0) cnt[wl * NC + c] = n;
        }
        if (lane == 0 && over) ovf[wl] = 1;
    }
}

// Workgroup: TW / 2 waves.  LDS: slots [NS][TW] u64 | stream states [TW][NC] |
// entry cursors and counts [TW][NC] | overflow flags [TW] | aggregate-count
// flags [2][TW] u64 (discarded, logical error) | walk positions [NWC][256].
// Phase S fetches each step's data before the stores of the step before it
// are issued: node records one EMIT step ahead (both tasks of a thread), the
// first flip entries of a NOISE step right after the previous NOISE step; a
// step record (scalar loads) names what the next steps need.  (Vector loads
// and stores share one completion counter, so a load issued behind fresh
// stores would wait for them.)  Every slot is zero between tiles: each one
// that receives a contribution is read and cleared by the node that owns it,
// and every node is emitted.
template <uint32_t TW>
__global__ void __launch_bounds__(TW * 32) __attribute__((amdgpu_waves_per_eu(4))) frame_kernel(FrameArgs A) {
    constexpr uint32_t NWC = Tile<TW>::NWC, NT = Tile<TW>::NT, WPW = Tile<TW>::WPW, QPN = Tile<TW>::QPN;
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
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    const uint64_t n_tiles = (A.n_words + TW - 1) / TW;
    uint64_t *scr = A.scratch + (size_t)blockIdx.x * (TW * A.word_entries + NWC * 128);
    uint32_t *gtmp = (uint32_t *)(scr + (size_t)TW * A.word_entries) + (size_t)wave * 256;  // fallback walks
    // LDS copies of the walk tables (channel records, step bytes, 32-bit gap tables), in 16-byte units
    // (the device program pads each array to 16 bytes), when they fit the slot region
    const uint32_t lt_ci16 = P.fr_n_cch / 4, lt_st16 = P.fr_n_cch / 16, lt_q16 = (NC * 4097 + 3) / 4;
    const bool ltab = P.fr_ltab && (size_t)(lt_ci16 + lt_q16 + lt_st16) * 16 <= (size_t)(NS + 1) * TW * 8;
    const WalkLds LT = {(const uint32_t *)slots, (const uint8_t *)(slots + 2 * (size_t)(lt_ci16 + lt_q16)),
                        (const uint32_t *)(slots + 2 * (size_t)lt_ci16)};
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
        if (ltab) {
            // the walk tables into the slot region, which phase S needs only from the next barrier on
            uint4 *d = (uint4 *)slots;
            for (uint32_t i = tid; i < lt_ci16; i += NT) d[i] = ((const uint4 *)P.fr_ci32)[i];
            for (uint32_t i = tid; i < lt_q16; i += NT) d[lt_ci16 + i] = ((const uint4 *)P.cls_Q32)[i];
            for (uint32_t i = tid; i < lt_st16; i += NT) d[lt_ci16 + lt_q16 + i] = ((const uint4 *)P.fr_st8)[i];
            __syncthreads();
            phase_g<TW, true>(P, A, LT, wt, scr, tmp, cnt, ovf, k0, k1);
        } else {
            phase_g<TW, false>(P, A, LT, wt, scr, tmp, cnt, ovf, k0, k1);
        }
        // each wave reads back only the entries it wrote (through other lanes); a
        // workgroup-scope fence orders them, all waves of a workgroup sharing one L1
        __threadfence_block();
        const bool any_ovf = __syncthreads_or(tid < TW && ovf[tid]) != 0;
        if (ltab) {
            // the slot region back to zero
            uint4 *d = (uint4 *)slots;
            for (uint32_t i = tid; i < lt_ci16 + lt_q16 + lt_st16; i += NT) d[i] = make_uint4(0, 0, 0, 0);
            __syncthreads();
        }
        // phase S
        const cptr<uint32_t> stp = uniform(P.fr_step);
        uint4 pa = make_uint4(0, 0, 0, 0), pa2 = pa;
        uint64_t pe[WPW];
        uint32_t pk[WPW];
        auto fetch_records = [&](uint32_t first, uint32_t n) {
            if (tid < n * QPN) pa = ((const uint4 *)P.fr_nodes16)[first + tid / QPN];
            if (tid + NT < n * QPN) pa2 = ((const uint4 *)P.fr_nodes16)[first + (tid + NT) / QPN];
        };
        auto fetch_entries = [&](uint32_t c) {
#pragma unroll
            for (uint32_t i = 0; i < WPW; ++i) {
                pe[i] = 0ull;
                pk[i] = FR_NONE;
            }
            if (c == FR_NONE) return;
            const uint32_t coff = A.cap_override ? c * A.cap_override : uniform(P.fr_capoff)[c];
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
        // SLOW: some word of the tile overflowed its capacity and walks afresh at each NOISE step (a copy
        // of the step loop of its own, so that the common loop carries none of that walk's registers)
        auto noise_step = [&](cptr<uint32_t> r, auto slow) {
            const uint32_t c = r[1], r1 = r[2], sl = r[3];
            const uint32_t coff = A.cap_override ? c * A.cap_override : uniform(P.fr_capoff)[c];
#pragma unroll
            for (uint32_t i = 0; i < WPW; ++i) {
                const uint32_t wl = wave + i * NWC;
                if (wt + wl >= A.n_words) continue;
                if (decltype(slow)::value && rfl(ovf[wl])) {
                    noise_direct<TW>(P, c, r1 * 64u, A.word_begin + wt + wl, &wst[wl * NC + c], gtmp, slots, wl, k0, k1);
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
        auto run_steps = [&](auto slow) {
        for (uint32_t step = 0; step < n_steps; ++step) {
            const cptr<uint32_t> r = stp + (size_t)step * FR_STEP_WORDS;
            const bool is_emit = r[0] == FR_EMIT;
            // Take the data fetched for this step before issuing any store: a wait
            // on vector memory covers every operation issued before it, so a load
            // consumed behind fresh stores would wait for the stores as well.
            const uint4 ra = pa, ra2 = pa2;
            if (is_emit) {
                const uint32_t n = r[2];
                fetch_records(r[5], r[6]);
                if (tid < n * QPN) emit_quad<TW>(P, A, ra, tid, wt, full, slots, fl, k0, k1);
                if (tid + NT < n * QPN) emit_quad<TW>(P, A, ra2, tid + NT, wt, full, slots, fl, k0, k1);
            } else {
#pragma unroll
                for (uint32_t i = 0; i < WPW; ++i) asm volatile("" : : "v"(pe[i]));
                noise_step(r, slow);
            }
            __syncthreads();
        }
        };
        if (any_ovf)
            run_steps(std::true_type());
        else
            run_steps(std::false_type());
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

// Gap decisions exactly as the walks take them (fast margins, else the three-read window, else the table).
__global__ void gap_check_kernel(GapFast F, const uint64_t *Q, const uint32_t *v, int32_t *g, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int G = 0;
    if (!gap_fast_lean(F, v[i], G)) G = v[i] >= F.vwin ? gap_window(Q, v[i], G) : gap_of(Q, F.invlog2q, v[i]);
    g[i] = G;
}

template <uint32_t TW>
static size_t lds_bytes_of(const DevProg &P) {
    if (!P.fr_rec_ok) return SIZE_MAX;  // slots past the entries' 12 bits: the kernel cannot run the schedule
    // slots | stream states | cursors and counts | overflow flags | count flags | walk positions
    const size_t head = (size_t)(P.fr_n_slots + 1) * TW * 8 + (size_t)TW * P.n_cls * (sizeof(FrWord) + 8) + TW * 4;
    const size_t flags = 2 * TW * 8;
    const size_t region = (size_t)Tile<TW>::NWC * 256 * 4;
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
