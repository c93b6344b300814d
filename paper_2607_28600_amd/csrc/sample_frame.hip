// sample_frame.hip -- pure-frame sampling (peak active width 0) for gfx950.
//
// A workgroup owns a tile of 16 consecutive 64-shot words.  One uint64 holds
// one row of one word's 64 shots, so a row of a tile is one aligned 128-byte
// line of the record-major output.  The workgroup runs the push-based
// schedule (launch_args.hpp) over its tile, with a barrier after every step:
//  * NOISE steps: the waves share out the tile's words; for each word a wave
//    applies the noise events of the step's channels, XOR-ing each event's
//    lane bit into the slots its (channel, branch) flips.  Events come from
//    the draw contract one walk at a time: 64 lanes x 4 gap draws decided
//    without the table except near a boundary, a 32-bit wave scan turning
//    gaps into positions, and one branch-draw Philox block per lane.  A walk's
//    events are kept in a per-(word, class) buffer of (flip index << 6 | lane)
//    entries until their step comes; a program with too many probability
//    classes for those buffers walks each step afresh and applies at once;
//  * EMIT levels: lanes take (node, pair of words): read and clear the node's
//    two slot words, add its constant or its RandomMeas words, store 16 bytes
//    of its output row and XOR the values into its successors' slots.
#include <hip/hip_runtime.h>

#include "launch_args.hpp"
#include "philox.hpp"

namespace symft {

constexpr uint32_t TW = 16;    // words per tile
constexpr uint32_t EVB = 256;  // event entries per buffer: one walk

struct FrWord {
    uint32_t pos, j, e;  // class stream: next position, next draw, next event index
    uint32_t bi, nb;     // buffered events [bi, nb) of the last walk
    uint32_t done;       // no events left in the stream
};

__device__ __forceinline__ uint32_t pick4(uint4 r, uint32_t i) {
    return i == 0 ? r.x : i == 1 ? r.y : i == 2 ? r.z : r.w;
}

__device__ __forceinline__ uint32_t branch_of(const DevProg &P, uint64_t info, uint32_t bv) {
    const uint32_t J = (uint32_t)(info >> 32) & 0xFFu;
    if ((info >> 40) & 1u) return (uint32_t)(((uint64_t)bv * J) >> 32);
    const uint64_t t0 = info >> 41;
    for (uint32_t t = 0; t < J; ++t)
        if ((uint64_t)bv < P.thr[t0 + t]) return t;
    return J - 1;
}

// XOR lane bit `ln` into every slot flipped by flip-table entry `fi`; `col`
// is the word's column of the slot array (slot s at col[s * TW]).
__device__ __forceinline__ void apply_flips(const DevProg &P, uint32_t fi, uint32_t ln, unsigned long long *col) {
    const uint64_t e = P.fr_fltab[fi];
    const uint32_t n = (uint32_t)(e & 0xFFu);
    const unsigned long long bit = 1ull << ln;
    if (n <= 2) {
        if (n > 0) atomicXor(&col[(size_t)((e >> 8) & 0xFFFFFFFu) * TW], bit);
        if (n > 1) atomicXor(&col[(size_t)(e >> 36) * TW], bit);
        return;
    }
    uint32_t off = (uint32_t)((e >> 8) & 0xFFFFFFFu), cnt = n;
    if (n == 255) cnt = P.fr_flslots[off++];
    for (uint32_t q = 0; q < cnt; ++q) atomicXor(&col[(size_t)P.fr_flslots[off + q] * TW], bit);
}

struct Walk {
    uint32_t pos, j, e;
};

// One walk of the stream (class c, word w): the 256 gap draws from st.j
// (aligned down to a Philox block), cut before the first event at a position
// >= R or with an index past the 64 branch blocks that start at st.e & ~3.
// Event st.e + k goes to buf[(st.e & 3) + k] as fi << 6 | lane (STORE) or is
// applied to the word's slot column.  Returns the event count; cutR reports a
// cut at R.  buf also holds the event positions between the two phases.
template <bool STORE>
__device__ uint32_t walk(const DevProg &P, const GapFast &F, const uint64_t *Q, uint32_t c, uint32_t coff, uint32_t wlo,
                         uint32_t whi, Walk &st, uint32_t R, uint32_t *buf, unsigned long long *col, uint32_t k0,
                         uint32_t k1, bool &cutR) {
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
    uint32_t x = mine;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    const uint32_t total = __shfl(x, 63, 64);
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
    if (cut_lane < 64) {
        n_pos = __shfl(cut_p, (int)cut_lane, 64);
        n_e = __shfl(cut_e, (int)cut_lane, 64);
        n_j = jal + 4 * cut_lane + (uint32_t)__shfl(cut_i, (int)cut_lane, 64);
        cutR = __shfl(cut_r, (int)cut_lane, 64) != 0;
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
                if (before && G[i] < 4096) buf[ee - eb] = pp + (uint32_t)G[i];
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
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        const uint32_t idx = 4 * lane + i, ev = eb + idx;
        if (ev >= st.e && ev < n_e) {
            const uint32_t at = buf[idx];
            const uint64_t info = P.fr_chinfo[coff + (at >> 6)];
            const uint32_t fi = (uint32_t)info + branch_of(P, info, pick4(bb, i));
            if (STORE) buf[idx] = (fi << 6) | (at & 63u);
            else apply_flips(P, fi, at & 63u, col);
        }
    }
    const uint32_t n = n_e - st.e;
    st.pos = n_pos;
    st.e = n_e;
    st.j = n_j;
    return n;
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Apply the word's buffered events of this step (flip index below `bound`),
// walking on whenever the buffer runs out.
__device__ void noise_buffered(const DevProg &P, const GapFast &F, const uint64_t *Q, uint32_t c, uint32_t coff,
                               uint32_t cend, uint32_t bound, uint64_t w, FrWord *S, uint32_t *buf,
                               unsigned long long *col, uint32_t k0, uint32_t k1) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t bi = rfl(S->bi), nb = rfl(S->nb), done = rfl(S->done);
    Walk st = {rfl(S->pos), rfl(S->j), rfl(S->e)};
    bool walked = false;
    while (true) {
        while (bi < nb) {
            const uint32_t idx = bi + lane;
            const uint32_t ev = idx < nb ? buf[idx] : 0u;
            const bool take = idx < nb && (ev >> 6) < bound;
            if (take) apply_flips(P, ev >> 6, ev & 63u, col);
            const uint32_t nd = (uint32_t)__popcll(__ballot(take));
            bi += nd;
            if (nd < 64) break;
        }
        if (bi < nb || done) break;  // the next buffered event belongs to a later step
        const uint32_t e0 = st.e;
        uint32_t n;
        bool cutR;
        do {
            n = walk<true>(P, F, Q, c, coff, (uint32_t)w, (uint32_t)(w >> 32), st, cend, buf, col, k0, k1, cutR);
        } while (n == 0 && !cutR && st.pos < cend);
        walked = true;
        if (n == 0) {
            done = 1;
            break;
        }
        bi = e0 & 3u;
        nb = bi + n;
    }
    if (lane == 0) {
        S->bi = bi;
        S->nb = nb;
        S->done = done;
        if (walked) {
            S->pos = st.pos;
            S->j = st.j;
            S->e = st.e;
        }
    }
}

// Walk the word's stream up to the end R of this step, applying events at once.
__device__ void noise_direct(const DevProg &P, const GapFast &F, const uint64_t *Q, uint32_t c, uint32_t coff,
                             uint32_t R, uint64_t w, FrWord *S, uint32_t *tmp, unsigned long long *col, uint32_t k0,
                             uint32_t k1) {
    Walk st = {rfl(S->pos), rfl(S->j), rfl(S->e)};
    if (st.pos >= R) return;
    bool cutR;
    do {
        walk<false>(P, F, Q, c, coff, (uint32_t)w, (uint32_t)(w >> 32), st, R, tmp, col, k0, k1, cutR);
    } while (!cutR && st.pos < R);
    if ((threadIdx.x & 63u) == 0) {
        S->pos = st.pos;
        S->j = st.j;
        S->e = st.e;
    }
}

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

// One EMIT level over the tile whose first word (within the call) is wt.
__device__ __forceinline__ void emit_level(const DevProg &P, const FrameArgs &A, uint32_t first, uint32_t n,
                                           uint64_t wt, unsigned long long *slots, uint32_t tid, uint32_t nthr,
                                           uint32_t k0, uint32_t k1) {
    for (uint32_t q = tid; q < n * (TW / 2); q += nthr) {
        const uint32_t v = first + q / (TW / 2), wl = 2 * (q % (TW / 2));
        const uint4 *rec = (const uint4 *)(P.fr_nodes + 8 * (size_t)v);
        const uint4 ra = rec[0], rb = rec[1];
        const uint32_t flags = ra.x >> 24;
        unsigned long long v0 = (flags & 1u) ? ~0ull : 0ull, v1 = v0;
        if (flags & 2u) {
            ulonglong2 *sp = (ulonglong2 *)&slots[(size_t)(ra.x & 0xFFFFFFu) * TW + wl];
            const ulonglong2 s = *sp;
            v0 ^= s.x;
            v1 ^= s.y;
            *sp = make_ulonglong2(0ull, 0ull);
        }
        const uint64_t wi = wt + wl;
        if (flags & 4u) {
            const uint64_t w = A.word_begin + wi;
            v0 ^= rm_word(ra.z, w, k0, k1);
            v1 ^= rm_word(ra.z, w + 1, k0, k1);
        }
        const uint32_t sec = (flags >> 4) & 3u;
        if (ra.y != FR_NO_ROW && sec && ((A.sections >> (sec - 1)) & 1u) && wi < A.n_words) {
            unsigned long long *dst = (unsigned long long *)A.out + (uint64_t)ra.y * A.row_stride + wi;
            const unsigned long long o0 = v0 & word_mask(wi, A.shots), o1 = v1 & word_mask(wi + 1, A.shots);
            if (A.store16 && wi + 1 < A.n_words) {
                *(ulonglong2 *)dst = make_ulonglong2(o0, o1);
            } else {
                dst[0] = o0;
                if (wi + 1 < A.n_words) dst[1] = o1;
            }
        }
        const uint32_t np = ra.w;
        if (np > 0) {
            unsigned long long *d = &slots[(size_t)rb.x * TW + wl];
            atomicXor(d, v0);
            atomicXor(d + 1, v1);
        }
        if (np > 1) {
            unsigned long long *d = &slots[(size_t)rb.y * TW + wl];
            atomicXor(d, v0);
            atomicXor(d + 1, v1);
        }
        for (uint32_t k = 2; k < np; ++k) {
            unsigned long long *d = &slots[(size_t)P.fr_push[rb.z + k - 2] * TW + wl];
            atomicXor(d, v0);
            atomicXor(d + 1, v1);
        }
    }
}

// LDS: slots [NS][TW] u64 | word states [TW][NC] | event buffers
// ([TW][NC][EVB] buffered, [NW][EVB] direct).  Every slot is zero between
// tiles: each one that receives a contribution is read and cleared by the
// node that owns it, and every node is emitted.
template <uint32_t NW>
__global__ void __launch_bounds__(NW * 64) frame_kernel(FrameArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const DevProg &P = A.P;
    const uint32_t NC = P.n_cls, NS = P.fr_n_slots;
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    unsigned long long *slots = (unsigned long long *)smem;
    FrWord *wst = (FrWord *)(slots + (size_t)NS * TW);
    uint32_t *evb = (uint32_t *)(wst + (size_t)TW * NC);
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    const uint64_t n_tiles = (A.n_words + TW - 1) / TW;
    for (uint32_t i = tid; i < NS * TW; i += NW * 64) slots[i] = 0ull;
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint64_t wt = tile * TW;
        for (uint32_t i = tid; i < TW * NC; i += NW * 64) wst[i] = FrWord{0, 0, 0, 0, 0, 0};
        __syncthreads();
        for (uint32_t step = 0; step < P.fr_n_steps; ++step) {
            const uint32_t code = P.fr_step[step];
            const uint32_t *d = P.fr_data + (code & 0x0FFFFFFFu);
            if ((code >> 28) == FR_NOISE) {
                const uint32_t c = d[0], r1 = d[2], bound = d[3];
                const uint32_t coff = P.cls_off[c];
                const uint32_t cend = (P.cls_off[c + 1] - coff) * 64u;
                const GapFast F = P.cls_fast[c];
                const uint64_t *Q = P.cls_Q + (size_t)c * 4097;
                for (uint32_t wl = wave; wl < TW && wt + wl < A.n_words; wl += NW) {
                    const uint64_t w = A.word_begin + wt + wl;
                    FrWord *S = &wst[wl * NC + c];
                    if (A.buffered)
                        noise_buffered(P, F, Q, c, coff, cend, bound, w, S, evb + ((size_t)wl * NC + c) * EVB,
                                       slots + wl, k0, k1);
                    else
                        noise_direct(P, F, Q, c, coff, r1 * 64u, w, S, evb + (size_t)wave * EVB, slots + wl, k0, k1);
                }
            } else {
                emit_level(P, A, d[0], d[1], wt, slots, tid, NW * 64, k0, k1);
            }
            __syncthreads();
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

size_t frame_lds_bytes(const DevProg &P, bool buffered, uint32_t nw) {
    return (size_t)P.fr_n_slots * TW * 8 + (size_t)TW * P.n_cls * sizeof(FrWord) +
           (buffered ? (size_t)TW * P.n_cls * EVB * 4 : (size_t)nw * EVB * 4) + 16;
}

int frame_max_blocks_per_cu(size_t lds, uint32_t nw) {
    int nb = 0;
    const void *f = nw == 8 ? (const void *)frame_kernel<8> : (const void *)frame_kernel<4>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, (int)nw * 64, lds) != hipSuccess) return 1;
    return nb;
}

hipError_t launch_frame(const FrameArgs &A, uint32_t grid, hipStream_t st) {
    const void *f = A.nwave == 8 ? (const void *)frame_kernel<8> : (const void *)frame_kernel<4>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)A.lds_bytes);
    if (e != hipSuccess) return e;
    if (A.nwave == 8)
        hipLaunchKernelGGL(frame_kernel<8>, dim3(grid), dim3(512), A.lds_bytes, st, A);
    else
        hipLaunchKernelGGL(frame_kernel<4>, dim3(grid), dim3(256), A.lds_bytes, st, A);
    return hipGetLastError();
}

hipError_t launch_gap_check(const GapFast &F, const uint64_t *Q, const uint32_t *v, int32_t *g, uint64_t n,
                            hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(gap_check_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, F, Q, v, g, n);
    return hipGetLastError();
}

}  // namespace symft
