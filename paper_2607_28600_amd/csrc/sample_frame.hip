// sample_frame.hip -- pure-frame sampling (peak active width 0) for gfx950.
//
// One wave (64 threads) owns a few consecutive 64-shot words at a time; one
// uint64 holds one row of a word's 64 shots.  The wave runs the push-based
// schedule (see launch_args.hpp) over its words:
//  * NOISE steps apply the word's noise events in stream order, 64 per
//    instruction: each event XORs its lane bit into the slots its
//    (channel, branch) flips (one 64-bit table entry with up to two slots
//    inline).  Events are drawn lazily, one step of the stream (64 lanes x 4
//    draws) at a time, under the draw contract: gaps from a log2 guess settled
//    on the exact integer table, a 64-lane shuffle scan turning gaps into
//    positions, then the branch draw; a batch is kept in LDS as
//    (flip-table index) << 6 | lane until the steps that own it are reached;
//  * EMIT levels run (node, word) pairs across the lanes: read and clear the
//    node's slot, add its constant or its RandomMeas word, store the row word
//    and XOR the value into the successor slots.
// Words are dealt so that consecutive words run on the same XCD, letting each
// L2 assemble whole 128-byte lines of every output row.
#include <hip/hip_runtime.h>

#include "launch_args.hpp"
#include "philox.hpp"

namespace symft {

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

// XOR lane bit `ln` into every slot flipped by flip-table entry `fi`.
__device__ __forceinline__ void apply_flips(const DevProg &P, uint32_t fi, uint32_t ln, unsigned long long *slots,
                                            uint32_t W, uint32_t wl) {
    const uint64_t e = P.fr_fltab[fi];
    const uint32_t n = (uint32_t)(e & 0xFFu);
    const unsigned long long bit = 1ull << ln;
    if (n <= 2) {
        if (n > 0) atomicXor(&slots[(size_t)((e >> 8) & 0xFFFFFFFu) * W + wl], bit);
        if (n > 1) atomicXor(&slots[(size_t)(e >> 36) * W + wl], bit);
        return;
    }
    uint32_t off = (uint32_t)((e >> 8) & 0xFFFFFFFu), cnt = n;
    if (n == 255) cnt = P.fr_flslots[off++];
    for (uint32_t q = 0; q < cnt; ++q) atomicXor(&slots[(size_t)P.fr_flslots[off + q] * W + wl], bit);
}

struct WalkState {
    uint64_t pos;
    uint32_t j, e;
};

// One wave walks the event stream of (class c, word w) from `st` until the
// first event at position >= R (which stays for the next call) or the end.
// STORE: append events to buf (returns false, without consuming the step,
// when the next 256 draws would overflow `cap`); otherwise apply them.
template <bool STORE>
__device__ bool wave_walk(const DevProg &P, uint32_t c, uint64_t w, uint64_t R, WalkState &st, uint32_t *buf,
                          uint32_t &nbuf, uint32_t cap, unsigned long long *slots, uint32_t W, uint32_t wl,
                          uint32_t k0, uint32_t k1) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t *Q = P.cls_Q + (size_t)c * 4097;
    const float il = P.cls_invlog2q[c];
    const uint32_t coff = P.cls_off[c];
    const uint32_t wlo = (uint32_t)w, whi = (uint32_t)(w >> 32);
    while (st.pos < R) {
        const uint32_t jal = st.j & ~3u;
        const uint4 rr = philox4x32_10(make_uint4((jal >> 2) + lane, wlo, c, (1u << 24) | whi), k0, k1);
        int G[4];
        uint32_t tinc = 0, tev = 0;
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            if (jal + 4 * lane + i >= st.j) {
                G[i] = gap_of(Q, il, pick4(rr, i));
                tinc += G[i] == 4096 ? 4096u : (uint32_t)G[i] + 1u;
                tev += G[i] < 4096 ? 1u : 0u;
            } else {
                G[i] = -1;
            }
        }
        const uint64_t mine = ((uint64_t)tev << 40) | tinc;
        uint64_t x = mine;
#pragma unroll
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint64_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        const uint64_t total = __shfl(x, 63, 64);
        const uint64_t ex = x - mine;
        const uint64_t p = st.pos + (ex & ((1ull << 40) - 1));
        const uint32_t ee = st.e + (uint32_t)(ex >> 40);
        int cut_i = 4;
        uint64_t cut_p = 0;
        uint32_t cut_e = 0;
        {
            uint64_t pp = p;
            uint32_t e2 = ee;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (G[i] >= 0) {
                    if (G[i] < 4096 && pp + (uint64_t)G[i] >= R && cut_i == 4) {
                        cut_i = i;
                        cut_p = pp;
                        cut_e = e2;
                    }
                    if (G[i] < 4096) ++e2;
                    pp += G[i] == 4096 ? 4096u : (uint32_t)G[i] + 1u;
                }
            }
        }
        const uint64_t bal = __ballot(cut_i < 4);
        const uint32_t cut_lane = bal ? (uint32_t)(__ffsll((long long)bal) - 1) : 64u;
        uint64_t new_pos;
        uint32_t new_e, new_j;
        if (cut_lane < 64) {
            new_pos = __shfl(cut_p, (int)cut_lane, 64);
            new_e = __shfl(cut_e, (int)cut_lane, 64);
            new_j = jal + 4 * cut_lane + (uint32_t)__shfl(cut_i, (int)cut_lane, 64);
        } else {
            new_pos = st.pos + (total & ((1ull << 40) - 1));
            new_e = st.e + (uint32_t)(total >> 40);
            new_j = jal + 256;
        }
        const uint32_t n_new = new_e - st.e;
        if (STORE && nbuf + n_new > cap) return false;
        uint4 bb = make_uint4(0, 0, 0, 0);
        uint32_t bblk = 0xFFFFFFFFu;
        {
            uint64_t pp = p;
            uint32_t e2 = ee;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (G[i] >= 0) {
                    const bool before = lane < cut_lane || (lane == cut_lane && i < cut_i);
                    if (before && G[i] < 4096) {
                        const uint64_t at = pp + (uint64_t)G[i];
                        const uint32_t rank = (uint32_t)(at >> 6), ln = (uint32_t)(at & 63);
                        const uint64_t info = P.fr_chinfo[coff + rank];
                        if ((e2 >> 2) != bblk) {
                            bblk = e2 >> 2;
                            bb = philox4x32_10(make_uint4(bblk, wlo, c, (2u << 24) | whi), k0, k1);
                        }
                        const uint32_t fi = (uint32_t)info + branch_of(P, info, pick4(bb, e2 & 3));
                        if (STORE) buf[nbuf + (e2 - st.e)] = (fi << 6) | ln;
                        else apply_flips(P, fi, ln, slots, W, wl);
                    }
                    if (G[i] < 4096) ++e2;
                    pp += G[i] == 4096 ? 4096u : (uint32_t)G[i] + 1u;
                }
            }
        }
        nbuf += n_new;
        st.pos = new_pos;
        st.e = new_e;
        st.j = new_j;
        if (cut_lane < 64) break;
    }
    return true;
}

// One wave owns WPW (1, 2 or 4) consecutive 64-shot words from their first
// draw to their last row, with private LDS (slots and a batch of drawn events
// per word), so waves never wait for each other.  A wave's LDS operations
// complete in issue order, which orders every push, flip and slot read.
// Emission maps lanes to (node, word) with the word fastest, so each row is
// stored as one contiguous 8*WPW-byte segment.
#define EVB 256u  // events kept per word: one draw step's worth

struct WordState {
    uint64_t pos;
    uint32_t j, e, nb, bi;  // stream state; buffered events [bi, nb) of the current batch
};

__global__ void __launch_bounds__(64) frame_kernel(FrameArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const DevProg &P = A.P;
    const uint32_t NC = P.n_cls, WPW = A.wpb, NS = P.fr_n_slots;
    const uint32_t lane = threadIdx.x;
    unsigned long long *slots = (unsigned long long *)smem;                // [WPW][NS]
    WordState *ws = (WordState *)(slots + (size_t)WPW * NS);               // [WPW][NC]
    uint32_t *evbuf = (uint32_t *)(ws + (size_t)WPW * NC);                 // [WPW][EVB]
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint64_t n_groups = (A.n_words + WPW - 1) / WPW;
    // consecutive word groups on the same XCD (blocks are dealt to the 8 XCDs in turn)
    const uint64_t first_group = (G % 8 == 0) ? (uint64_t)(b % 8) * (G / 8) + b / 8 : b;
    const uint32_t my_w = lane % WPW, my_v = lane / WPW, nv = 64u / WPW;

    for (uint64_t grp = first_group; grp < n_groups; grp += G) {
        const uint64_t wi0 = grp * WPW;
        for (uint32_t i = lane; i < WPW * NS; i += 64) slots[i] = 0;
        for (uint32_t i = lane; i < WPW * NC; i += 64) ws[i] = WordState{0, 0, 0, 0, 0};
        for (uint32_t step = 0; step < P.fr_n_steps; ++step) {
            const uint32_t code = P.fr_step[step];
            const uint32_t *d = P.fr_data + (code & 0x0FFFFFFFu);
            if ((code >> 28) == FR_NOISE) {
                const uint32_t c = d[0], bound = d[3];
                const uint64_t end = (uint64_t)(P.cls_off[c + 1] - P.cls_off[c]) * 64;
                for (uint32_t wl = 0; wl < WPW; ++wl) {
                    const uint64_t w = A.word_begin + wi0 + wl;
                    WordState &S = ws[wl * NC + c];
                    unsigned long long *sl = slots + (size_t)wl * NS;
                    uint32_t *eb = evbuf + (size_t)wl * EVB;
                    uint32_t k = S.bi, kend = S.nb;
                    while (true) {
                        // apply buffered events of this step, 64 per instruction
                        bool more = false;
                        while (k < kend) {
                            const uint32_t idx = k + lane;
                            const uint32_t ev = idx < kend ? eb[idx] : 0xFFFFFFFFu;
                            const bool mine = idx < kend && (ev >> 6) < bound;
                            if (mine) apply_flips(P, ev >> 6, ev & 63u, sl, 1, 0);
                            const uint32_t nd = (uint32_t)__popcll(__ballot(mine));
                            k += nd;
                            if (nd < 64) {
                                more = k < kend;
                                break;
                            }
                        }
                        if (more) break;  // the next buffered event belongs to a later step
                        WalkState st = {S.pos, S.j, S.e};
                        if (st.pos >= end) break;  // stream finished
                        uint32_t nb = 0;
                        wave_walk<true>(P, c, w, end, st, eb, nb, EVB, sl, 1, 0, k0, k1);
                        // a walk stops early only to keep events it already holds, so a
                        // walk that holds none has reached the end of the stream
                        if (nb == 0) st.pos = end;
                        if (lane == 0) {
                            S.pos = st.pos;
                            S.j = st.j;
                            S.e = st.e;
                        }
                        k = 0;
                        kend = nb;
                    }
                    if (lane == 0) {
                        S.bi = k;
                        S.nb = kend;
                    }
                }
            } else {
                const uint32_t first = d[0], n = d[1];
                const uint64_t wi = wi0 + my_w;  // word index within the call
                const uint64_t w = A.word_begin + wi;
                const uint64_t lanes = (wi * 64 + 64 <= A.shots) ? ~0ull
                                       : (wi * 64 >= A.shots ? 0ull : ((1ull << (A.shots - wi * 64)) - 1ull));
                unsigned long long *sl = slots + (size_t)my_w * NS;
                for (uint32_t v = my_v; v < n; v += nv) {
                    const uint4 *rec = (const uint4 *)(P.fr_nodes + 8 * (size_t)(first + v));
                    const uint4 ra = rec[0], rb = rec[1];
                    const uint32_t flags = ra.x >> 24;
                    unsigned long long val = (flags & 1u) ? ~0ull : 0ull;
                    if (flags & 2u) {
                        unsigned long long *sp = &sl[ra.x & 0xFFFFFFu];
                        val ^= *sp;
                        *sp = 0;
                    }
                    if (flags & 4u) {
                        const uint32_t t = ra.z;
                        const uint4 o = philox4x32_10(make_uint4(t >> 1, (uint32_t)w, 0u, (3u << 24) | (uint32_t)(w >> 32)), k0, k1);
                        val ^= (t & 1) ? ((uint64_t)o.z | ((uint64_t)o.w << 32)) : ((uint64_t)o.x | ((uint64_t)o.y << 32));
                    }
                    const uint32_t sec = (flags >> 4) & 3u;
                    if (ra.y != FR_NO_ROW && sec && ((A.sections >> (sec - 1)) & 1u) && wi < A.n_words)
                        A.out[(uint64_t)ra.y * A.row_stride + wi] = val & lanes;
                    const uint32_t np = ra.w;
                    if (np > 0) atomicXor(&sl[rb.x], val);
                    if (np > 1) atomicXor(&sl[rb.y], val);
                    for (uint32_t q = 2; q < np; ++q) atomicXor(&sl[P.fr_push[rb.z + q - 2]], val);
                }
            }
        }
    }
}

size_t frame_lds_bytes(const DevProg &P, uint32_t wpb) {
    return (size_t)wpb * ((size_t)P.fr_n_slots * 8 + (size_t)P.n_cls * sizeof(WordState) + EVB * 4) + 16;
}

int frame_max_blocks_per_cu(size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, frame_kernel, 64, lds) != hipSuccess) return 1;
    return nb;
}

hipError_t launch_frame(const FrameArgs &A, uint32_t grid, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)frame_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)A.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(frame_kernel, dim3(grid), dim3(64), A.lds_bytes, st, A);
    return hipGetLastError();
}

}  // namespace symft
