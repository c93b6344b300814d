// sample_frame.hip -- pure-frame sampling (peak active width 0) for gfx950.
//
// A workgroup of 256 threads owns a tile of W consecutive 64-shot words and
// runs the push-based schedule (see launch_args.hpp) over it.  Everything is
// bit-sliced: one uint64 holds one row of 64 shots.
//  * NOISE steps: the TPW = 256/W threads of a word walk that word's
//    geometric event stream for one probability class cooperatively: each
//    thread takes one Philox block (4 draws), a TPW-wide shuffle scan turns
//    gaps into positions, events up to the step's last rank are applied (LDS
//    atomic XOR of the event's lane bit into every consumer slot) and the
//    stream stops at the first event that belongs to a later step, which is
//    drawn again there.
//  * EMIT steps: W consecutive lanes handle the W words of one node, so the
//    output row segment of the tile (8W bytes) is written by one coalesced
//    store; pushes go to successor slots with LDS atomic XOR.
#include <hip/hip_runtime.h>

#include "launch_args.hpp"
#include "philox.hpp"

namespace symft {

__device__ __forceinline__ int gap_search_f(const uint64_t *__restrict__ Q, uint32_t v) {
    if ((uint64_t)v < Q[4096]) return 4096;
    int lo = 0, hi = 4096;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if ((uint64_t)v < Q[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t pick4(uint4 r, uint32_t i) {
    return i == 0 ? r.x : i == 1 ? r.y : i == 2 ? r.z : r.w;
}

__global__ void __launch_bounds__(256) frame_kernel(FrameArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const DevProg &P = A.P;
    const uint32_t W = A.wpb, TPW = 256u / W;
    unsigned long long *slots = (unsigned long long *)smem;
    uint64_t *st_pos = (uint64_t *)(slots + (size_t)P.fr_n_slots * W);
    uint32_t *st_j = (uint32_t *)(st_pos + (size_t)P.n_cls * W);
    uint32_t *st_e = st_j + (size_t)P.n_cls * W;
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    const uint32_t nlw = threadIdx.x / TPW, sub = threadIdx.x % TPW;    // noise mapping
    const uint32_t elw = threadIdx.x % W, enode = threadIdx.x / W;     // emit mapping
    const uint32_t lane64 = threadIdx.x & 63;
    const uint32_t gbase = (lane64 / TPW) * TPW;                         // first lane of my word group
    const uint64_t n_tiles = (A.n_words + W - 1) / W;

    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        for (uint32_t i = threadIdx.x; i < P.fr_n_slots * W; i += 256) slots[i] = 0;
        for (uint32_t i = threadIdx.x; i < P.n_cls * W; i += 256) { st_pos[i] = 0; st_j[i] = 0; st_e[i] = 0; }
        __syncthreads();
        for (uint32_t step = 0; step < P.fr_n_steps; ++step) {
            const uint32_t code = P.fr_step[step];
            const uint32_t kind = code >> 28;
            const uint32_t *d = P.fr_data + (code & 0x0FFFFFFFu);
            if (kind == FR_NOISE) {
                const uint32_t c = d[0];
                const uint64_t R = (uint64_t)d[2] * 64;
                const uint64_t *Q = P.cls_Q + (size_t)c * 4097;
                const uint32_t coff = P.cls_off[c];
                const uint64_t w = A.word_begin + tile * W + nlw;
                const uint32_t wlo = (uint32_t)w, whi = (uint32_t)(w >> 32);
                uint64_t pos = st_pos[c * W + nlw];
                uint32_t j = st_j[c * W + nlw], e = st_e[c * W + nlw];
                bool done = pos >= R;
                while (!done) {
                    const uint32_t jal = j & ~3u;
                    const uint4 rr = philox4x32_10(make_uint4((jal >> 2) + sub, wlo, c, (1u << 24) | whi), k0, k1);
                    int G[4];
                    uint32_t tinc = 0, tev = 0;
#pragma unroll
                    for (uint32_t i = 0; i < 4; ++i) {
                        const uint32_t dj = jal + 4 * sub + i;
                        if (dj >= j) {
                            G[i] = gap_search_f(Q, pick4(rr, i));
                            tinc += G[i] == 4096 ? 4096u : (uint32_t)G[i] + 1u;
                            tev += G[i] < 4096 ? 1u : 0u;
                        } else {
                            G[i] = -1;
                        }
                    }
                    // exclusive scan over the TPW lanes of this word
                    const uint64_t mine = ((uint64_t)tev << 40) | tinc;
                    uint64_t x = mine;
                    for (uint32_t off = 1; off < TPW; off <<= 1) {
                        const uint64_t y = __shfl_up(x, off, TPW);
                        if (sub >= off) x += y;
                    }
                    const uint64_t total = __shfl(x, (int)(gbase + TPW - 1), 64);
                    const uint64_t ex = x - mine;
                    // locate the first event at or beyond R
                    uint64_t p = pos + (ex & ((1ull << 40) - 1));
                    uint32_t ee = e + (uint32_t)(ex >> 40);
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
                    const uint64_t gmask = (TPW == 64) ? ~0ull : (((1ull << TPW) - 1ull) << gbase);
                    const uint64_t gb = bal & gmask;
                    const uint32_t cut_sub = gb ? (uint32_t)(__ffsll((long long)gb) - 1) - gbase : TPW;
                    // apply events strictly before the cut
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const bool before = sub < cut_sub || (sub == cut_sub && i < cut_i);
                        if (G[i] >= 0) {
                            if (before && G[i] < 4096) {
                                const uint64_t at = p + (uint64_t)G[i];
                                const uint32_t rank = (uint32_t)(at >> 6), lane = (uint32_t)(at & 63);
                                const DevChan ch = P.chan[P.cls_chan[coff + rank]];
                                const uint4 br = philox4x32_10(make_uint4(ee >> 2, wlo, c, (2u << 24) | whi), k0, k1);
                                const uint32_t bv = pick4(br, ee & 3);
                                uint32_t jb;
                                if (ch.uniform) {
                                    jb = (uint32_t)(((uint64_t)bv * ch.J) >> 32);
                                } else {
                                    jb = ch.J - 1;
                                    for (uint32_t t = 0; t < ch.J; ++t)
                                        if ((uint64_t)bv < P.thr[ch.thr_off + t]) { jb = t; break; }
                                }
                                uint32_t mask = P.bmask[ch.bm_off + jb];
                                while (mask) {
                                    const uint32_t s = ch.sym0 + (uint32_t)__ffs(mask) - 1u;
                                    mask &= mask - 1u;
                                    for (uint32_t q = P.fr_sym_off[s]; q < P.fr_sym_off[s + 1]; ++q)
                                        atomicXor(&slots[(size_t)P.fr_sym_slot[q] * W + nlw], 1ull << lane);
                                }
                            }
                            if (G[i] < 4096) ++ee;
                            p += G[i] == 4096 ? 4096u : (uint32_t)G[i] + 1u;
                        }
                    }
                    if (cut_sub < TPW) {
                        const int src = (int)(gbase + cut_sub);
                        const uint32_t ci = (uint32_t)__shfl(cut_i, src, 64);
                        pos = __shfl(cut_p, src, 64);
                        e = __shfl(cut_e, src, 64);
                        j = jal + 4 * cut_sub + ci;
                        done = true;
                    } else {
                        pos += total & ((1ull << 40) - 1);
                        e += (uint32_t)(total >> 40);
                        j = jal + 4 * TPW;
                        done = pos >= R;
                    }
                }
                if (sub == 0) {
                    st_pos[c * W + nlw] = pos;
                    st_j[c * W + nlw] = j;
                    st_e[c * W + nlw] = e;
                }
            } else {
                const uint32_t n = d[0];
                const uint64_t wi = tile * W + elw;  // word index within the call
                const uint64_t w = A.word_begin + wi;
                uint64_t lanes = ~0ull;
                if (wi * 64 + 64 > A.shots) lanes = (wi * 64 >= A.shots) ? 0ull : ((1ull << (A.shots - wi * 64)) - 1ull);
                for (uint32_t v = enode; v < n; v += 256u / W) {
                    const uint32_t *nd = P.fr_data + d[1 + v];
                    const uint32_t flags = nd[0];
                    unsigned long long val = (flags & 1u) ? ~0ull : 0ull;
                    if (flags & 2u) {
                        unsigned long long *sp = &slots[(size_t)nd[1] * W + elw];
                        val ^= *sp;
                        *sp = 0;
                    }
                    if (flags & 4u) {
                        const uint32_t t = nd[2];
                        const uint4 o = philox4x32_10(make_uint4(t >> 1, (uint32_t)w, 0u, (3u << 24) | (uint32_t)(w >> 32)), k0, k1);
                        val ^= (t & 1) ? ((uint64_t)o.z | ((uint64_t)o.w << 32)) : ((uint64_t)o.x | ((uint64_t)o.y << 32));
                    }
                    const uint32_t np = nd[4];
                    for (uint32_t q = 0; q < np; ++q) atomicXor(&slots[(size_t)nd[5 + q] * W + elw], val);
                    const uint32_t sec = (flags >> 4) & 3u;
                    if (nd[3] != FR_NO_ROW && sec && ((A.sections >> (sec - 1)) & 1u) && wi < A.n_words)
                        A.out[(uint64_t)nd[3] * A.row_stride + wi] = val & lanes;
                }
            }
            __syncthreads();
        }
    }
}

size_t frame_lds_bytes(const DevProg &P, uint32_t wpb) {
    return (size_t)P.fr_n_slots * wpb * 8 + (size_t)P.n_cls * wpb * 16 + 16;
}

int frame_max_blocks_per_cu(size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, frame_kernel, 256, lds) != hipSuccess) return 1;
    return nb;
}

hipError_t launch_frame(const FrameArgs &A, uint32_t grid, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)frame_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)A.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(frame_kernel, dim3(grid), dim3(256), A.lds_bytes, st, A);
    return hipGetLastError();
}

}  // namespace symft
