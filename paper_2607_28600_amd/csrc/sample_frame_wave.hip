// sample_frame_wave.hip -- pure-frame sampling (peak active width 0) for
// gfx950 with wave-owned words.
//
// A workgroup of 16 waves owns a tile of 16 consecutive 64-shot words; wave w
// owns word w of the tile for the whole schedule.  Everything a record needs
// lives in that wave's own column of LDS accumulator slots (one uint64 holds
// one row of one word's 64 shots), so the schedule runs with no barrier
// between steps: a wave applies its word's noise flips, evaluates its nodes
// and pushes their values into successors' slots in program order, and LDS
// keeps one wave's accesses in order.  Waves meet only where their values
// become rows: nodes are staged in a double buffer [2][128 rows][16 words],
// and at each flush (one workgroup barrier) the 1024 threads store the staged
// rows as whole 128-byte lines while staging goes on in the other buffer.
//
// Per tile and wave:
//  * phase G: every noise event of the word's (class) streams under the draw
//    contract -- walks of 64 lanes x 4 gap draws decided without the table
//    except near a boundary, a wave prefix sum turning gaps into positions,
//    one branch-draw Philox block per lane -- each resolved through its
//    channel record and flip table into 32-bit flip entries (shot lane | step
//    << 6 | slot << 14), written in stream order to the workgroup's scratch;
//    then the word's RandomMeas columns, into LDS;
//  * phase S: the schedule ops (launch_args.hpp): NOISE streams the word's
//    entries of the step from scratch and XORs the lane bits into its slots;
//    BATCH evaluates up to 64 nodes, one per lane; FLUSH stores staged rows.
// A (word, class) stream with more slot flips than its capacity is instead
// walked afresh at each of its NOISE steps and applied at once, so records
// never depend on the capacity.
// Aggregate-count mode (paper Sec. 6) writes no rows: each lane ORs the
// postselected detectors and (expected-value-corrected) observables of its
// nodes into two registers, and the wave reduces them to its word's flags.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "frame_device.hpp"
#include "launch_args.hpp"
#include "philox.hpp"

namespace symft {

static constexpr uint32_t WV_THREADS = WV_TILE * 64;

// LDS layout: slots [16][NS + 1] u64 (wave w's column; slot NS stays 0) |
// RandomMeas words [16][n_rm] u64 | staging [2][128][16] u64 | walk positions
// [16][256] u32 | stream states [16][NC] | entry cursors, counts [16][NC] u32 |
// overflow flags [16] u32.
struct WaveLds {
    size_t slots, rmw, stage, tmp, wst, cur, cnt, ovf, total;
};

__host__ __device__ inline WaveLds wave_lds_layout(uint32_t n_slots, uint32_t n_rm, uint32_t n_cls) {
    WaveLds L;
    size_t o = 0;
    L.slots = o;
    o += (size_t)WV_TILE * (n_slots + 1) * 8;
    L.rmw = o;
    o += (size_t)WV_TILE * n_rm * 8;
    o = (o + 15) & ~(size_t)15;
    L.stage = o;
    o += (size_t)2 * WV_STAGE_ROWS * WV_TILE * 8;
    L.tmp = o;
    o += (size_t)WV_TILE * 256 * 4;
    L.wst = o;
    o += (size_t)WV_TILE * n_cls * sizeof(FrWord);
    L.cur = o;
    o += (size_t)WV_TILE * n_cls * 4;
    L.cnt = o;
    o += (size_t)WV_TILE * n_cls * 4;
    L.ovf = o;
    o += (size_t)WV_TILE * 4;
    L.total = (o + 15) & ~(size_t)15;
    return L;
}

// Stores of one flush: thread t takes staged row t / 8, words 2 (t % 8) and
// 2 (t % 8) + 1 of the tile (16 bytes; the 8 threads of a row write one
// 128-byte line).
__device__ __forceinline__ void wv_store(const WaveArgs &A, const unsigned long long *stg, uint32_t off, uint32_t n,
                                         uint64_t wt, bool full) {
    const uint32_t t = threadIdx.x, r = t >> 3, part = t & 7u;
    if (r >= n) return;
    const uint32_t row = A.P.wv_rows[off + r];
    if (row == FR_NO_ROW) return;
    const uint32_t sec = row < A.P.n_rec ? 1u : row < A.P.n_rec + A.P.n_det ? 2u : 4u;
    if (!(A.sections & sec)) return;
    const ulonglong2 val = *(const ulonglong2 *)&stg[(size_t)r * WV_TILE + 2 * part];
    const uint64_t wh = wt + 2 * part;
    unsigned long long *dst = (unsigned long long *)A.out + (uint64_t)row * A.row_stride + wh;
    if (full) {
        *(ulonglong2 *)dst = val;
        return;
    }
    if (wh >= A.n_words) return;
    const unsigned long long m0 = word_mask(wh, A.shots), m1 = word_mask(wh + 1, A.shots);
    if (A.store16 && wh + 1 < A.n_words) {
        *(ulonglong2 *)dst = make_ulonglong2(val.x & m0, val.y & m1);
    } else {
        dst[0] = val.x & m0;
        if (wh + 1 < A.n_words) dst[1] = val.y & m1;
    }
}

template <bool CM>
__global__ void __launch_bounds__(WV_THREADS) frame_wave_kernel(WaveArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const DevProg &P = A.P;
    const uint32_t NC = P.n_cls, NS = P.fr_n_slots;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const WaveLds L = wave_lds_layout(NS, P.wv_n_rm, NC);
    unsigned long long *col = (unsigned long long *)(smem + L.slots) + (size_t)wave * (NS + 1);
    unsigned long long *rmw = (unsigned long long *)(smem + L.rmw) + (size_t)wave * P.wv_n_rm;
    unsigned long long *stage = (unsigned long long *)(smem + L.stage);
    uint32_t *tmp = (uint32_t *)(smem + L.tmp) + (size_t)wave * 256;
    FrWord *wst = (FrWord *)(smem + L.wst) + (size_t)wave * NC;
    uint32_t *cur = (uint32_t *)(smem + L.cur) + (size_t)wave * NC;
    uint32_t *cnt = (uint32_t *)(smem + L.cnt) + (size_t)wave * NC;
    uint32_t *ovf = (uint32_t *)(smem + L.ovf);
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    const uint64_t n_tiles = (A.n_words + WV_TILE - 1) / WV_TILE;
    uint32_t *scr = A.scratch + (size_t)blockIdx.x * WV_TILE * A.word_entries + (size_t)wave * A.word_entries;
    const cptr<uint32_t> ops = uniform(P.wv_ops);
    for (uint32_t i = lane; i <= NS; i += 64) col[i] = 0ull;
    unsigned long long n_disc = 0, n_logic = 0;  // aggregate counts of this wave (lane 0)
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const uint64_t wt = tile * WV_TILE;
        const bool live = wt + wave < A.n_words;
        const uint64_t w = A.word_begin + wt + wave;
        const bool full = A.store16 && (wt + WV_TILE) * 64 <= A.shots;
        // phase G: the word's noise events as flip entries, then its RandomMeas columns
        bool over = false;
        for (uint32_t c = 0; c < NC; ++c) {
            const uint32_t coff = uniform(P.cls_off)[c], cend = (uniform(P.cls_off)[c + 1] - coff) * 64u;
            const uint32_t cap = A.cap_override ? A.cap_override : uniform(P.wv_cap)[c];
            uint32_t *out = scr + (A.cap_override ? c * A.cap_override : uniform(P.wv_capoff)[c]);
            uint32_t n = 0;
            if (live && !over) {
                const GapFast F = load_fast(P.cls_fast, c);
                Walk st = {0, 0, 0};
                auto none = [](uint32_t, unsigned long long) {};
                while (!walk_resolved<true>(P, F, c, coff, w, st, cend, tmp, out, cap, &n, k0, k1, none) &&
                       st.pos < cend && n <= cap) {
                }
                over = n > cap;
            }
            if (lane == 0) {
                cnt[c] = n;
                cur[c] = 0;
                wst[c] = FrWord{0, 0, 0, 0};
            }
        }
        if (lane == 0) ovf[wave] = over ? 1u : 0u;
        for (uint32_t i = lane; i < P.wv_n_rm; i += 64) rmw[i] = rm_word(P.wv_rm[i], w, k0, k1);
        // the wave reads back only what it wrote itself (entries through other lanes)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the previous tile's last flush has read its staging buffer
        __syncthreads();
        const bool ov = rfl(ovf[wave]) != 0;
        // phase S
        uint32_t pe = 0, pk = FR_NONE;  // entry prefetched for the next NOISE op, and its cursor
        auto fetch_entries = [&](uint32_t c) {
            pe = 0;
            pk = FR_NONE;
            if (c == FR_NONE || ov) return;
            const uint32_t k = rfl(cur[c]), kend = rfl(cnt[c]);
            const uint32_t *src = scr + (A.cap_override ? c * A.cap_override : uniform(P.wv_capoff)[c]);
            pk = k;
            if (k + lane < kend) pe = src[k + lane];
        };
        uint4 ra = make_uint4(0, 0, 0, 0), rb = ra;  // node record prefetched for the next BATCH op
        auto fetch_node = [&](uint32_t first, uint32_t n) {
            if (lane < n) {
                const uint4 *rec = (const uint4 *)(P.fr_nodes + 8 * (size_t)(first + lane));
                ra = rec[0];
                rb = rec[1];
            }
        };
        fetch_node(P.wv_first_batch, P.wv_first_batch_n);
        fetch_entries(P.wv_first_noise_cls);
        unsigned long long d_acc = 0, l_acc = 0;
        for (uint32_t o = 0; o < P.wv_n_ops; ++o) {
            const cptr<uint32_t> r = ops + (size_t)o * WV_OP_WORDS;
            const uint32_t kind = r[0];
            if (kind == WV_NOISE) {
                const uint32_t c = r[1], sl = r[3];
                if (ov) {
                    if (live) {
                        FrWord s0 = wst[c];
                        Walk st = {rfl(s0.pos), rfl(s0.j), rfl(s0.e)};
                        const uint32_t R = r[2] * 64u;
                        if (st.pos < R) {
                            const GapFast F = load_fast(P.cls_fast, c);
                            const uint32_t coff = uniform(P.cls_off)[c];
                            auto flip = [col](uint32_t sl, unsigned long long bit) { atomicXor(col + sl, bit); };
                            while (!walk_resolved<false>(P, F, c, coff, w, st, R, tmp, nullptr, 0, nullptr, k0, k1,
                                                         flip) &&
                                   st.pos < R) {
                            }
                            if (lane == 0) wst[c] = FrWord{st.pos, st.j, st.e, 0};
                        }
                    }
                } else {
                    const uint32_t *src = scr + (A.cap_override ? c * A.cap_override : uniform(P.wv_capoff)[c]);
                    uint32_t k = rfl(cur[c]);
                    const uint32_t kend = rfl(cnt[c]);
                    bool first = pk == k;
                    while (k < kend) {
                        const uint32_t idx = k + lane;
                        const uint32_t e = first ? pe : (idx < kend ? src[idx] : 0u);
                        first = false;
                        const bool take = idx < kend && ((e >> 6) & 0xFFu) == sl;
                        if (take) atomicXor(col + (e >> 14), 1ull << (e & 63u));
                        const uint32_t nd = (uint32_t)__popcll(__ballot(take));
                        k += nd;
                        if (nd < 64) break;
                    }
                    if (lane == 0) cur[c] = k;
                }
                fetch_entries(r[4]);
            } else if (kind == WV_BATCH) {
                const uint32_t n = r[2], pos = r[3], buf = r[4];
                const uint4 xa = ra, xb = rb;
                fetch_node(r[5], r[6]);
                if (lane < n) {
                    // record: slot | flags << 24, row, RandomMeas measurement, push count, first two
                    // successor slots, offset of further successors, RandomMeas index
                    const uint32_t flags = xa.x >> 24;
                    unsigned long long v =
                        __hip_atomic_exchange(col + (xa.x & 0xFFFFFFu), 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    if (flags & 1u) v = ~v;
                    if (flags & 4u) v ^= rmw[xb.w];
                    if (CM) {
                        const uint32_t sec = (flags >> 4) & 3u;
                        if (sec == 2u) {
                            const uint32_t d = xa.y - P.n_rec;
                            if ((A.cnt.post[d >> 5] >> (d & 31u)) & 1u) d_acc |= v;
                        } else if (sec == 3u) {
                            const uint32_t ob = xa.y - P.n_rec - P.n_det;
                            l_acc |= v ^ (((A.cnt.obs_exp[ob >> 5] >> (ob & 31u)) & 1u) ? ~0ull : 0ull);
                        }
                    } else {
                        stage[((size_t)buf * WV_STAGE_ROWS + pos + lane) * WV_TILE + wave] = v;
                    }
                    const uint32_t np = xa.w;
                    if (np > 0) atomicXor(col + xb.x, v);
                    if (np > 1) atomicXor(col + xb.y, v);
                    for (uint32_t q = 2; q < np; ++q) atomicXor(col + P.fr_push[xb.z + q - 2], v);
                }
            } else {
                // WV_FLUSH: every wave has staged its values of these rows
                __syncthreads();
                if (!CM) wv_store(A, stage + (size_t)r[3] * WV_STAGE_ROWS * WV_TILE, r[1], r[2], wt, full);
            }
        }
        if (CM) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                d_acc |= __shfl_xor(d_acc, off, 64);
                l_acc |= __shfl_xor(l_acc, off, 64);
            }
            if (lane == 0 && live) {
                const uint64_t wi = wt + wave;
                const unsigned long long m = word_mask(wi, A.shots), d = d_acc & m, l = l_acc & ~d & m;
                if (A.cnt.flags) {
                    A.cnt.flags[wi] = d;
                    A.cnt.flags[A.n_words + wi] = l;
                }
                n_disc += (unsigned long long)__popcll(d);
                n_logic += (unsigned long long)__popcll(l);
            }
        }
    }
    if (CM && A.cnt.counts && lane == 0) {
        if (n_disc) atomicAdd(&A.cnt.counts[0], n_disc);
        if (n_logic) atomicAdd(&A.cnt.counts[1], n_logic);
    }
}

size_t frame_wave_lds_bytes(const DevProg &P) { return wave_lds_layout(P.fr_n_slots, P.wv_n_rm, P.n_cls).total; }

uint32_t frame_wave_threads() { return WV_THREADS; }

int frame_wave_max_blocks_per_cu(size_t lds, bool cm) {
    int nb = 0;
    const void *k = cm ? (const void *)frame_wave_kernel<true> : (const void *)frame_wave_kernel<false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)WV_THREADS, lds) != hipSuccess) return 1;
    return nb;
}

hipError_t launch_frame_wave(const WaveArgs &A, uint32_t grid, hipStream_t st) {
    const void *k = A.cnt.on ? (const void *)frame_wave_kernel<true> : (const void *)frame_wave_kernel<false>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)A.lds_bytes);
    if (e != hipSuccess) return e;
    if (A.cnt.on)
        hipLaunchKernelGGL(frame_wave_kernel<true>, dim3(grid), dim3(WV_THREADS), A.lds_bytes, st, A);
    else
        hipLaunchKernelGGL(frame_wave_kernel<false>, dim3(grid), dim3(WV_THREADS), A.lds_bytes, st, A);
    return hipGetLastError();
}

}  // namespace symft
