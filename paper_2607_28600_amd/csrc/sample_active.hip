// sample_active.hip -- per-shot replay of a SymFT program with a dense active
// vector (paper Sec. 5), for gfx950.
//
// One workgroup owns one 64-shot word at a time (persistent loop over words):
//   1. noise events of the word are drawn cooperatively under the draw
//      contract (geometric gaps per probability class, block-wide prefix
//      sums over 1024 draws per step) and scattered by LDS atomic XOR into
//      the exogenous part of every consuming sign expression, exo[i];
//   2. RandomMeas words (64 bits per measurement) are drawn into exo[i];
//   3. shot groups of TPS threads step through the instruction stream in
//      lockstep (the stream and the active width trajectory are the same for
//      every shot).  lambda = const ^ exo bit ^ parity of earlier outcomes of
//      the shot.  The vector of each group lives in LDS or, when 2^k_max does
//      not fit, in an HBM scratch slice of the workgroup;
//   4. the word's records, detectors and observables are written.
// Aggregate-count mode (detector postselection, paper Sec. 6) writes per shot
// only a discarded flag and a logical-error flag.  A postselected detector is
// evaluated right after the instruction that makes its last record; a shot
// it rejects stops its dense work there (its group keeps to the workgroup's
// barriers), and the stream is left early once every shot group in flight is
// discarded.
// Branch probabilities are reduced in the amplitude precision (FP32 with
// compensated per-thread sums and pairwise wave trees, or FP64), and the
// threshold Pr(m = 0) and the renormalisation scale are formed in FP64.
#include <hip/hip_runtime.h>

#include "launch_args.hpp"
#include "philox.hpp"

namespace symft {

template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };



__device__ __forceinline__ uint32_t insert_bit(uint32_t z, uint32_t h, uint32_t v) {
    uint32_t lo = z & ((1u << h) - 1u);
    return lo | (v << h) | ((z >> h) << (h + 1));
}

__device__ __forceinline__ int parity(uint32_t v) { return __popc(v) & 1; }

// Instruction descriptors are read with a wave-uniform index; through the
// constant address space they come by scalar loads (no vector-memory wait, no
// lane-to-scalar moves).
__device__ __forceinline__ DevInstr load_instr(const DevInstr *p, uint32_t i) {
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)(p + i);
    DevInstr d;
    const uint32_t w0 = q[0], w1 = q[1];
    d.kind = (uint8_t)w0;
    d.k_in = (uint8_t)(w0 >> 8);
    d.h = (uint8_t)(w0 >> 16);
    d.mu = (uint8_t)(w0 >> 24);
    d.eta = (uint8_t)w1;
    d.lam_c = (uint8_t)(w1 >> 8);
    d.fuse = (uint8_t)(w1 >> 16);
    d.mg_len = (uint8_t)(w1 >> 24);
    d.a = q[2];
    d.b = q[3];
    d.meas = (int32_t)q[4];
    d.cm_off = q[5];
    d.cm_len = q[6];
    d.am_idx = q[7];
    d.c = __hiloint2double((int)q[9], (int)q[8]);
    d.s = __hiloint2double((int)q[11], (int)q[10]);
    d.cf = __uint_as_float(q[12]);
    d.sf = __uint_as_float(q[13]);
    d.base = q[14];
    d.mg_off = q[15];
    return d;
}

__device__ __forceinline__ DevMerge load_merge(const DevMerge *p, uint32_t i) {
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)(p + i);
    DevMerge m;
    m.dst = q[0];
    m.src1 = q[1];
    m.src2 = q[2];
    m.m1w = q[3];
    return m;
}

// The bits of x at the set bits of m, packed in increasing order (m wave-uniform).
__device__ __forceinline__ uint32_t gather_bits(uint32_t x, uint32_t m) {
    uint32_t r = 0, b = 1;
    while (m) {
        if (x & m & (0u - m)) r |= b;
        b <<= 1;
        m &= m - 1u;
    }
    return r;
}

// One pair of an ActivePairRot: (va at ya, vb at yb = ya ^ a) become
// c va + s i^q(ya) vb and c vb + s i^q(yb) va, q(y) = e0 + 2 b.(y ^ a) mod 4.
template <typename V, typename T>
__device__ __forceinline__ void pair_update(V &va, V &vb, uint32_t ya, uint32_t yb, int e0, uint32_t b, T c, T s) {
    const int qa = (e0 + 2 * parity(b & yb)) & 3;
    const int qb = (e0 + 2 * parity(b & ya)) & 3;
    // multiply by i^q
    V ta, tb;
    ta.x = (qa == 0) ? vb.x : (qa == 1) ? -vb.y : (qa == 2) ? -vb.x : vb.y;
    ta.y = (qa == 0) ? vb.y : (qa == 1) ? vb.x : (qa == 2) ? -vb.y : -vb.x;
    tb.x = (qb == 0) ? va.x : (qb == 1) ? -va.y : (qb == 2) ? -va.x : va.y;
    tb.y = (qb == 0) ? va.y : (qb == 1) ? va.x : (qb == 2) ? -va.y : -va.x;
    V na, nb;
    na.x = c * va.x + s * ta.x; na.y = c * va.y + s * ta.y;
    nb.x = c * vb.x + s * tb.x; nb.y = c * vb.y + s * tb.y;
    va = na;
    vb = nb;
}

// PromoteRot of amplitude v at x < N: x keeps c v, x + N gets -i ss v (ss = (-1)^lambda s).
template <typename V, typename T>
__device__ __forceinline__ void put_promoted(V *vec, uint32_t x, uint32_t N, V v, T c, T ss) {
    V hi;
    hi.x = ss * v.y;
    hi.y = -ss * v.x;
    vec[x + N] = hi;
    v.x *= c;
    v.y *= c;
    vec[x] = v;
}

// Block-wide exclusive scan of (a, b) pairs packed as 64-bit (a in low 32).
template <int BS>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *tmp, uint64_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) tmp[wid] = x;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) {
        uint64_t t = tmp[i];
        if (i < wid) base += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

// Draw the word's noise events and XOR them into exo[] (draw contract, domains 1 and 2).
template <int BS>
__device__ __forceinline__ void word_noise(const DevProg &P, uint64_t seed, uint64_t w, unsigned long long *exo, uint64_t *tmp) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t wlo = (uint32_t)w, whi = (uint32_t)(w >> 32);
    for (uint32_t c = 0; c < P.n_cls; ++c) {
        const uint64_t *Q = P.cls_Q + (size_t)c * 4097;
        const float il = P.cls_invlog2q[c];
        const GapFast F = P.cls_fast[c];
        const uint32_t coff = P.cls_off[c];
        const uint64_t end = (uint64_t)(P.cls_off[c + 1] - coff) * 64;
        uint64_t pos = 0, ev0 = 0, blk0 = 0;
        while (pos < end) {
            uint4 r = philox4x32_10(make_uint4((uint32_t)(blk0 + threadIdx.x), wlo, c, (1u << 24) | whi), k0, k1);
            uint32_t v[4] = {r.x, r.y, r.z, r.w};
            int G[4];
            uint32_t inc = 0, evc = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // the table-free margins, else the three-read window, else the table search (the same
                // decision as the pure-frame walks)
                if (!gap_fast_lean(F, v[i], G[i])) G[i] = v[i] >= F.vwin ? gap_window(Q, v[i], G[i]) : gap_of(Q, il, v[i]);
                inc += (G[i] == 4096) ? 4096u : (uint32_t)G[i] + 1u;
                evc += (G[i] < 4096) ? 1u : 0u;
            }
            uint64_t total;
            uint64_t ex = block_excl_scan<BS>(((uint64_t)evc << 40) | inc, tmp, total);
            uint64_t p = pos + (ex & ((1ull << 40) - 1));
            uint64_t e = ev0 + (ex >> 40);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (G[i] < 4096) {
                    uint64_t at = p + (uint64_t)G[i];
                    if (at < end) {
                        uint32_t rank = (uint32_t)(at >> 6), lane = (uint32_t)(at & 63);
                        const DevChan ch = P.chan[P.cls_chan[coff + rank]];
                        uint4 br = philox4x32_10(make_uint4((uint32_t)(e >> 2), wlo, c, (2u << 24) | whi), k0, k1);
                        uint32_t bv = (e & 3) == 0 ? br.x : (e & 3) == 1 ? br.y : (e & 3) == 2 ? br.z : br.w;
                        uint32_t j;
                        if (ch.uniform) {
                            j = (uint32_t)(((uint64_t)bv * ch.J) >> 32);
                        } else {
                            j = ch.J - 1;
                            for (uint32_t t = 0; t < ch.J; ++t)
                                if ((uint64_t)bv < P.thr[ch.thr_off + t]) { j = t; break; }
                        }
                        uint32_t mask = P.bmask[ch.bm_off + j];
                        while (mask) {
                            uint32_t s = ch.sym0 + (uint32_t)__ffs(mask) - 1u;
                            mask &= mask - 1u;
                            for (uint32_t q = P.sym_off[s]; q < P.sym_off[s + 1]; ++q)
                                atomicXor(&exo[P.sym_cons[q]], 1ull << lane);
                        }
                    }
                    ++e;
                }
                p += (G[i] == 4096) ? 4096u : (uint32_t)G[i] + 1u;
            }
            pos += total & ((1ull << 40) - 1);
            ev0 += total >> 40;
            blk0 += BS;
        }
    }
}

// v from another lane of the same row by the DPP pattern CTRL (a lane
// permutation: quad permutes and row mirrors).
template <int CTRL>
__device__ __forceinline__ float dpp_perm(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_perm(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over the TPS lanes of a shot group; every lane gets the same value
// (each step adds a lane's partner, and a + b == b + a exactly).  Inside a
// row of 16 lanes the partners come by DPP: quad permutes [1,0,3,2] and
// [2,3,0,1], then the half-row and row mirrors; wider groups add the other
// row halves of the wave by shuffles.
template <typename T, int BS>
__device__ __forceinline__ void group_sum2(T &s0, T &s1, int tps, T *red) {
    if (tps >= 2) {
        s0 += dpp_perm<0xB1>(s0);
        s1 += dpp_perm<0xB1>(s1);
    }
    if (tps >= 4) {
        s0 += dpp_perm<0x4E>(s0);
        s1 += dpp_perm<0x4E>(s1);
    }
    if (tps >= 8) {
        s0 += dpp_perm<0x141>(s0);
        s1 += dpp_perm<0x141>(s1);
    }
    if (tps >= 16) {
        s0 += dpp_perm<0x140>(s0);
        s1 += dpp_perm<0x140>(s1);
    }
    for (int off = 16; off < 64 && off < tps; off <<= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
    }
    if (tps > 64) {
        const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if (lane == 0) { red[2 * wid] = s0; red[2 * wid + 1] = s1; }
        __syncthreads();
        const int w0 = (threadIdx.x / tps) * (tps >> 6), nw = tps >> 6;
        T a = 0, b = 0;
        for (int i = 0; i < nw; ++i) { a += red[2 * (w0 + i)]; b += red[2 * (w0 + i) + 1]; }
        __syncthreads();
        s0 = a; s1 = b;
    }
}

// Parity of the causal part of lambda for the shot of this group: the refs
// come as (outcome word, bit mask) pairs, read by scalar loads, and the
// group's outcome words from LDS.
__device__ __forceinline__ int causal_parity(const DevProg &P, const DevInstr &I, const uint32_t *mb) {
    const __attribute__((address_space(4))) uint32_t *q =
        (const __attribute__((address_space(4))) uint32_t *)(P.cmeas + 2 * (size_t)I.cm_off);
    uint32_t x = 0;
    for (uint32_t j = 0; j < I.cm_len; ++j) x ^= mb[q[2 * j]] & q[2 * j + 1];
    return __popc(x) & 1;
}

template <typename T>
__device__ __forceinline__ void kahan_add(T &s, T &c, T v) {
    T y = v - c;
    T t = s + y;
    c = (t - s) - y;
    s = t;
}

// Words [wi_begin, wi_end) (step wi_step, call-relative) of the call described
// by A, run by this workgroup.  `slice` picks the HBM vector slice when the
// vectors do not fit LDS.  CM: aggregate-count mode (A.cnt), compiled apart
// so that the record path carries none of its state.
template <typename T, int BS, bool LDSV, bool CM>
__device__ __forceinline__ void run_active_words(const ActiveArgs &A, uint64_t wi_begin, uint64_t wi_end, uint64_t wi_step,
                                 uint32_t slice, unsigned char *smem) {
    using V = typename C2<T>::type;
    const DevProg &P = A.P;
    const int tps = (int)A.tps;
    const int G = BS / tps;
    const int g = threadIdx.x / tps, r = threadIdx.x % tps;
    const uint32_t mw = (P.n_meas + 31) / 32;
    // LDS carve-up
    unsigned long long *exo = (unsigned long long *)smem;                       // n_instr
    unsigned long long *recw = exo + P.n_instr;                                  // n_rec
    uint64_t *tmp = (uint64_t *)(recw + P.n_rec);                                // 16 + 4 + 24 count words
    T *red = (T *)(tmp + 44);                                                    // 2 * BS/64
    uint32_t *mbits = (uint32_t *)(red + 2 * (BS / 64) + 2);                     // G * mw
    // G * 2^kmax (LDS mode); offset from smem so the pointer stays in the LDS address space
    V *vec_lds = (V *)(smem + ((((unsigned char *)(mbits + G * mw) - smem) + 15) & ~(ptrdiff_t)15));
    const size_t vlen = (size_t)1 << P.k_max;
    V *vec;
    if (LDSV) vec = vec_lds + (size_t)g * vlen;
    else vec = (V *)A.scratch + ((size_t)slice * G + g) * A.scratch_stride;
    uint32_t *mb = mbits + g * mw;
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    constexpr bool cm = CM;
    // count mode: the word's discarded / logical-error flags, and the workgroup's totals
    unsigned long long *fdisc = (unsigned long long *)&tmp[16], *flogic = (unsigned long long *)&tmp[17];
    unsigned long long *tot = (unsigned long long *)&tmp[18];
    // three rows of 64 verdict bytes, one byte per shot group (G <= 64)
    uint8_t *gv = (uint8_t *)&tmp[20];
    if (cm && threadIdx.x == 0) {
        tot[0] = 0ull;
        tot[1] = 0ull;
    }

    // Work units: whole words, or in count mode 2^part_log2 parts of a word (consecutive shots).  A part
    // recomputes its word's draws and owns its shots' flag bits.
    const uint32_t pl = CM ? A.part_log2 : 0u;
    for (uint64_t ui = wi_begin; ui < wi_end; ui += wi_step) {
        const uint64_t wi = ui >> pl;
        const int lane0 = (int)((uint32_t)(ui & ((1u << pl) - 1u)) << (6u - pl)), lane1 = lane0 + (64 >> pl);
        const uint64_t w = A.word_begin + wi;
        for (uint32_t i = threadIdx.x; i < P.n_instr; i += BS) exo[i] = 0;
        for (uint32_t i = threadIdx.x; i < P.n_rec; i += BS) recw[i] = 0;
        if (cm && threadIdx.x == 0) {
            *fdisc = 0ull;
            *flogic = 0ull;
        }
        __syncthreads();
        word_noise<BS>(P, A.seed, w, exo, tmp);
        for (uint32_t i = threadIdx.x; i < P.n_rm; i += BS) {
            const uint32_t ii = P.rm_list[i];
            const uint32_t t = (uint32_t)P.instr[ii].meas;
            uint4 o = philox4x32_10(make_uint4(t >> 1, (uint32_t)w, 0u, (3u << 24) | (uint32_t)(w >> 32)), k0, k1);
            exo[ii] = (t & 1) ? ((uint64_t)o.z | ((uint64_t)o.w << 32)) : ((uint64_t)o.x | ((uint64_t)o.y << 32));
        }
        __syncthreads();

        // Shot groups of at most 64 threads lie inside one wave and touch only
        // their own vector and outcome bits, so with LDS vectors the batch loop
        // needs no workgroup barrier: a wave's LDS accesses are performed in
        // issue order, and a wave-scope fence keeps the compiler's order.  The
        // waves then run their shots independently until the word's end.
        const bool wsync = LDSV && tps <= 64;
        auto gsync = [&]() {
            if (wsync) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else {
                __syncthreads();
            }
        };
        for (int base = lane0; base < lane1; base += G) {
            const int lane = base + g;
            const uint64_t shot = w * 64 + (uint64_t)lane;
            for (uint32_t i = (uint32_t)r; i < mw; i += (uint32_t)tps) mb[i] = 0;
            if (r == 0) { vec[0].x = (T)1; vec[0].y = (T)0; }
            bool dead = false;  // the shot was discarded by a postselected detector
            // Uniform draws of active measurements: each lane of a group draws the one
            // for a different upcoming active measurement of the group's shot, a batch
            // of min(tps, 64) at a time, and the group reads the one it needs by a
            // shuffle (one Philox block per lane per batch instead of per measurement).
            const uint32_t unit = tps < 64 ? (uint32_t)tps : 64u;
            uint32_t ux = 0, uy = 0, ubase = 0, uend = 0;
            uint32_t nchk = 0;  // checks done in this batch of shots
            if (cm && !wsync) {
                // verdict rows start "live" for the G groups and "discarded" past them
                for (uint32_t i = threadIdx.x; i < 3 * 64; i += BS) gv[i] = (i & 63u) < (uint32_t)G ? 0 : 1;
            }
            gsync();
            // the next instruction's descriptor and first causal ref are fetched
            // while this one runs
            // coefficients of the PromoteRot at instruction j, for a rotation that runs it in its own pass
            auto promote_coef = [&](uint32_t j, T &pc, T &pss) {
                const DevInstr J = load_instr(P.instr, j);
                const int lam2 = (int)J.lam_c ^ (int)((exo[j] >> lane) & 1ull) ^ causal_parity(P, J, mb);
                pc = sizeof(T) == 8 ? (T)J.c : (T)J.cf;
                const T s2 = sizeof(T) == 8 ? (T)J.s : (T)J.sf;
                pss = lam2 ? -s2 : s2;
            };
            for (uint32_t ii = 0; ii < P.n_instr; ++ii) {
                const DevInstr I = load_instr(P.instr, ii);
                const uint32_t N = 1u << I.k_in;
                // A discarded group skips the barrier-free loops below; guarding them
                // (rather than shortening their bounds) keeps the loop control scalar.
                const bool live = !dead;
                const int lam = (int)I.lam_c ^ (int)((exo[ii] >> lane) & 1ull) ^ causal_parity(P, I, mb);
                const T c = sizeof(T) == 8 ? (T)I.c : (T)I.cf;
                const T s = sizeof(T) == 8 ? (T)I.s : (T)I.sf;
                uint32_t mbit = 0;  // this instruction's outcome, known to every thread of the group
                // Product-component programs: the component this instruction runs on,
                // after the Kronecker merges of the components its masks span
                V *vb = vec + I.base;
                for (uint32_t q = 0; q < I.mg_len; ++q) {
                    const DevMerge M = load_merge(P.merges, I.mg_off + q);
                    const uint32_t NW = 1u << (M.m1w >> 24), m1 = M.m1w & 0xFFFFFFu, m2 = (NW - 1u) & ~m1;
                    if (live)
                    for (uint32_t x = (uint32_t)r; x < NW; x += (uint32_t)tps) {
                        const V u = vec[M.src1 + gather_bits(x, m1)], w = vec[M.src2 + gather_bits(x, m2)];
                        V o;
                        o.x = u.x * w.x - u.y * w.y;
                        o.y = u.x * w.y + u.y * w.x;
                        vec[M.dst + x] = o;
                    }
                    gsync();
                }
                switch (I.kind) {
                case 8: {  // PromoteRot that starts a component of its own, from the amplitude 1
                    const T ss = lam ? -s : s;
                    if (live && r == 0) {
                        V lo, hi;
                        lo.x = c;
                        lo.y = (T)0;
                        hi.x = (T)0;
                        hi.y = -ss;
                        vb[0] = lo;
                        vb[1] = hi;
                    }
                    break;
                }
                case 1: {  // PromoteRot: x0 <- c a_x, x1 <- -i (-1)^lam s a_x
                    const T ss = lam ? -s : s;
                    if (live)
                    for (uint32_t x = (uint32_t)r; x < N; x += (uint32_t)tps) put_promoted(vb, x, N, vb[x], c, ss);
                    break;
                }
                case 2: {  // ActiveDiagRot: a_x *= c - i sigma s, sigma = (-1)^lam mu (-1)^(b.x)
                    const int neg = lam ^ (I.mu == 2 ? 1 : 0);
                    T pc = 0, pss = 0;
                    if (I.fuse) promote_coef(ii + 1, pc, pss);
                    if (live)
                    for (uint32_t x = (uint32_t)r; x < N; x += (uint32_t)tps) {
                        const T sg = (neg ^ parity(I.b & x)) ? -s : s;
                        V v = vb[x];
                        V o;
                        o.x = c * v.x + sg * v.y;
                        o.y = c * v.y - sg * v.x;
                        if (I.fuse) put_promoted(vb, x, N, o, pc, pss);
                        else vb[x] = o;
                    }
                    if (I.fuse) ++ii;  // the PromoteRot ran in this pass
                    break;
                }
                case 3: {  // ActivePairRot on pairs (x0, x0 ^ a), bit h of x0 = 0
                    // a'_x = c a_x - i (-1)^lam s mu (-1)^(b.(x^a)) a_(x^a); with mu = i^m:
                    // -i mu = i^(m+3)
                    const int e0 = (int)I.mu + 3 + 2 * lam;
                    // passes over two pair rotations: vectors in HBM scratch and FP32 only
                    // (with LDS vectors the four scattered reads of a coset cost more than
                    // the second pass; FP64 would lose occupancy), and only when every
                    // thread of the group has a coset
                    const uint32_t fz =
                        (I.fuse >= 2 && (LDSV || sizeof(T) == 8 || (N >> 2) < (uint32_t)tps)) ? 0u : I.fuse;
                    T pc = 0, pss = 0;
                    if (fz == 1 || fz == 3) promote_coef(ii + (fz == 3 ? 2u : 1u), pc, pss);
                    if (fz >= 2) {
                        // with the pair rotation (mask a2) that follows, on the cosets
                        // x + {0, a, a2, a ^ a2}: x has zeros at h and at the top bit of
                        // a2 reduced by a at h, two pivots no coset repeats
                        const DevInstr I2 = load_instr(P.instr, ii + 1);
                        const int lam2 = (int)I2.lam_c ^ (int)((exo[ii + 1] >> lane) & 1ull) ^ causal_parity(P, I2, mb);
                        const T c2 = sizeof(T) == 8 ? (T)I2.c : (T)I2.cf;
                        const T s2 = sizeof(T) == 8 ? (T)I2.s : (T)I2.sf;
                        const int e02 = (int)I2.mu + 3 + 2 * lam2;
                        const uint32_t a2r = I2.a ^ (((I2.a >> I.h) & 1u) ? I.a : 0u);
                        const uint32_t h2 = 31u - (uint32_t)__builtin_clz(a2r);
                        const uint32_t plo = h2 < I.h ? h2 : (uint32_t)I.h, phi = h2 < I.h ? (uint32_t)I.h : h2;
                        if (live)
                        for (uint32_t z = (uint32_t)r; z < (N >> 2); z += (uint32_t)tps) {
                            const uint32_t y0 = insert_bit(insert_bit(z, plo, 0), phi, 0);
                            const uint32_t y1 = y0 ^ I.a, y2 = y0 ^ I2.a, y3 = y1 ^ I2.a;
                            V v0 = vb[y0], v1 = vb[y1], v2 = vb[y2], v3 = vb[y3];
                            pair_update(v0, v1, y0, y1, e0, I.b, c, s);
                            pair_update(v2, v3, y2, y3, e0, I.b, c, s);
                            pair_update(v0, v2, y0, y2, e02, I2.b, c2, s2);
                            pair_update(v1, v3, y1, y3, e02, I2.b, c2, s2);
                            if (fz == 3) {
                                put_promoted(vb, y0, N, v0, pc, pss);
                                put_promoted(vb, y1, N, v1, pc, pss);
                                put_promoted(vb, y2, N, v2, pc, pss);
                                put_promoted(vb, y3, N, v3, pc, pss);
                            } else {
                                vb[y0] = v0;
                                vb[y1] = v1;
                                vb[y2] = v2;
                                vb[y3] = v3;
                            }
                        }
                        ii += fz == 3 ? 2u : 1u;  // the instructions that ran in this pass
                        break;
                    }
                    const uint32_t half = N >> 1;
                    if (live)
                    for (uint32_t z = (uint32_t)r; z < half; z += (uint32_t)tps) {
                        const uint32_t x0 = insert_bit(z, I.h, 0), x1 = x0 ^ I.a;
                        V a0 = vb[x0], a1 = vb[x1];
                        // factor f0 multiplies a1 into x0's update, f1 multiplies a0 into x1's
                        const int q0 = (e0 + 2 * parity(I.b & x1)) & 3;
                        const int q1 = (e0 + 2 * parity(I.b & x0)) & 3;
                        // multiply by s * i^q
                        V t0, t1;
                        t0.x = (q0 == 0) ? a1.x : (q0 == 1) ? -a1.y : (q0 == 2) ? -a1.x : a1.y;
                        t0.y = (q0 == 0) ? a1.y : (q0 == 1) ? a1.x : (q0 == 2) ? -a1.y : -a1.x;
                        t1.x = (q1 == 0) ? a0.x : (q1 == 1) ? -a0.y : (q1 == 2) ? -a0.x : a0.y;
                        t1.y = (q1 == 0) ? a0.y : (q1 == 1) ? a0.x : (q1 == 2) ? -a0.y : -a0.x;
                        V n0, n1;
                        n0.x = c * a0.x + s * t0.x; n0.y = c * a0.y + s * t0.y;
                        n1.x = c * a1.x + s * t1.x; n1.y = c * a1.y + s * t1.y;
                        if (fz) {
                            put_promoted(vb, x0, N, n0, pc, pss);
                            put_promoted(vb, x1, N, n1, pc, pss);
                        } else {
                            vb[x0] = n0;
                            vb[x1] = n1;
                        }
                    }
                    if (fz) ++ii;  // the PromoteRot ran in this pass
                    break;
                }
                case 4: {  // RandomMeas
                    mbit = (uint32_t)(exo[ii] >> lane) & 1u;
                    if (r == 0) {
                        const uint32_t t = (uint32_t)I.meas;
                        if ((exo[ii] >> lane) & 1ull) mb[t >> 5] |= 1u << (t & 31);
                        if (A.p0_out && shot - A.probe_shot0 < A.probe_n) A.p0_out[(shot - A.probe_shot0) * P.n_meas + t] = 0.5;
                    }
                    break;
                }
                case 5: {  // DetMeas: m = lambda ^ eta (exo holds the noise part of lambda)
                    mbit = (uint32_t)(lam ^ I.eta);
                    if (r == 0) {
                        const uint32_t t = (uint32_t)I.meas;
                        if (lam ^ I.eta) mb[t >> 5] |= 1u << (t & 31);
                        if (A.p0_out && shot - A.probe_shot0 < A.probe_n)
                            A.p0_out[(shot - A.probe_shot0) * P.n_meas + t] = (lam ^ I.eta) ? 0.0 : 1.0;
                    }
                    break;
                }
                case 6:    // ActiveDiagMeas
                case 7: {  // ActivePairMeas
                    const uint32_t half = N >> 1;
                    const bool pair = I.kind == 7;
                    const uint32_t t = (uint32_t)I.meas;
                    if (I.am_idx >= uend) {
                        ubase = I.am_idx;
                        uend = ubase + unit;
                        const uint32_t j = ubase + threadIdx.x % unit;
                        if (j < P.n_am) {
                            const uint32_t tj = P.am_meas[j];
                            const uint4 oj =
                                philox4x32_10(make_uint4(tj, (uint32_t)shot, (uint32_t)(shot >> 32), 4u << 24), k0, k1);
                            ux = oj.x;
                            uy = oj.y;
                        }
                    }
                    const int usrc = (int)(((threadIdx.x & 63u) & ~(unit - 1u)) + (I.am_idx - ubase));
                    const uint32_t ox = (uint32_t)__shfl((int)ux, usrc, 64), oy = (uint32_t)__shfl((int)uy, usrc, 64);
                    // conj(mu) (-1)^(b.u0) for the pair case; diag: parity classes of b.x
                    T s0 = 0, s1 = 0, c0 = 0, c1 = 0;
                    const T rs2 = (T)0.70710678118654752440;
                    if (!live) {
                    } else if (!pair) {
                        for (uint32_t x = (uint32_t)r; x < N; x += (uint32_t)tps) {
                            V v = vb[x];
                            T m2 = v.x * v.x + v.y * v.y;
                            if (parity(I.b & x)) kahan_add(s1, c1, m2); else kahan_add(s0, c0, m2);
                        }
                    } else {
                        const int mc = (4 - (int)I.mu) & 3;  // conj(mu) = i^mc
                        for (uint32_t z = (uint32_t)r; z < half; z += (uint32_t)tps) {
                            const uint32_t u0 = insert_bit(z, I.h, 0);
                            V a0 = vb[u0], a1 = vb[u0 ^ I.a];
                            const int q = (mc + 2 * parity(I.b & u0)) & 3;
                            T tx = (q == 0) ? a1.x : (q == 1) ? -a1.y : (q == 2) ? -a1.x : a1.y;
                            T ty = (q == 0) ? a1.y : (q == 1) ? a1.x : (q == 2) ? -a1.y : -a1.x;
                            T bx = (a0.x + tx) * rs2, by = (a0.y + ty) * rs2;
                            T dx = (a0.x - tx) * rs2, dy = (a0.y - ty) * rs2;
                            kahan_add(s0, c0, bx * bx + by * by);
                            kahan_add(s1, c1, dx * dx + dy * dy);
                        }
                    }
                    group_sum2<T, BS>(s0, s1, tps, red);
                    // y = classes: diag keeps b.x = m ^ lam ^ eta, pair keeps y = m ^ lam
                    const int flip = pair ? lam : (lam ^ (int)I.eta);
                    const double S0 = (double)s0, S1 = (double)s1;
                    const double p0 = (flip ? S1 : S0) / (S0 + S1);
                    const double u = (double)(((uint64_t)ox << 21) + (uint64_t)(oy >> 11)) * 0x1p-53;
                    const int m = (u < p0) ? 0 : 1;
                    mbit = (uint32_t)m;
                    const int y = m ^ flip;  // kept class
                    const double Sy = y ? S1 : S0;
                    const T scale = (T)(1.0 / sqrt(Sy > 0x1p-1000 ? Sy : 0x1p-1000));
                    if (r == 0) {
                        if (m) mb[t >> 5] |= 1u << (t & 31);
                        if (A.p0_out && shot - A.probe_shot0 < A.probe_n) A.p0_out[(shot - A.probe_shot0) * P.n_meas + t] = p0;
                    }
                    // compaction 2^k -> 2^(k-1); sources of output z lie at indices >= z, so
                    // chunks are read into registers, then written after a barrier
                    const uint32_t chunk = (uint32_t)tps * 4u;
                    const int mc = (4 - (int)I.mu) & 3;
                    const uint32_t bl = I.b & ~(1u << I.h);
                    for (uint32_t z0 = 0; z0 < half; z0 += chunk) {
                        V vals[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const uint32_t z = z0 + (uint32_t)e * (uint32_t)tps + (uint32_t)r;
                            if (z < half && !dead) {
                                if (!pair) {
                                    const uint32_t uu = insert_bit(z, I.h, (uint32_t)y);
                                    const uint32_t x = uu ^ ((uint32_t)parity(bl & uu) << I.h);
                                    V v = vb[x];
                                    vals[e].x = v.x * scale; vals[e].y = v.y * scale;
                                } else {
                                    const uint32_t u0 = insert_bit(z, I.h, 0);
                                    V a0 = vb[u0], a1 = vb[u0 ^ I.a];
                                    const int q = (mc + 2 * parity(I.b & u0) + 2 * y) & 3;
                                    T tx = (q == 0) ? a1.x : (q == 1) ? -a1.y : (q == 2) ? -a1.x : a1.y;
                                    T ty = (q == 0) ? a1.y : (q == 1) ? a1.x : (q == 2) ? -a1.y : -a1.x;
                                    vals[e].x = (a0.x + tx) * rs2 * scale;
                                    vals[e].y = (a0.y + ty) * rs2 * scale;
                                }
                            }
                        }
                        gsync();
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const uint32_t z = z0 + (uint32_t)e * (uint32_t)tps + (uint32_t)r;
                            if (z < half && !dead) vb[z] = vals[e];
                        }
                        gsync();
                    }
                    break;
                }
                default: break;
                }
                // Postselected detectors whose last record this instruction made:
                // the group's threads take one detector each; its parity comes
                // from the group's earlier outcome bits and, for this
                // instruction's own outcome, from the register every thread of
                // the group holds.
                uint32_t c0 = 0, c1 = 0;  // this instruction's checks (scalar loads)
                if (cm) {
                    const __attribute__((address_space(4))) uint32_t *co =
                        (const __attribute__((address_space(4))) uint32_t *)A.cnt.chk_off;
                    c0 = co[ii];
                    c1 = co[ii + 1];
                }
                const bool chk = c0 < c1;
                uint32_t fired = 0;
                if (chk && !dead) {
                    for (uint32_t q = c0 + (uint32_t)r; q < c1; q += (uint32_t)tps) {
                        uint32_t x = 0;
                        for (uint32_t e = A.cnt.chk_mo[q]; e < A.cnt.chk_mo[q + 1]; ++e) {
                            const uint32_t t = A.cnt.chk_meas[e];
                            x ^= t == (uint32_t)I.meas ? mbit : (mb[t >> 5] >> (t & 31)) & 1u;
                        }
                        fired |= x;
                    }
                }
                if (wsync) {
                    gsync();
                    if (chk) {
                        // the group's lanes are contiguous in the wave
                        const uint64_t bal = __ballot(fired);
                        const uint32_t sub = (threadIdx.x & 63u) & ~((uint32_t)tps - 1u);
                        const uint64_t gm = (tps == 64 ? ~0ull : ((1ull << tps) - 1ull)) << sub;
                        dead = dead || (bal & gm) != 0;
                        // this wave leaves the stream once all its groups are discarded
                        if (__ballot(!dead) == 0) break;
                    }
                    continue;
                }
                // Groups spanning waves: a verdict byte per group in row c % 3
                // (check c of this batch), read back after the barrier that ends
                // the instruction.  Row (c + 2) % 3 is cleared after it: its last
                // reads precede this barrier, its next writes follow the next one.
                uint8_t *row = gv + 64u * (nchk % 3u);
                if (chk && (dead ? r == 0 : fired != 0)) row[g] = 1;
                __syncthreads();
                if (chk) {
                    dead = row[g] != 0;
                    // leave the stream once no group in flight has a live shot
                    bool all = true;  // bytes past G read as discarded
                    for (uint32_t i = 0; i < (uint32_t)G; i += 4u) all = all && *(const uint32_t *)(row + i) == 0x01010101u;
                    if (all) break;
                    if (threadIdx.x < 64u) gv[64u * ((nchk + 2u) % 3u) + threadIdx.x] = threadIdx.x < (uint32_t)G ? 0 : 1;
                    ++nchk;
                }
            }
            if (A.amp_out && shot - A.probe_shot0 < A.probe_n) {
                // probe: the shot's final active vector (complete: every instruction
                // ends with the group's synchronisation)
                double *dst = A.amp_out + (shot - A.probe_shot0) * (2ull << A.amp_k);
                for (uint32_t x = (uint32_t)r; x < (1u << A.amp_k); x += (uint32_t)tps) {
                    const V v = vec[x];
                    dst[2 * x] = (double)v.x;
                    dst[2 * x + 1] = (double)v.y;
                }
            }
            if (cm) {
                // the shot's flags: discarded, or a logical error when an
                // observable differs from its expected value
                if (r == 0) {
                    if (dead) {
                        atomicOr(fdisc, 1ull << lane);
                    } else {
                        uint32_t le = 0;
                        for (uint32_t b = 0; b < P.n_obs; ++b) {
                            uint32_t x = (A.cnt.obs_exp[b >> 5] >> (b & 31)) & 1u;
                            for (uint32_t q = P.obs_off[b]; q < P.obs_off[b + 1]; ++q) {
                                const uint32_t t = P.rec_meas[P.obs_rows[q]];
                                x ^= (mb[t >> 5] >> (t & 31)) & 1u;
                            }
                            le |= x;
                        }
                        if (le) atomicOr(flogic, 1ull << lane);
                    }
                }
            } else if (shot - A.word_begin * 64 < A.shots) {
                // visible records of this shot into the word's rows
                for (uint32_t row = (uint32_t)r; row < P.n_rec; row += (uint32_t)tps) {
                    const uint32_t t = P.rec_meas[row];
                    if ((mb[t >> 5] >> (t & 31)) & 1u) atomicOr(&recw[row], 1ull << lane);
                }
            }
            gsync();
        }
        __syncthreads();
        const uint64_t col = wi;
        if (cm) {
            if (threadIdx.x == 0) {
                const uint64_t s0 = wi * 64;
                unsigned long long m = s0 + 64 <= A.shots ? ~0ull : (1ull << (A.shots - s0)) - 1ull;
                const unsigned long long pm = (~0ull >> (64 - (64 >> pl))) << lane0;  // this unit's bits
                m &= pm;
                const unsigned long long d = *fdisc & m, l = *flogic & ~d & m;
                if (A.cnt.flags) {
                    if (pl == 0) {
                        A.cnt.flags[col] = d;
                        A.cnt.flags[A.n_words + col] = l;
                    } else if (pl == 1) {  // this part's 32 bits of the two flag words
                        ((uint32_t *)(A.cnt.flags + col))[lane0 >> 5] = (uint32_t)(d >> lane0);
                        ((uint32_t *)(A.cnt.flags + A.n_words + col))[lane0 >> 5] = (uint32_t)(l >> lane0);
                    } else if (pl == 2) {  // 16 bits
                        ((uint16_t *)(A.cnt.flags + col))[lane0 >> 4] = (uint16_t)(d >> lane0);
                        ((uint16_t *)(A.cnt.flags + A.n_words + col))[lane0 >> 4] = (uint16_t)(l >> lane0);
                    } else if (pl == 3) {  // 8 bits
                        ((uint8_t *)(A.cnt.flags + col))[lane0 >> 3] = (uint8_t)(d >> lane0);
                        ((uint8_t *)(A.cnt.flags + A.n_words + col))[lane0 >> 3] = (uint8_t)(l >> lane0);
                    } else {  // parts below a byte: clear and set this part's bits (padding included),
                              // which no other unit touches
                        unsigned long long *f0 = (unsigned long long *)(A.cnt.flags + col);
                        unsigned long long *f1 = (unsigned long long *)(A.cnt.flags + A.n_words + col);
                        atomicAnd(f0, ~pm);
                        atomicOr(f0, d);
                        atomicAnd(f1, ~pm);
                        atomicOr(f1, l);
                    }
                }
                tot[0] += (unsigned long long)__popcll(d);
                tot[1] += (unsigned long long)__popcll(l);
            }
            __syncthreads();
            continue;
        }
        // write rows: records, detectors, observables
        if (A.sections & 1u)
            for (uint32_t row = threadIdx.x; row < P.n_rec; row += BS) A.out[(uint64_t)row * A.row_stride + col] = recw[row];
        if (A.sections & 2u)
            for (uint32_t d = threadIdx.x; d < P.n_det; d += BS) {
                uint64_t v = 0;
                for (uint32_t q = P.det_off[d]; q < P.det_off[d + 1]; ++q) v ^= recw[P.det_rows[q]];
                A.out[(uint64_t)(P.n_rec + d) * A.row_stride + col] = v;
            }
        if (A.sections & 4u)
            for (uint32_t b = threadIdx.x; b < P.n_obs; b += BS) {
                uint64_t v = 0;
                for (uint32_t q = P.obs_off[b]; q < P.obs_off[b + 1]; ++q) v ^= recw[P.obs_rows[q]];
                A.out[(uint64_t)(P.n_rec + P.n_det + b) * A.row_stride + col] = v;
            }
        __syncthreads();
    }
    if (cm && A.cnt.counts && threadIdx.x == 0) {
        if (tot[0]) atomicAdd(&A.cnt.counts[0], tot[0]);
        if (tot[1]) atomicAdd(&A.cnt.counts[1], tot[1]);
    }
}

template <typename T, int BS, bool LDSV, bool CM>
__global__ void __launch_bounds__(BS) active_kernel(ActiveArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint64_t n_units = CM ? A.n_words << A.part_log2 : A.n_words;
    if (CM && A.unit_counter) {
        // count mode: units from a global counter, so that workgroups whose shots were rejected early
        // take more of them; every workgroup leaves once the counter passes the last unit
        __shared__ uint32_t s_u;
        while (true) {
            __syncthreads();  // the previous unit's reads of s_u are done
            if (threadIdx.x == 0) s_u = atomicAdd(A.unit_counter, 1u);
            __syncthreads();
            const uint32_t u = s_u;
            if (u >= n_units) break;
            run_active_words<T, BS, LDSV, CM>(A, u, (uint64_t)u + 1, 1, blockIdx.x, smem);
        }
        return;
    }
    run_active_words<T, BS, LDSV, CM>(A, blockIdx.x, n_units, gridDim.x, blockIdx.x, smem);
}

// ----------------------------------------------------------------- lane kernel
// One wave per 64-shot word and one lane per shot, for programs whose vector
// buffer is small (typically product components, a few amplitudes per shot).
// Each shot's buffer lives in LDS amplitude-major (amplitude x of lane l at
// x * 64 + l), and its outcome bits likewise (word j of lane l at j * 64 + l).
// Every index, pivot and mask parity of an instruction is then the same for
// all lanes (scalar work shared by the 64 shots); only the sign bits, the
// branch decisions and the kept class differ per lane.  A measurement's sums,
// decision and compaction are each lane's own, so the wave needs no shuffles,
// reductions or barriers; the word's noise and RandomMeas words are drawn by
// the same wave under the same draw contract (its 64-lane draw rounds take
// the same sequence of Philox blocks as the shot-group kernel's wider ones).

__device__ __forceinline__ void lane_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The word's noise events, XORed into exo[] (domains 1 and 2 of the draw contract).
__device__ __forceinline__ void word_noise_wave(const DevProg &P, uint64_t seed, uint64_t w, unsigned long long *exo) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t wlo = (uint32_t)w, whi = (uint32_t)(w >> 32);
    for (uint32_t c = 0; c < P.n_cls; ++c) {
        const uint64_t *Q = P.cls_Q + (size_t)c * 4097;
        const float il = P.cls_invlog2q[c];
        const GapFast F = P.cls_fast[c];
        const uint32_t coff = P.cls_off[c];
        const uint64_t end = (uint64_t)(P.cls_off[c + 1] - coff) * 64;
        uint64_t pos = 0, ev0 = 0, blk0 = 0;
        while (pos < end) {
            const uint4 r = philox4x32_10(make_uint4((uint32_t)(blk0 + lane), wlo, c, (1u << 24) | whi), k0, k1);
            const uint32_t v[4] = {r.x, r.y, r.z, r.w};
            int G[4];
            uint32_t inc = 0, evc = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (!gap_fast_lean(F, v[i], G[i])) G[i] = v[i] >= F.vwin ? gap_window(Q, v[i], G[i]) : gap_of(Q, il, v[i]);
                inc += (G[i] == 4096) ? 4096u : (uint32_t)G[i] + 1u;
                evc += (G[i] < 4096) ? 1u : 0u;
            }
            const uint64_t mine = ((uint64_t)evc << 40) | inc;
            uint64_t x = mine;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint64_t y = __shfl_up(x, off, 64);
                if ((int)lane >= off) x += y;
            }
            const uint64_t total = __shfl(x, 63, 64);
            const uint64_t ex = x - mine;
            // this lane's events (at most four): position, event index
            uint64_t p = pos + (ex & ((1ull << 40) - 1));
            uint64_t e = ev0 + (ex >> 40);
            uint64_t at[4], ee[4];
            bool has[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                at[i] = p + (uint64_t)G[i];
                ee[i] = e;
                has[i] = G[i] < 4096 && at[i] < end;
                if (G[i] < 4096) ++e;
                p += (G[i] == 4096) ? 4096u : (uint32_t)G[i] + 1u;
            }
            // The events' loads are issued together (channel descriptors, then branch masks), so a lane
            // with several events waits for one chain of dependent loads, not one per event.
            uint32_t chid[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) chid[i] = has[i] ? P.cls_chan[coff + (uint32_t)(at[i] >> 6)] : 0u;
            DevChan ch[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (has[i]) ch[i] = P.chan[chid[i]];
            uint32_t mask[4];
            uint4 br = make_uint4(0, 0, 0, 0);
            uint64_t brb = ~0ull;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                mask[i] = 0;
                if (!has[i]) continue;
                if ((ee[i] >> 2) != brb) {  // four consecutive events share a branch block
                    brb = ee[i] >> 2;
                    br = philox4x32_10(make_uint4((uint32_t)brb, wlo, c, (2u << 24) | whi), k0, k1);
                }
                const uint32_t q = (uint32_t)(ee[i] & 3);
                const uint32_t bv = q == 0 ? br.x : q == 1 ? br.y : q == 2 ? br.z : br.w;
                uint32_t j;
                if (ch[i].uniform) {
                    j = (uint32_t)(((uint64_t)bv * ch[i].J) >> 32);
                } else {
                    j = ch[i].J - 1;
                    for (uint32_t t = 0; t < ch[i].J; ++t)
                        if ((uint64_t)bv < P.thr[ch[i].thr_off + t]) { j = t; break; }
                }
                mask[i] = P.bmask[ch[i].bm_off + j];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t sl = (uint32_t)(at[i] & 63);
                uint32_t m = mask[i];
                while (m) {
                    const uint32_t sym = ch[i].sym0 + (uint32_t)__ffs(m) - 1u;
                    m &= m - 1u;
                    for (uint32_t q = P.sym_off[sym]; q < P.sym_off[sym + 1]; ++q)
                        atomicXor(&exo[P.sym_cons[q]], 1ull << sl);
                }
            }
            pos += total & ((1ull << 40) - 1);
            ev0 += total >> 40;
            blk0 += 64;
        }
    }
}

// Parity of the causal part of lambda for this lane's shot.
__device__ __forceinline__ int lane_parity(const DevProg &P, const DevInstr &I, const uint32_t *mb, uint32_t lane) {
    const __attribute__((address_space(4))) uint32_t *q =
        (const __attribute__((address_space(4))) uint32_t *)(P.cmeas + 2 * (size_t)I.cm_off);
    uint32_t x = 0;
    for (uint32_t j = 0; j < I.cm_len; ++j) x ^= mb[q[2 * j] * 64u + lane] & q[2 * j + 1];
    return __popc(x) & 1;
}

// v * i^q
template <typename V>
__device__ __forceinline__ V lane_iq(V v, int q) {
    V t;
    t.x = (q == 0) ? v.x : (q == 1) ? -v.y : (q == 2) ? -v.x : v.y;
    t.y = (q == 0) ? v.y : (q == 1) ? v.x : (q == 2) ? -v.y : -v.x;
    return t;
}

// LDS of the lane kernel (one wave): exogenous words, outcome bits, vectors.
__host__ __device__ inline size_t lane_vec_offset(uint32_t n_instr, uint32_t n_meas) {
    const size_t mw = (n_meas + 31) / 32;
    return ((size_t)8 * n_instr + (size_t)256 * mw + 15) & ~(size_t)15;
}

// CM: count mode (paper Sec. 6, detector postselection): each lane's shot is
// discarded once a postselected detector whose last record an instruction
// makes is 1; the wave leaves the instruction stream when every live shot of
// its word is discarded (a live-shot mask over the 64 lanes).  The word's two
// flag words and the totals are written instead of rows.
template <typename T, bool CM>
__device__ __forceinline__ void run_lane_words(const ActiveArgs &A, uint64_t wi_begin, uint64_t wi_end, uint64_t wi_step,
                                               unsigned char *smem) {
    using V = typename C2<T>::type;
    const DevProg &P = A.P;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t mw = (P.n_meas + 31) / 32;
    unsigned long long *exo = (unsigned long long *)smem;  // n_instr
    uint32_t *mb = (uint32_t *)(exo + P.n_instr);            // [mw][64]
    V *vec = (V *)(smem + lane_vec_offset(P.n_instr, P.n_meas));  // [vcap][64]
    const uint32_t k0 = (uint32_t)A.seed, k1 = (uint32_t)(A.seed >> 32);
    const T rs2 = (T)0.70710678118654752440;
    unsigned long long n_disc = 0, n_logic = 0;  // count mode: this wave's totals
    for (uint64_t wi = wi_begin; wi < wi_end; wi += wi_step) {
        const uint64_t w = A.word_begin + wi;
        const uint64_t shot = w * 64 + lane;
        const bool valid = shot - A.word_begin * 64 < A.shots;
        bool dead = false;
        for (uint32_t i = lane; i < P.n_instr; i += 64) exo[i] = 0;
        for (uint32_t j = 0; j < mw; ++j) mb[j * 64u + lane] = 0;
        {
            V one;
            one.x = (T)1;
            one.y = (T)0;
            vec[lane] = one;
        }
        lane_sync();
        word_noise_wave(P, A.seed, w, exo);
        for (uint32_t i = lane; i < P.n_rm; i += 64) {
            const uint32_t ii = P.rm_list[i];
            const uint32_t t = (uint32_t)P.instr[ii].meas;
            const uint4 o = philox4x32_10(make_uint4(t >> 1, (uint32_t)w, 0u, (3u << 24) | (uint32_t)(w >> 32)), k0, k1);
            exo[ii] = (t & 1) ? ((uint64_t)o.z | ((uint64_t)o.w << 32)) : ((uint64_t)o.x | ((uint64_t)o.y << 32));
        }
        lane_sync();
        const bool probe = shot - A.probe_shot0 < A.probe_n;
        for (uint32_t ii = 0; ii < P.n_instr; ++ii) {
            const DevInstr I = load_instr(P.instr, ii);
            const uint32_t N = 1u << I.k_in;
            V *vb = vec + (size_t)I.base * 64u;
            for (uint32_t q = 0; q < I.mg_len; ++q) {
                const DevMerge M = load_merge(P.merges, I.mg_off + q);
                const uint32_t NW = 1u << (M.m1w >> 24), m1 = M.m1w & 0xFFFFFFu, m2 = (NW - 1u) & ~m1;
                for (uint32_t x = 0; x < NW; ++x) {
                    const V u = vec[(size_t)(M.src1 + gather_bits(x, m1)) * 64u + lane];
                    const V v = vec[(size_t)(M.src2 + gather_bits(x, m2)) * 64u + lane];
                    V o;
                    o.x = u.x * v.x - u.y * v.y;
                    o.y = u.x * v.y + u.y * v.x;
                    vec[(size_t)(M.dst + x) * 64u + lane] = o;
                }
            }
            const int lam = (int)I.lam_c ^ (int)((exo[ii] >> lane) & 1ull) ^ lane_parity(P, I, mb, lane);
            const T c = sizeof(T) == 8 ? (T)I.c : (T)I.cf;
            const T s = sizeof(T) == 8 ? (T)I.s : (T)I.sf;
            switch (I.kind) {
            case 1: {  // PromoteRot: x <- c a_x, x + N <- -i (-1)^lam s a_x
                const T ss = lam ? -s : s;
                for (uint32_t x = 0; x < N; ++x) {
                    V v = vb[x * 64u + lane];
                    V hi;
                    hi.x = ss * v.y;
                    hi.y = -ss * v.x;
                    vb[(x + N) * 64u + lane] = hi;
                    v.x *= c;
                    v.y *= c;
                    vb[x * 64u + lane] = v;
                }
                break;
            }
            case 8: {  // PromoteRot starting a component of its own, from the amplitude 1
                const T ss = lam ? -s : s;
                V lo, hi;
                lo.x = c;
                lo.y = (T)0;
                hi.x = (T)0;
                hi.y = -ss;
                vb[lane] = lo;
                vb[64u + lane] = hi;
                break;
            }
            case 2: {  // ActiveDiagRot: a_x *= c - i sigma s, sigma = (-1)^lam mu (-1)^(b.x)
                const int neg = lam ^ (I.mu == 2 ? 1 : 0);
                for (uint32_t x = 0; x < N; ++x) {
                    const T sg = (neg ^ parity(I.b & x)) ? -s : s;
                    const V v = vb[x * 64u + lane];
                    V o;
                    o.x = c * v.x + sg * v.y;
                    o.y = c * v.y - sg * v.x;
                    vb[x * 64u + lane] = o;
                }
                break;
            }
            case 3: {  // ActivePairRot on pairs (x0, x0 ^ a), bit h of x0 = 0
                const int e0 = (int)I.mu + 3 + 2 * lam;
                for (uint32_t z = 0; z < (N >> 1); ++z) {
                    const uint32_t x0 = insert_bit(z, I.h, 0), x1 = x0 ^ I.a;
                    V a0 = vb[x0 * 64u + lane], a1 = vb[x1 * 64u + lane];
                    pair_update(a0, a1, x0, x1, e0, I.b, c, s);
                    vb[x0 * 64u + lane] = a0;
                    vb[x1 * 64u + lane] = a1;
                }
                break;
            }
            case 4: {  // RandomMeas
                const uint32_t t = (uint32_t)I.meas;
                mb[(t >> 5) * 64u + lane] |= (uint32_t)((exo[ii] >> lane) & 1ull) << (t & 31);
                if (A.p0_out && probe) A.p0_out[(shot - A.probe_shot0) * P.n_meas + t] = 0.5;
                break;
            }
            case 5: {  // DetMeas: m = lambda ^ eta
                const uint32_t t = (uint32_t)I.meas;
                mb[(t >> 5) * 64u + lane] |= (uint32_t)(lam ^ I.eta) << (t & 31);
                if (A.p0_out && probe) A.p0_out[(shot - A.probe_shot0) * P.n_meas + t] = (lam ^ I.eta) ? 0.0 : 1.0;
                break;
            }
            case 6:    // ActiveDiagMeas
            case 7: {  // ActivePairMeas
                const bool pair = I.kind == 7;
                const uint32_t t = (uint32_t)I.meas, half = N >> 1;
                const uint4 od = philox4x32_10(make_uint4(t, (uint32_t)shot, (uint32_t)(shot >> 32), 4u << 24), k0, k1);
                const int mc = (4 - (int)I.mu) & 3;  // conj(mu) = i^mc
                T s0 = 0, s1 = 0, c0 = 0, c1 = 0;
                if (!pair) {
                    for (uint32_t x = 0; x < N; ++x) {
                        const V v = vb[x * 64u + lane];
                        const T m2 = v.x * v.x + v.y * v.y;
                        if (parity(I.b & x)) kahan_add(s1, c1, m2); else kahan_add(s0, c0, m2);
                    }
                } else {
                    for (uint32_t z = 0; z < half; ++z) {
                        const uint32_t u0 = insert_bit(z, I.h, 0);
                        const V a0 = vb[u0 * 64u + lane];
                        const V tt = lane_iq(vb[(u0 ^ I.a) * 64u + lane], (mc + 2 * parity(I.b & u0)) & 3);
                        const T bx = (a0.x + tt.x) * rs2, by = (a0.y + tt.y) * rs2;
                        const T dx = (a0.x - tt.x) * rs2, dy = (a0.y - tt.y) * rs2;
                        kahan_add(s0, c0, bx * bx + by * by);
                        kahan_add(s1, c1, dx * dx + dy * dy);
                    }
                }
                const int flip = pair ? lam : (lam ^ (int)I.eta);
                const double S0 = (double)s0, S1 = (double)s1;
                const double p0 = (flip ? S1 : S0) / (S0 + S1);
                const double u = (double)(((uint64_t)od.x << 21) + (uint64_t)(od.y >> 11)) * 0x1p-53;
                const int m = (u < p0) ? 0 : 1;
                const int y = m ^ flip;  // kept class
                const double Sy = y ? S1 : S0;
                const T scale = (T)(1.0 / sqrt(Sy > 0x1p-1000 ? Sy : 0x1p-1000));
                mb[(t >> 5) * 64u + lane] |= (uint32_t)m << (t & 31);
                if (A.p0_out && probe) A.p0_out[(shot - A.probe_shot0) * P.n_meas + t] = p0;
                // compaction 2^k -> 2^(k-1) in place: output z's sources lie at indices >= z,
                // so increasing z never overwrites a source still to be read
                const uint32_t bl = I.b & ~(1u << I.h);
                for (uint32_t z = 0; z < half; ++z) {
                    V o;
                    if (!pair) {
                        const uint32_t uu = insert_bit(z, I.h, (uint32_t)y);
                        const uint32_t x = uu ^ ((uint32_t)parity(bl & uu) << I.h);
                        const V v = vb[x * 64u + lane];
                        o.x = v.x * scale;
                        o.y = v.y * scale;
                    } else {
                        const uint32_t u0 = insert_bit(z, I.h, 0);
                        const V a0 = vb[u0 * 64u + lane];
                        const V tt = lane_iq(vb[(u0 ^ I.a) * 64u + lane], (mc + 2 * parity(I.b & u0) + 2 * y) & 3);
                        o.x = (a0.x + tt.x) * rs2 * scale;
                        o.y = (a0.y + tt.y) * rs2 * scale;
                    }
                    vb[z * 64u + lane] = o;
                }
                break;
            }
            default: break;
            }
            if (CM) {
                // postselected detectors whose last record this instruction made (scalar offsets)
                const __attribute__((address_space(4))) uint32_t *co =
                    (const __attribute__((address_space(4))) uint32_t *)A.cnt.chk_off;
                const uint32_t c0 = co[ii], c1 = co[ii + 1];
                if (c0 < c1) {
                    uint32_t fired = 0;
                    for (uint32_t q = c0; q < c1; ++q) {
                        uint32_t x = 0;
                        for (uint32_t e = A.cnt.chk_mo[q]; e < A.cnt.chk_mo[q + 1]; ++e) {
                            const uint32_t t = A.cnt.chk_meas[e];
                            x ^= (mb[(t >> 5) * 64u + lane] >> (t & 31)) & 1u;
                        }
                        fired |= x;
                    }
                    dead = dead || fired != 0;
                    if (__ballot(valid && !dead) == 0) break;  // every shot of the word discarded
                }
            }
        }
        if (A.amp_out && probe) {
            double *dst = A.amp_out + (shot - A.probe_shot0) * (2ull << A.amp_k);
            for (uint32_t x = 0; x < (1u << A.amp_k); ++x) {
                const V v = vec[x * 64u + lane];
                dst[2 * x] = (double)v.x;
                dst[2 * x + 1] = (double)v.y;
            }
        }
        const uint64_t col = wi;
        if (CM) {
            // the word's flags: discarded; kept with an observable off its expected value
            uint32_t le = 0;
            for (uint32_t b = 0; b < P.n_obs; ++b) {
                uint32_t x = (A.cnt.obs_exp[b >> 5] >> (b & 31)) & 1u;
                for (uint32_t q = P.obs_off[b]; q < P.obs_off[b + 1]; ++q) {
                    const uint32_t t = P.rec_meas[P.obs_rows[q]];
                    x ^= (mb[(t >> 5) * 64u + lane] >> (t & 31)) & 1u;
                }
                le |= x;
            }
            const uint64_t d = __ballot(valid && dead), l = __ballot(valid && !dead && le != 0);
            if (lane == 0) {
                if (A.cnt.flags) {
                    A.cnt.flags[col] = d;
                    A.cnt.flags[A.n_words + col] = l;
                }
                n_disc += (unsigned long long)__popcll(d);
                n_logic += (unsigned long long)__popcll(l);
            }
            lane_sync();
            continue;
        }
        // rows: one ballot per row over the word's shots (bits past the call's shots are 0)
        auto rec_bit = [&](uint32_t row) -> uint32_t {
            const uint32_t t = P.rec_meas[row];
            return (mb[(t >> 5) * 64u + lane] >> (t & 31)) & 1u;
        };
        if (A.sections & 1u)
            for (uint32_t row = 0; row < P.n_rec; ++row) {
                const uint64_t v = __ballot(valid && rec_bit(row));
                if (lane == 0) A.out[(uint64_t)row * A.row_stride + col] = v;
            }
        if (A.sections & 2u)
            for (uint32_t d = 0; d < P.n_det; ++d) {
                uint32_t x = 0;
                for (uint32_t q = P.det_off[d]; q < P.det_off[d + 1]; ++q) x ^= rec_bit(P.det_rows[q]);
                const uint64_t v = __ballot(valid && x);
                if (lane == 0) A.out[(uint64_t)(P.n_rec + d) * A.row_stride + col] = v;
            }
        if (A.sections & 4u)
            for (uint32_t b = 0; b < P.n_obs; ++b) {
                uint32_t x = 0;
                for (uint32_t q = P.obs_off[b]; q < P.obs_off[b + 1]; ++q) x ^= rec_bit(P.obs_rows[q]);
                const uint64_t v = __ballot(valid && x);
                if (lane == 0) A.out[(uint64_t)(P.n_rec + P.n_det + b) * A.row_stride + col] = v;
            }
        lane_sync();
    }
    if (CM && A.cnt.counts && lane == 0) {
        if (n_disc) atomicAdd(&A.cnt.counts[0], n_disc);
        if (n_logic) atomicAdd(&A.cnt.counts[1], n_logic);
    }
}

template <typename T, bool CM>
__global__ void __launch_bounds__(64) lane_kernel(ActiveArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    run_lane_words<T, CM>(A, blockIdx.x, A.n_words, gridDim.x, smem);
}

// The lane kernel behind a persistent queue of (program, word range) items:
// each one-wave workgroup takes the next item with a global atomic until the
// list is exhausted.
template <typename T, bool CM>
__global__ void __launch_bounds__(64) lane_batch_kernel(BatchArgs B) {
    extern __shared__ __align__(16) unsigned char smem[];
    while (true) {
        uint32_t idx = 0;
        if ((threadIdx.x & 63u) == 0) idx = atomicAdd(B.counter, 1u);
        // a wave-uniform index: the item and its argument block come by scalar loads
        idx = __builtin_amdgcn_readfirstlane((uint32_t)__shfl((int)idx, 0, 64));
        if (idx >= B.n_items) break;
        const BatchItem it = B.items[idx];
        run_lane_words<T, CM>(B.calls[it.call], it.w0, it.w1, 1, smem);
    }
}

// Persistent work queue over (program, word range) items: every workgroup
// takes the next item index with a global atomic until the list is exhausted,
// so every wave reaches the exit.  Items are ordered by decreasing cost.
template <typename T, int BS, bool CM>
__global__ void __launch_bounds__(BS) batch_kernel(BatchArgs B) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_idx;
    while (true) {
        if (threadIdx.x == 0) s_idx = atomicAdd(B.counter, 1u);
        __syncthreads();
        const uint32_t idx = __builtin_amdgcn_readfirstlane(s_idx);
        __syncthreads();
        if (idx >= B.n_items) break;
        const BatchItem it = B.items[idx];
        run_active_words<T, BS, true, CM>(B.calls[it.call], it.w0, it.w1, 1, blockIdx.x, smem);
    }
}

__global__ void reset_counter_kernel(uint32_t *counter) { counter[threadIdx.x] = 0u; }

// Aggregate counts from full rows (the count path that writes detector and
// observable rows first): per 64-shot word, discarded = OR of the postselected
// detectors, logical error = OR of (observable XOR expected) on kept shots.
// One thread per word; one atomic add per wave and counter.
__global__ void flags_from_rows_kernel(const uint64_t *rows, uint64_t n_words, uint64_t shots, uint64_t n_rec,
                                       uint32_t n_det, uint32_t n_obs, CountArgs C, uint64_t flag_off,
                                       uint64_t flag_stride) {
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long d = 0, l = 0;
    if (w < n_words) {
        for (uint32_t k = 0; k < n_det; ++k)
            if ((C.post[k >> 5] >> (k & 31u)) & 1u) d |= rows[(n_rec + k) * n_words + w];
        for (uint32_t o = 0; o < n_obs; ++o) {
            const unsigned long long x = ((C.obs_exp[o >> 5] >> (o & 31u)) & 1u) ? ~0ull : 0ull;
            l |= rows[(n_rec + n_det + o) * n_words + w] ^ x;
        }
        const uint64_t s0 = w * 64;
        const unsigned long long m = s0 + 64 <= shots ? ~0ull : ((1ull << (shots - s0)) - 1ull);
        d &= m;
        l &= ~d & m;
        if (C.flags) {
            C.flags[flag_off + w] = d;
            C.flags[flag_stride + flag_off + w] = l;
        }
    }
    unsigned long long nd = (unsigned long long)__popcll(d), nl = (unsigned long long)__popcll(l);
    for (int off = 32; off > 0; off >>= 1) {
        nd += __shfl_xor(nd, off, 64);
        nl += __shfl_xor(nl, off, 64);
    }
    if ((threadIdx.x & 63u) == 0 && C.counts) {
        if (nd) atomicAdd(&C.counts[0], nd);
        if (nl) atomicAdd(&C.counts[1], nl);
    }
}

// rows: n_rec + n_det + n_obs rows of n_words words (only rows from n_rec on
// are read); flags row 0 at flags[flag_off ..], row 1 at flags[flag_stride + flag_off ..].
hipError_t launch_flags_from_rows(const uint64_t *rows, uint64_t n_words, uint64_t shots, uint64_t n_rec,
                                  uint32_t n_det, uint32_t n_obs, const CountArgs &C, uint64_t flag_off,
                                  uint64_t flag_stride, hipStream_t st) {
    if (n_words == 0) return hipSuccess;
    hipLaunchKernelGGL(flags_from_rows_kernel, dim3((uint32_t)((n_words + 255) / 256)), dim3(256), 0, st, rows,
                       n_words, shots, n_rec, n_det, n_obs, C, flag_off, flag_stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------- host ----
template <typename T, int BS, bool LDSV, bool CM>
static hipError_t launch_one(const ActiveArgs &A, uint32_t grid, hipStream_t st) {
    auto kfn = active_kernel<T, BS, LDSV, CM>;
    hipError_t e = hipFuncSetAttribute((const void *)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)A.lds_bytes);
    if (e != hipSuccess) return e;
    if (A.unit_counter) hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, A.unit_counter);
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(BS), A.lds_bytes, st, A);
    return hipGetLastError();
}

size_t active_lds_bytes(const DevProg &P, uint32_t bs, uint32_t tps, bool lds_vec, bool fp64) {
    const uint32_t G = bs / tps;
    const uint32_t mw = (P.n_meas + 31) / 32;
    size_t b = 8ull * P.n_instr + 8ull * P.n_rec + 8 * 44 + (fp64 ? 8 : 4) * (2 * (bs / 64) + 2) + 4ull * G * mw;
    b = (b + 15) & ~(size_t)15;
    if (lds_vec) b += (size_t)G * ((size_t)1 << P.k_max) * (fp64 ? 16 : 8);
    return b;
}

template <typename T, int BS, bool LDSV, bool CM>
static int blocks_per_cu(size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, active_kernel<T, BS, LDSV, CM>, BS, lds) != hipSuccess) return 1;
    return nb;
}

// The instantiation for (precision, block size, vector residency, count mode).
template <template <typename, int, bool, bool> class F, typename... Args>
static auto dispatch(bool fp64, uint32_t bs, bool lds_vec, bool cm, Args... args) {
#define SYMFT_PICK(T, B)                                                                             \
    return lds_vec ? (cm ? F<T, B, true, true>::run(args...) : F<T, B, true, false>::run(args...))  \
                   : (cm ? F<T, B, false, true>::run(args...) : F<T, B, false, false>::run(args...))
    // one-group workgroups of 64 or 128 threads exist in count mode only
#define SYMFT_PICK_CM(T, B) \
    return lds_vec ? F<T, B, true, true>::run(args...) : F<T, B, false, true>::run(args...)
    if (fp64) {
        if (bs == 1024) SYMFT_PICK(double, 1024);
        if (cm && bs == 128) SYMFT_PICK_CM(double, 128);
        if (cm && bs == 64) SYMFT_PICK_CM(double, 64);
        SYMFT_PICK(double, 256);
    }
    if (bs == 1024) SYMFT_PICK(float, 1024);
    if (cm && bs == 128) SYMFT_PICK_CM(float, 128);
    if (cm && bs == 64) SYMFT_PICK_CM(float, 64);
    SYMFT_PICK(float, 256);
#undef SYMFT_PICK
#undef SYMFT_PICK_CM
}

template <typename T, int BS, bool LDSV, bool CM>
struct LaunchOne {
    static hipError_t run(const ActiveArgs &A, uint32_t grid, hipStream_t st) { return launch_one<T, BS, LDSV, CM>(A, grid, st); }
};
template <typename T, int BS, bool LDSV, bool CM>
struct BlocksPerCu {
    static int run(size_t lds) { return blocks_per_cu<T, BS, LDSV, CM>(lds); }
};

int active_max_blocks_per_cu(bool fp64, uint32_t bs, bool lds_vec, size_t lds, bool cm) {
    return dispatch<BlocksPerCu>(fp64, bs, lds_vec, cm, lds);
}

template <typename T, bool CM>
static hipError_t launch_batch_t(const BatchArgs &B, uint32_t grid, uint32_t lds, hipStream_t st) {
    auto kfn = batch_kernel<T, 256, CM>;
    hipError_t e = hipFuncSetAttribute((const void *)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, B.counter);
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(256), lds, st, B);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs &B, bool fp64, bool cm, uint32_t grid, uint32_t lds, hipStream_t st) {
    if (cm) return fp64 ? launch_batch_t<double, true>(B, grid, lds, st) : launch_batch_t<float, true>(B, grid, lds, st);
    return fp64 ? launch_batch_t<double, false>(B, grid, lds, st) : launch_batch_t<float, false>(B, grid, lds, st);
}

int batch_max_blocks_per_cu(bool fp64, bool cm, size_t lds) {
    int nb = 0;
    const void *k = cm ? (fp64 ? (const void *)batch_kernel<double, 256, true> : (const void *)batch_kernel<float, 256, true>)
                       : (fp64 ? (const void *)batch_kernel<double, 256, false> : (const void *)batch_kernel<float, 256, false>);
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, lds);
    return e == hipSuccess ? nb : 1;
}

hipError_t launch_active(const ActiveArgs &A, bool fp64, uint32_t bs, uint32_t grid, hipStream_t st) {
    return dispatch<LaunchOne>(fp64, bs, A.lds_vec != 0, A.cnt.on != 0, A, grid, st);
}


// The lane kernel: LDS bytes per wave (= per workgroup), the batch queue's occupancy, and launch.
size_t lane_lds_bytes(const DevProg &P, bool fp64) {
    return lane_vec_offset(P.n_instr, P.n_meas) + (size_t)64 * P.vcap * (fp64 ? 16 : 8);
}

static const void *lane_batch_kfn(bool fp64, bool cm) {
    if (fp64) return cm ? (const void *)lane_batch_kernel<double, true> : (const void *)lane_batch_kernel<double, false>;
    return cm ? (const void *)lane_batch_kernel<float, true> : (const void *)lane_batch_kernel<float, false>;
}

int lane_batch_max_blocks_per_cu(bool fp64, size_t lds, bool cm) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lane_batch_kfn(fp64, cm), 64, lds) != hipSuccess) return 1;
    return nb;
}

template <typename T, bool CM>
static hipError_t launch_lane_batch_t(const BatchArgs &B, uint32_t grid, uint32_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)lane_batch_kernel<T, CM>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, B.counter);
    hipLaunchKernelGGL((lane_batch_kernel<T, CM>), dim3(grid), dim3(64), lds, st, B);
    return hipGetLastError();
}

hipError_t launch_lane_batch(const BatchArgs &B, bool fp64, bool cm, uint32_t grid, uint32_t lds, hipStream_t st) {
    if (cm) return fp64 ? launch_lane_batch_t<double, true>(B, grid, lds, st) : launch_lane_batch_t<float, true>(B, grid, lds, st);
    return fp64 ? launch_lane_batch_t<double, false>(B, grid, lds, st) : launch_lane_batch_t<float, false>(B, grid, lds, st);
}

template <typename T, bool CM>
static hipError_t launch_lane_t(const ActiveArgs &A, uint32_t grid, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)lane_kernel<T, CM>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)A.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((lane_kernel<T, CM>), dim3(grid), dim3(64), A.lds_bytes, st, A);
    return hipGetLastError();
}

hipError_t launch_lane(const ActiveArgs &A, bool fp64, uint32_t grid, hipStream_t st) {
    const bool cm = A.cnt.on != 0;
    if (cm) return fp64 ? launch_lane_t<double, true>(A, grid, st) : launch_lane_t<float, true>(A, grid, st);
    return fp64 ? launch_lane_t<double, false>(A, grid, st) : launch_lane_t<float, false>(A, grid, st);
}

}  // namespace symft
