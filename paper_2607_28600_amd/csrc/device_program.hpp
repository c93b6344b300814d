// device_program.hpp -- the sampling program as laid out in device memory.
// Shared by the host lowering (capi.cpp) and the HIP kernels.
#pragma once

#include <cstdint>

namespace symft {

// One sampling instruction (56 bytes).  cos/sin(theta/2) are computed once on
// the host in FP64; the FP32 copies are rounded from them, so the kernels
// evaluate no transcendental function.
struct DevInstr {
    uint8_t kind, k_in, h, mu;     // mu: power of i
    uint8_t eta, lam_c;
    uint8_t fuse;                  // rotations: instructions that follow at the same width and run in the
                                   // same pass over the vector: 1 a PromoteRot; 2 a pair rotation (after a
                                   // pair rotation with another mask); 3 a pair rotation, then a PromoteRot
                                   // (2 and 3 with FP32 vectors in HBM scratch and a coset per thread
                                   // only; otherwise such a pair rotation runs alone, and the middle one
                                   // of 3 carries mark 1)
    uint8_t mg_len;                // product-component programs: Kronecker merges run before it
    uint32_t a, b;
    int32_t meas;                  // measurement index (measurements)
    uint32_t cm_off, cm_len;       // causal refs of lambda: cm_len (word, mask) pairs from pair cm_off
    uint32_t am_idx;               // active measurements: ordinal among them in stream order
    double c, s;
    float cf, sf;
    uint32_t base;                 // region of the shot's vector buffer it runs on (0 for dense programs)
    uint32_t mg_off;               // its first merge in DevProg::merges
};
static_assert(sizeof(DevInstr) == 64, "DevInstr layout");

// A Kronecker merge of two components (paper Sec. 6): for x < 2^w,
// dst[x] = src1[x1] * src2[x2], where x1 gathers the bits of x at the set bits
// of m1 and x2 those at the others, each in increasing order (offsets in
// amplitudes of the shot's vector buffer; the three regions do not overlap).
struct DevMerge {
    uint32_t dst, src1, src2;
    uint32_t m1w;  // m1 in bits 0..23, w in bits 24..31
};
static_assert(sizeof(DevMerge) == 16, "DevMerge layout");

// Noise channel under the draw contract.
struct DevChan {
    uint8_t J, uniform, nsym, pad;
    uint32_t sym0;     // first noise symbol
    uint32_t bm_off;   // J branch masks in bmask[]
    uint32_t thr_off;  // J thresholds in thr[] (non-uniform only)
};

// Per-class constants of the table-free gap decision.  With q = 1 - P32/2^32
// and R[g] = 2^32 q^g, the integer table obeys R[g] - D < Q[g] <= R[g] with
// D = 2^32 / P32 (each floor loses less than one, shrunk by q at every later
// step).  For v >= Q[4096] let t = log2(v / 2^32) / log2(q); then v < R[g]
// exactly when g < t, so v >= R[floor(t) + 1] >= Q[floor(t) + 1], and
// v < Q[floor(t)] is guaranteed once v + D < R[floor(t)], i.e. once
// frac(t) > log2(1 + D/v) / |log2 q|, which frac(t) >= A / v with
// A >= D / (ln 2 |log2 q|) implies.  Then G = floor(t).  eps bounds the FP32
// error of t; draws outside these margins take the exact table search.
// Near a boundary the computed t is still within one of the exact one, and
// G >= floor(t) - 1 once v (1 - q) / q > D (the step from R[floor(t) - 1] down
// to v exceeds the table's rounding loss), so then G = g0 - 2 + #{k in g0 - 1
// .. g0 + 1 : v < Q[k]} with g0 = floor(t computed): three independent table
// reads decide the draws the margins leave (vwin: the least v for which this
// holds; UINT32_MAX when the error bound does not allow it).
struct GapFast {
    float invlog2q;   // 1 / log2(q)
    float A;          // margin numerator (inflated)
    float eps;        // bound on |t computed - t|
    uint32_t vwin;    // three-read window decision for v >= vwin
    uint64_t qW;      // Q[4096]: v < qW means G = 4096
    uint64_t vmin;    // fast path only for v >= vmin (1, or never when P32 = 2^32)
};
static_assert(sizeof(GapFast) == 32, "GapFast layout");

// Pointers into one device allocation (all read-only in the kernels).
struct DevProg {
    const DevInstr *instr;
    const DevMerge *merges;      // product-component programs: merges before instructions
    const uint32_t *cmeas;       // causal refs of each lambda: (outcome word, bit mask) pairs
    const uint32_t *am_meas;     // measurement id of every active measurement, in stream order
    const uint32_t *rm_list;     // instructions that are RandomMeas
    const uint32_t *rec_meas;    // record row -> measurement id
    const uint32_t *det_off;     // n_det + 1
    const uint32_t *det_rows;    // record rows per detector
    const uint32_t *obs_off;     // n_obs + 1
    const uint32_t *obs_rows;    // record rows per observable (XOR)
    const uint64_t *cls_Q;       // n_cls x 4097
    const uint32_t *cls_off;     // n_cls + 1 into cls_chan
    const uint32_t *cls_chan;    // channel ids by rank
    const DevChan *chan;
    const uint32_t *bmask;
    const uint64_t *thr;
    const uint32_t *sym_off;     // n_sym + 1 into sym_cons
    const uint32_t *sym_cons;    // consumer instruction ids per noise symbol
    const float *cls_invlog2q;   // per class 1 / log2(1 - P32 / 2^32): initial guess of a geometric gap
    const GapFast *cls_fast;     // per class: table-free gap decision margins
    // pure-frame schedule (k_max == 0 programs), see sample_frame.hip
    const uint32_t *fr_step;     // 8 words per step (launch_args.hpp)
    const uint32_t *fr_nodes;    // 8 words per node: slot | flags << 24, row, meas, push count, two successor slots, push offset, 0
    const uint32_t *fr_push;     // successor slots
    const uint32_t *fr_nodes16;  // 4 words per node: slot | flags << 12 | push count << 20, row,
                                 // successor slots s0 | s1 << 12, offset into fr_push16
    const uint32_t *fr_push16;   // per node: its measurement if RandomMeas, then successor slots past two
    const uint64_t *fr_chinfo;   // per (class, rank): flip-table offset | J << 26 | uniform << 32 | step << 33 | thr_off << 41
    const uint64_t *fr_frec;     // per (channel, branch): flip record of two entries (16 bytes, 16-byte aligned)
    const uint64_t *fr_fl3;      // flip entries past a record's two, from an even index (16-byte aligned)
    const uint32_t *fr_ci32;     // per (class, rank): flip-table offset | J << 20 (for the LDS copy)
    const uint8_t *fr_st8;       // per (class, rank): NOISE step index within the class
    const uint32_t *cls_Q32;     // n_cls x 4097: Q[g] as 32 bits (Q[0] = 2^32 stored as 2^32 - 1; walks decide g = 0 without it)
    const uint32_t *fr_cap;      // per class: flip entries kept per (word, class)
    const uint32_t *fr_capoff;   // per class + 1: prefix of fr_cap
    // wave-owned pure-frame schedule (sample_frame_wave.hip, launch_args.hpp)
    const uint32_t *wv_ops;      // ops of 8 words
    const uint32_t *wv_rows;     // output row of every staged position
    const uint64_t *wv_fl;       // per (channel, branch): slot flips (inline up to three, else a list)
    const uint16_t *wv_sl;       // slot lists
    const uint32_t *wv_rm;       // measurement of every RandomMeas node
    const uint32_t *wv_cap;      // per class: slot flips kept per word
    const uint32_t *wv_capoff;   // per class + 1: prefix of wv_cap
    uint32_t n_instr, n_meas, n_rm, n_rec, n_det, n_obs, n_cls, k_max;
    uint32_t fr_n_steps, fr_n_slots, n_sym, fr_ok;   // fr_ok: the pure-frame kernel can run the program
    uint32_t fr_first_emit, fr_first_emit_n, fr_first_noise_cls, n_am;
    uint32_t wv_n_ops, wv_n_rm, wv_first_noise_cls, wv_first_batch, wv_first_batch_n, wv_ok;
    uint32_t vcap, vcap_pad;     // amplitudes per shot the instruction stream touches (<= 2^k_max)
    uint32_t fr_n_cch;           // entries of fr_ci32 / fr_st8: channels over all classes, padded to a multiple of 16
    uint32_t fr_ltab;            // nonzero: phase G copies fr_ci32, fr_st8 and cls_Q32 into LDS
    uint32_t fr_rec_ok;          // nonzero: slots below 2^12, as the step-synchronous kernel's entries need
};

}  // namespace symft
