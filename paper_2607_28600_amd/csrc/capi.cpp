// capi.cpp -- the C ABI: compile, introspection, device upload and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/symft.h"
#include "device_program.hpp"
#include "program.hpp"

namespace symft {
struct ActiveArgs;
hipError_t launch_active(const ActiveArgs &A, bool fp64, uint32_t bs, uint32_t grid, hipStream_t st);
size_t active_lds_bytes(const DevProg &P, uint32_t bs, uint32_t tps, bool lds_vec, bool fp64);
int active_max_blocks_per_cu(bool fp64, uint32_t bs, bool lds_vec, size_t lds, bool cm);
size_t lane_lds_bytes(const DevProg &P, bool fp64);
hipError_t launch_lane(const ActiveArgs &A, bool fp64, uint32_t grid, hipStream_t st);
int lane_batch_max_blocks_per_cu(bool fp64, size_t lds, bool cm);
struct FrameArgs;
struct CountArgs;
hipError_t launch_frame(const FrameArgs &A, uint32_t grid, hipStream_t st, uint32_t tw);
struct BatchArgs;
hipError_t launch_batch(const BatchArgs &B, bool fp64, bool cm, uint32_t grid, uint32_t lds, hipStream_t st);
hipError_t launch_lane_batch(const BatchArgs &B, bool fp64, bool cm, uint32_t grid, uint32_t lds, hipStream_t st);
int batch_max_blocks_per_cu(bool fp64, bool cm, size_t lds);
size_t frame_lds_bytes(const DevProg &P, uint32_t tw);
hipError_t launch_flags_from_rows(const uint64_t *rows, uint64_t n_words, uint64_t shots, uint64_t n_rec,
                                  uint32_t n_det, uint32_t n_obs, const CountArgs &C, uint64_t flag_off,
                                  uint64_t flag_stride, hipStream_t st);
size_t frame_scratch_words(uint32_t word_entries, uint32_t tw);
struct WaveArgs;
hipError_t launch_frame_wave(const WaveArgs &A, uint32_t grid, hipStream_t st);
size_t frame_wave_lds_bytes(const DevProg &P);
int frame_wave_max_blocks_per_cu(size_t lds, bool cm);
int frame_max_blocks_per_cu(size_t lds, uint32_t tw);
hipError_t launch_gap_check(const GapFast &F, const uint64_t *Q, const uint32_t *v, int32_t *g, uint64_t n,
                            hipStream_t st);
}  // namespace symft

#include "launch_args.hpp"

using namespace symft;

static const size_t kLdsLimit = 160 * 1024;  // LDS of one gfx950 CU

// Margins of the table-free gap decision for one probability class (the
// derivation is with GapFast).  The FP32 error of t = log2(v / 2^32) / log2 q
// is bounded from: rounding v to float (2^-24 relative), the hardware log2
// (taken as 2^-21 |log2 x| + 2^-22 absolute, several ulp, with |log2 x| at
// most log2(2^32 / Q[4096]) since smaller draws never reach it), and rounding
// of 1 / log2 q and of the product (2^-24 relative each, t < 4097); eps
// doubles that sum.
static GapFast gap_fast_constants(uint64_t p32, const uint64_t *Q) {
    GapFast f;
    std::memset(&f, 0, sizeof(f));
    f.qW = Q[4096];
    f.vwin = UINT32_MAX;
    if (p32 == 0 || p32 >= (uint64_t(1) << 32)) {
        f.invlog2q = -0.0f;
        f.vmin = UINT64_MAX;  // P32 = 0: every draw is below Q[4096]; P32 = 2^32: table only
        return f;
    }
    const double q = 1.0 - std::ldexp((double)p32, -32);
    const double l = -std::log2(q);  // |log2 q|
    const double D = std::ldexp(1.0, 32) / (double)p32;
    // |log2 x| over the fast path's draws: x = v / 2^32 with v >= max(Q[4096], 1)
    const double Lmax = 32.0 - std::log2((double)std::max<uint64_t>(Q[4096], 1)) + 1e-6;
    const double err_log = std::ldexp(1.0, -24) / std::log(2.0) + std::ldexp(1.0, -21) * Lmax + std::ldexp(1.0, -22);
    const double err_t = err_log / l * (1.0 + std::ldexp(1.0, -20)) + 4097.0 * std::ldexp(1.0, -23);
    f.invlog2q = (float)(-1.0 / l);
    f.A = (float)(1.25 * D / (std::log(2.0) * l));
    f.eps = (float)(2.0 * err_t);
    f.vmin = 1;
    if (err_t < 0.5) {
        // G >= floor(t) - 1 needs v (2^32 - P32) / P32 > D; the error bound needs v >= max(Q[4096], 1)
        const double vw = std::ceil(D * (std::ldexp(1.0, 32) - (double)p32) / (double)p32) + 2.0;
        const double lo = std::max<double>(vw, (double)std::max<uint64_t>(Q[4096], 1));
        if (lo < 4294967295.0) f.vwin = (uint32_t)lo;
    }
    return f;
}

static thread_local std::string g_err;

static symft_status set_err(symft_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

static symft_status hip_err(const char *what, hipError_t e) {
    return set_err(SYMFT_EHIP, std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

struct HostLayout {
    std::vector<uint8_t> blob;
    // offsets of each array inside blob
    size_t o_instr, o_cmeas, o_am, o_rm, o_recmeas, o_detoff, o_detrows, o_obsoff, o_obsrows, o_clsQ, o_clsoff, o_clschan,
        o_chan, o_bmask, o_thr, o_symoff, o_symcons, o_invlog, o_clsfast, o_frstep, o_frnodes, o_frpush, o_frnodes16, o_frpush16, o_frchinfo,
        o_frrec, o_frfl3, o_frcap, o_frcapoff, o_wvops, o_wvrows, o_wvfl, o_wvsl, o_wvrm, o_wvcap, o_wvcapoff, o_ci32, o_st8, o_q32,
        o_pinstr, o_merge;
    uint32_t word_entries = 0;  // flip entries per word over all classes (frame kernel scratch)
    uint32_t wv_word_entries = 0;  // slot flips per word over all classes (wave kernel scratch)
    DevProg meta;  // counts only; pointers filled at upload
};

struct symft_program;
// Batch plans cache device argument blocks that point into a program's device
// blob; freeing the program must release every plan that holds it.
static void drop_batch_plans(const symft_program *p);
// Programs are told apart by a serial number, never by their address, which
// the allocator may hand to a later program.
static std::atomic<uint64_t> g_prog_serial{1};

struct symft_program {
    const uint64_t serial = g_prog_serial.fetch_add(1);
    Program P;
    HostLayout L;
    FrameSchedule F;
    ProductPlan PP;
    uint32_t comp_mode = 0;  // symft_compile_opts.components
    bool product = false;    // sampling runs the product-component stream
    uint32_t k_eff = 0;      // its vector buffer holds 2^k_eff amplitudes per shot
    std::mutex mu;
    std::map<int, void *> dev;  // device id -> uploaded blob
    // aggregate-count tables (postselection bits, expected observables, check lists) by (device, content)
    std::map<std::pair<int, std::vector<uint32_t>>, void *> count_dev;
    // count-mode threads per shot chosen by symft_autotune_counts, by (tables, FP64)
    std::map<std::pair<std::vector<uint32_t>, bool>, uint32_t> count_tune;
    ~symft_program() {
        drop_batch_plans(this);
        auto drop = [](int d, void *ptr) {
            // a destructor has no caller to report to: failures here are ignored
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(d);
            (void)hipFree(ptr);
            (void)hipSetDevice(cur);
        };
        for (auto &kv : dev) drop(kv.first, kv.second);
        for (auto &kv : count_dev) drop(kv.first.first, kv.second);
    }
};

template <typename T>
static size_t put(std::vector<uint8_t> &blob, const std::vector<T> &v) {
    size_t off = (blob.size() + 15) & ~(size_t)15;
    blob.resize(off + std::max<size_t>(v.size() * sizeof(T), 16), 0);
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

static void lower(symft_program *h) {
    const Program &P = h->P;
    HostLayout &L = h->L;
    std::vector<DevInstr> ins(P.instrs.size());
    std::vector<uint32_t> cmeas, rm, am;
    std::vector<std::vector<uint32_t>> cons(P.n_noise_sym);
    for (size_t i = 0; i < P.instrs.size(); ++i) {
        const Instr &I = P.instrs[i];
        DevInstr &D = ins[i];
        std::memset(&D, 0, sizeof(D));
        D.kind = I.kind;
        D.k_in = I.k_in;
        D.h = I.h;
        D.mu = I.mu;
        D.eta = I.eta;
        D.a = I.a;
        D.b = I.b;
        D.meas = I.meas;
        D.c = std::cos(I.theta / 2);
        D.s = std::sin(I.theta / 2);
        D.cf = (float)D.c;
        D.sf = (float)D.s;
        if (I.kind == ACTIVE_DIAG_MEAS || I.kind == ACTIVE_PAIR_MEAS) {
            D.am_idx = (uint32_t)am.size();
            am.push_back((uint32_t)I.meas);
        }
        if (I.kind == RANDOM_MEAS) {
            rm.push_back((uint32_t)i);
            continue;  // its sign is never evaluated while sampling
        }
        D.lam_c = I.lam.c;
        // causal refs as (outcome word, bit mask) pairs; a ref listed twice cancels
        std::map<uint32_t, uint32_t> words;
        for (uint32_t t : I.lam.meas) words[t >> 5] ^= 1u << (t & 31);
        D.cm_off = (uint32_t)(cmeas.size() / 2);
        D.cm_len = 0;
        for (auto &kv : words) {
            if (!kv.second) continue;
            cmeas.push_back(kv.first);
            cmeas.push_back(kv.second);
            ++D.cm_len;
        }
        for (uint32_t s : I.lam.noise) cons[s].push_back((uint32_t)i);
    }
    // Rotations followed at once by more work at the same width share one pass
    // over the vector (each step reads what the one before it writes): a pair
    // rotation and a pair rotation with another mask (on the cosets of both
    // masks), optionally then a promotion; or any rotation and a promotion.
    for (size_t i = 0; i + 1 < ins.size(); ++i) {
        DevInstr &R = ins[i];
        if (R.kind != ACTIVE_DIAG_ROT && R.kind != ACTIVE_PAIR_ROT) continue;
        const DevInstr &X = ins[i + 1];
        if (R.kind == ACTIVE_PAIR_ROT && X.kind == ACTIVE_PAIR_ROT && X.k_in == R.k_in && X.a != R.a) {
            const bool prom = i + 2 < ins.size() && ins[i + 2].kind == PROMOTE_ROT && ins[i + 2].k_in == R.k_in;
            R.fuse = prom ? 3 : 2;
            // FP64 kernels run only rotation-promotion passes; they take this mark
            if (prom) ins[i + 1].fuse = 1;
            i += prom ? 2 : 1;
        } else if (X.kind == PROMOTE_ROT && X.k_in == R.k_in) {
            R.fuse = 1;
            i += 1;
        }
    }
    // The product-component stream (paper Sec. 6): the same instructions with
    // the component's region, local width, masks and pivot, the merges before
    // them, and no fused passes.  Selected when the dense work it saves is
    // clear: at most half the dense flops, merges counted, and a vector
    // buffer no larger than the dense one.
    plan_components(P, h->PP);
    std::vector<DevInstr> pins = ins;
    std::vector<DevMerge> pmerge;
    for (size_t i = 0; i < ins.size(); ++i) {
        const ProductPlan::PInstr &Q = h->PP.ins[i];
        DevInstr &D = pins[i];
        D.fuse = 0;
        if (Q.kind == RANDOM_MEAS || Q.kind == DET_MEAS) continue;
        D.kind = Q.kind;
        D.k_in = Q.k_in;
        D.h = Q.h;
        D.a = Q.a;
        D.b = Q.b;
        D.base = Q.base;
        D.mg_off = Q.mg_off;
        D.mg_len = (uint8_t)Q.mg_len;
    }
    for (const ProductPlan::Merge &m : h->PP.merges) {
        DevMerge d;
        std::memset(&d, 0, sizeof(d));
        d.dst = m.dst;
        d.src1 = m.src1;
        d.src2 = m.src2;
        d.m1w = (m.m1 & 0xFFFFFFu) | (m.w << 24);
        pmerge.push_back(d);
    }
    {
        uint32_t ke = 0;
        while (((uint64_t)1 << ke) < h->PP.vcap) ++ke;
        h->k_eff = ke;
        bool fits = h->PP.valid && P.k_max >= 1 && ke <= 20;
        for (const ProductPlan::PInstr &Q : h->PP.ins) fits = fits && Q.mg_len < 256;
        const bool clear = h->PP.work_product + 64.0 * h->PP.n_merges <= 0.5 * h->PP.work_dense && ke <= P.k_max;
        h->product = fits && (h->comp_mode == 2 || (h->comp_mode == 0 && clear));
    }
    std::vector<uint32_t> symoff(P.n_noise_sym + 1, 0), symcons;
    for (uint32_t s = 0; s < P.n_noise_sym; ++s) {
        symoff[s] = (uint32_t)symcons.size();
        symcons.insert(symcons.end(), cons[s].begin(), cons[s].end());
    }
    symoff[P.n_noise_sym] = (uint32_t)symcons.size();
    std::vector<uint32_t> recmeas(P.n_rec);
    for (uint64_t t = 0; t < P.n_meas; ++t)
        if (P.meas_row[t] >= 0) recmeas[(size_t)P.meas_row[t]] = (uint32_t)t;
    std::vector<uint32_t> detoff, detrows, obsoff, obsrows;
    for (auto &d : P.det_meas) {
        detoff.push_back((uint32_t)detrows.size());
        for (uint32_t t : d) detrows.push_back((uint32_t)P.meas_row[t]);
    }
    detoff.push_back((uint32_t)detrows.size());
    for (auto &o : P.obs_meas) {
        obsoff.push_back((uint32_t)obsrows.size());
        for (uint32_t t : o) obsrows.push_back((uint32_t)P.meas_row[t]);
    }
    obsoff.push_back((uint32_t)obsrows.size());
    std::vector<uint64_t> clsQ;
    std::vector<uint32_t> clsoff, clschan;
    std::vector<float> invlog;
    std::vector<GapFast> clsfast;
    for (auto &c : P.classes) {
        const double q = 1.0 - std::ldexp((double)c.p32, -32);
        invlog.push_back(q > 0 ? (float)(1.0 / std::log2(q)) : -0.0f);
        clsfast.push_back(gap_fast_constants(c.p32, c.Q.data()));
        clsQ.insert(clsQ.end(), c.Q.begin(), c.Q.end());
        clsoff.push_back((uint32_t)clschan.size());
        for (int32_t ch : c.chans) clschan.push_back((uint32_t)ch);
    }
    clsoff.push_back((uint32_t)clschan.size());
    std::vector<DevChan> chans(P.chans.size());
    std::vector<uint32_t> bmask;
    std::vector<uint64_t> thr;
    for (size_t i = 0; i < P.chans.size(); ++i) {
        const Channel &c = P.chans[i];
        DevChan &d = chans[i];
        d.J = (uint8_t)c.J;
        d.uniform = c.uniform;
        d.nsym = (uint8_t)c.nsym;
        d.pad = 0;
        d.sym0 = c.sym0;
        d.bm_off = (uint32_t)bmask.size();
        bmask.insert(bmask.end(), c.bmask.begin(), c.bmask.end());
        d.thr_off = (uint32_t)thr.size();
        thr.insert(thr.end(), c.thr.begin(), c.thr.end());
    }
    build_frame_schedule(P, h->F);
    L.blob.clear();
    L.o_instr = put(L.blob, ins);
    L.o_pinstr = put(L.blob, pins);
    L.o_merge = put(L.blob, pmerge);
    L.o_cmeas = put(L.blob, cmeas);
    L.o_am = put(L.blob, am);
    L.o_rm = put(L.blob, rm);
    L.o_recmeas = put(L.blob, recmeas);
    L.o_detoff = put(L.blob, detoff);
    L.o_detrows = put(L.blob, detrows);
    L.o_obsoff = put(L.blob, obsoff);
    L.o_obsrows = put(L.blob, obsrows);
    L.o_clsQ = put(L.blob, clsQ);
    L.o_clsoff = put(L.blob, clsoff);
    L.o_clschan = put(L.blob, clschan);
    L.o_chan = put(L.blob, chans);
    L.o_bmask = put(L.blob, bmask);
    L.o_thr = put(L.blob, thr);
    L.o_symoff = put(L.blob, symoff);
    L.o_symcons = put(L.blob, symcons);
    L.o_invlog = put(L.blob, invlog);
    L.o_clsfast = put(L.blob, clsfast);
    L.o_frstep = put(L.blob, h->F.steps);
    L.o_frnodes = put(L.blob, h->F.nodes);
    L.o_frpush = put(L.blob, h->F.push);
    L.o_frnodes16 = put(L.blob, h->F.nodes16);
    L.o_frpush16 = put(L.blob, h->F.push16);
    L.o_frchinfo = put(L.blob, h->F.chinfo);
    L.o_ci32 = put(L.blob, h->F.ci32);
    L.o_st8 = put(L.blob, h->F.st8);
    {
        std::vector<uint32_t> q32;
        for (auto &c : P.classes)
            for (size_t g = 0; g < c.Q.size(); ++g) q32.push_back(c.Q[g] >= (uint64_t(1) << 32) ? 0xFFFFFFFFu : (uint32_t)c.Q[g]);
        // whole 16-byte units for the LDS copy; the walks treat entry 0 (2^32) as above every draw
        q32.resize((q32.size() + 3) & ~(size_t)3, 0u);
        L.o_q32 = put(L.blob, q32);
    }
    L.o_frrec = put(L.blob, h->F.frec);
    L.o_frfl3 = put(L.blob, h->F.fl3);
    {
        std::vector<uint32_t> capoff(1, 0);
        for (uint32_t c : h->F.cls_cap) capoff.push_back(capoff.back() + c);
        L.o_frcap = put(L.blob, h->F.cls_cap);
        L.o_frcapoff = put(L.blob, capoff);
        L.word_entries = capoff.back();
    }
    L.o_wvops = put(L.blob, h->F.wops);
    L.o_wvrows = put(L.blob, h->F.wrows);
    L.o_wvfl = put(L.blob, h->F.wfl);
    L.o_wvsl = put(L.blob, h->F.wsl);
    L.o_wvrm = put(L.blob, h->F.rm_meas);
    {
        std::vector<uint32_t> capoff(1, 0);
        for (uint32_t c : h->F.wcap) capoff.push_back(capoff.back() + c);
        L.o_wvcap = put(L.blob, h->F.wcap);
        L.o_wvcapoff = put(L.blob, capoff);
        L.wv_word_entries = capoff.back();
    }
    DevProg &m = L.meta;
    std::memset(&m, 0, sizeof(m));
    m.n_instr = (uint32_t)ins.size();
    m.n_meas = (uint32_t)P.n_meas;
    m.n_rm = (uint32_t)rm.size();
    m.n_am = (uint32_t)am.size();
    m.n_rec = (uint32_t)P.n_rec;
    m.n_det = (uint32_t)P.n_det;
    m.n_obs = (uint32_t)P.n_obs;
    m.n_cls = (uint32_t)P.classes.size();
    m.k_max = P.k_max;
    m.fr_n_steps = (uint32_t)h->F.n_steps;
    m.fr_n_slots = h->F.n_slots;
    m.fr_first_emit = h->F.first_emit[0];
    m.fr_first_emit_n = h->F.first_emit[1];
    m.fr_first_noise_cls = h->F.first_noise_cls;
    m.n_sym = P.n_noise_sym;
    m.fr_n_cch = (uint32_t)h->F.ci32.size();
    m.fr_rec_ok = h->F.rec_ok ? 1u : 0u;
    {
        // the 32-bit gap tables are exact when every Q[g], g >= 1, is below 2^32
        bool q_ok = true;
        for (auto &c : P.classes)
            for (size_t g = 1; g < c.Q.size(); ++g) q_ok = q_ok && c.Q[g] < (uint64_t(1) << 32);
        m.fr_ltab = h->F.ltab_ok && q_ok ? 1u : 0u;
    }
    m.wv_n_ops = (uint32_t)(h->F.wops.size() / WV_OP_WORDS);
    m.wv_n_rm = (uint32_t)h->F.rm_meas.size();
    m.wv_first_noise_cls = h->F.w_first_noise_cls;
    m.wv_first_batch = h->F.w_first_batch[0];
    m.wv_first_batch_n = h->F.w_first_batch[1];
    m.wv_ok = h->F.ok && h->F.wave_ok && frame_wave_lds_bytes(m) <= kLdsLimit ? 1u : 0u;
    m.fr_ok = h->F.ok && (m.wv_ok || frame_lds_bytes(m, 16) <= kLdsLimit) ? 1u : 0u;
}

// Scratch memory handed in by the caller of a launch instead of taken from the
// pool: the launch caps its grid so that its scratch fits `bytes`.
struct FixedScratch {
    void *ptr;
    size_t bytes;
};

// upload = false: fail instead of uploading a program that is not resident on
// the current device (the allocation-free entry point allocates nothing).
// dense = true: the dense instruction stream even for a product-component
// program (the amplitude probe reads the whole vector).
static symft_status device_prog(symft_program *h, DevProg &out, bool upload = true, bool dense = false) {
    int dev = 0;
    if (const hipError_t e = hipGetDevice(&dev)) return hip_err("hipGetDevice failed", e);
    std::lock_guard<std::mutex> lk(h->mu);
    void *base = nullptr;
    auto it = h->dev.find(dev);
    if (it == h->dev.end() && !upload)
        return set_err(SYMFT_EINVAL, "the program is not resident on this device (sample it once with symft_sample_ex)");
    if (it == h->dev.end()) {
        if (hipMalloc(&base, h->L.blob.size()) != hipSuccess) return set_err(SYMFT_ENOMEM, "device program allocation failed");
        if (hipMemcpy(base, h->L.blob.data(), h->L.blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(base);
            return set_err(SYMFT_EHIP, "device program upload failed");
        }
        h->dev[dev] = base;
    } else {
        base = it->second;
    }
    const uint8_t *b = (const uint8_t *)base;
    const HostLayout &L = h->L;
    out = L.meta;
    out.instr = (const DevInstr *)(b + L.o_instr);
    out.merges = (const DevMerge *)(b + L.o_merge);
    out.vcap = 1u << out.k_max;
    if (h->product && !dense) {
        out.instr = (const DevInstr *)(b + L.o_pinstr);
        out.k_max = h->k_eff;
        out.vcap = h->PP.vcap;
    }
    out.cmeas = (const uint32_t *)(b + L.o_cmeas);
    out.am_meas = (const uint32_t *)(b + L.o_am);
    out.rm_list = (const uint32_t *)(b + L.o_rm);
    out.rec_meas = (const uint32_t *)(b + L.o_recmeas);
    out.det_off = (const uint32_t *)(b + L.o_detoff);
    out.det_rows = (const uint32_t *)(b + L.o_detrows);
    out.obs_off = (const uint32_t *)(b + L.o_obsoff);
    out.obs_rows = (const uint32_t *)(b + L.o_obsrows);
    out.cls_Q = (const uint64_t *)(b + L.o_clsQ);
    out.cls_off = (const uint32_t *)(b + L.o_clsoff);
    out.cls_chan = (const uint32_t *)(b + L.o_clschan);
    out.chan = (const DevChan *)(b + L.o_chan);
    out.bmask = (const uint32_t *)(b + L.o_bmask);
    out.thr = (const uint64_t *)(b + L.o_thr);
    out.sym_off = (const uint32_t *)(b + L.o_symoff);
    out.sym_cons = (const uint32_t *)(b + L.o_symcons);
    out.cls_invlog2q = (const float *)(b + L.o_invlog);
    out.cls_fast = (const GapFast *)(b + L.o_clsfast);
    out.fr_step = (const uint32_t *)(b + L.o_frstep);
    out.fr_nodes = (const uint32_t *)(b + L.o_frnodes);
    out.fr_push = (const uint32_t *)(b + L.o_frpush);
    out.fr_nodes16 = (const uint32_t *)(b + L.o_frnodes16);
    out.fr_push16 = (const uint32_t *)(b + L.o_frpush16);
    out.fr_chinfo = (const uint64_t *)(b + L.o_frchinfo);
    out.fr_ci32 = (const uint32_t *)(b + L.o_ci32);
    out.fr_st8 = (const uint8_t *)(b + L.o_st8);
    out.cls_Q32 = (const uint32_t *)(b + L.o_q32);
    out.fr_frec = (const uint64_t *)(b + L.o_frrec);
    out.fr_fl3 = (const uint64_t *)(b + L.o_frfl3);
    out.fr_cap = (const uint32_t *)(b + L.o_frcap);
    out.fr_capoff = (const uint32_t *)(b + L.o_frcapoff);
    out.wv_ops = (const uint32_t *)(b + L.o_wvops);
    out.wv_rows = (const uint32_t *)(b + L.o_wvrows);
    out.wv_fl = (const uint64_t *)(b + L.o_wvfl);
    out.wv_sl = (const uint16_t *)(b + L.o_wvsl);
    out.wv_rm = (const uint32_t *)(b + L.o_wvrm);
    out.wv_cap = (const uint32_t *)(b + L.o_wvcap);
    out.wv_capoff = (const uint32_t *)(b + L.o_wvcapoff);
    return SYMFT_OK;
}

// Stream-ordered scratch from one library-owned pool per device, which keeps
// its memory between calls (release threshold at its maximum), so repeated
// launches of the same size do not go back to the driver.
static std::mutex g_pool_mu;
static std::map<int, hipMemPool_t> g_pools;

static hipError_t pool_alloc(void **p, size_t bytes, hipStream_t st) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipMemPool_t pool;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        auto it = g_pools.find(dev);
        if (it == g_pools.end()) {
            hipMemPoolProps pr;
            std::memset(&pr, 0, sizeof(pr));
            pr.allocType = hipMemAllocationTypePinned;
            pr.location.type = hipMemLocationTypeDevice;
            pr.location.id = dev;
            e = hipMemPoolCreate(&pool, &pr);
            if (e != hipSuccess) return e;
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
            g_pools[dev] = pool;
        } else {
            pool = it->second;
        }
    }
    return hipMallocFromPoolAsync(p, std::max<size_t>(bytes, 256), pool, st);
}

static int g_num_cus = 0;
static int num_cus() {
    if (!g_num_cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, dev) == hipSuccess) g_num_cus = pr.multiProcessorCount;
        if (g_num_cus <= 0) g_num_cus = 256;
    }
    return g_num_cus;
}

// Launch configuration of the active kernel for a program.
struct ActiveConfig {
    uint32_t bs, tps;
    bool lds_vec;
    bool lane = false;  // the lane kernel: one wave per word, one lane per shot
    size_t lds;
};

// Threads per shot chosen by the autotuner for launches that have the GPU to
// themselves, per (peak active width, precision); tuned on 4096 words, so
// occupancy weighs in.
static std::mutex g_tune_mu;
static std::map<std::pair<uint32_t, bool>, uint32_t> g_tune;

// Threads per shot of a batch member.  The members share one workgroup size
// (256) and the LDS size of the largest member, which sets the occupancy of
// the whole batch.  Each member takes G = budget / (2^k amplitudes) shot
// groups per workgroup (at most 64), 256 / G threads each, for an LDS budget
// per workgroup that the batch chooses (symft_sample_batch times 32 and 64
// KB).  On the 128-program batch with dense vectors (widths 1..12), 64 KB, two
// workgroups per CU, ran every width fastest; with most members on small
// product components, 32 KB (three per CU) did, one wide member no longer
// holding the others to two.  Timing members alone cannot find this: a few
// hundred words give each CU one workgroup whatever its LDS size.
static const uint64_t kBatchBudgets[2] = {65536, 32768};
static uint32_t batch_tps(uint32_t k, bool fp64, uint64_t budget) {
    const uint64_t per_shot = ((uint64_t)1 << k) * (fp64 ? 16u : 8u);
    const uint64_t G = std::max<uint64_t>(1, std::min<uint64_t>(64, budget / per_shot));
    return (uint32_t)(256 / G);
}

// Threads per shot before the autotuner has run: about 2^(k-4) amplitudes'
// worth of threads in FP32 and twice that in FP64, at least 4 (the choices
// the autotuner makes on near-Clifford programs of width 1..12).
static uint32_t default_tps(uint32_t k, bool fp64) {
    const int e = (int)k - (fp64 ? 3 : 4);
    return e <= 2 ? 4u : e >= 8 ? 256u : (1u << e);
}

// Peak widths 13 and 14: narrow shot groups with vectors in HBM scratch
// (which the L2 and the Infinity Cache hold at these sizes) keep many shots
// in flight.  One shot per 1024-thread workgroup, with its vector in LDS,
// left most threads idle at the small widths where a shot spends most of its
// instructions (C5 at width 14: 72 ms against 15 ms at 128 threads per
// shot).  From width 15 on, streaming the vector bounds the kernel, and 1024
// threads per shot stream it best.
static bool narrow_wide(uint32_t k) { return k >= 13 && k <= 14; }

// A tuned (or forced) launch choice at peak widths 9..12 may carry this bit:
// narrow groups with vectors in HBM scratch instead of LDS.  Only launches
// that have the GPU to themselves are tuned that way; batch members keep LDS
// vectors, which the batch kernel needs.
static const uint32_t kHbmVec = 1u << 16;
static bool hbm_candidate(uint32_t k) { return k >= 9 && k <= 12; }

// A tuned (or forced) choice may carry this bit instead: the lane kernel, for
// programs whose whole per-wave state (64 shots' vector buffers, outcome bits
// and exogenous words) fits kLaneLds of LDS; records path only, not in batches.
static const uint32_t kLaneVec = 1u << 17;
static const size_t kLaneLds = 64 * 1024;
static bool lane_candidate(const DevProg &P, bool fp64) { return P.k_max >= 1 && lane_lds_bytes(P, fp64) <= kLaneLds; }
// In a batch the lane queue's LDS size is its largest member's, which sets the
// occupancy of all of them: members above the cap stay in the shot-group queue
// (on C4, admitting members up to 64 KB took the FP32 batch from 5.3 to 6.6
// ms).  Measured on C4 with the caps 24 / 32 / 40 KB: FP32 3.91 / 3.02 / 3.36
// ms, FP64 6.77 / 5.97 / 5.76 ms.
static size_t lane_batch_cap(bool fp64) { return fp64 ? 40 * 1024 : 32 * 1024; }
// A forced choice with this bit keeps the tuned thread count but never the lane kernel.
static const uint32_t kNoLane = 1u << 18;
// Grid cap of the launches of one workgroup per work unit; above it workgroups stride over units.
static const uint64_t kMaxGrid = (uint64_t)1 << 30;
// Count mode with one shot group per workgroup: words split into 2^kCountPartLog2 work units (1 .. 6).
static const uint32_t kCountPartLog2 = 4;

// force_tps of a sampling call from symft_sample_opts.active_kernel.
static symft_status active_choice(const DevProg &D, bool fp64, uint32_t sel, uint32_t &force) {
    force = 0;
    if (sel == 0) return SYMFT_OK;
    if (sel == 1) {
        force = kNoLane;
        return SYMFT_OK;
    }
    if (sel != 2) return set_err(SYMFT_EINVAL, "active_kernel must be 0, 1 or 2");
    if (!lane_candidate(D, fp64)) return set_err(SYMFT_ECAPACITY, "the lane kernel's state does not fit 64 KB of LDS");
    force = 1u | kLaneVec;
    return SYMFT_OK;
}

// count_mode: a workgroup holds one shot group when groups are a wave or
// more (64 .. 256 threads), so it drops a discarded shot at once.
// batch_budget: nonzero for a batch member, the batch's LDS budget per workgroup.
ActiveConfig choose_active(const DevProg &P, bool fp64, uint32_t force_tps = 0, uint64_t batch_budget = 0,
                           bool count_mode = false) {
    ActiveConfig c;
    uint32_t k = P.k_max;
    c.bs = 256;
    c.tps = narrow_wide(k) ? (fp64 ? 256u : 128u) : default_tps(k, fp64);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find({k, fp64});
        if (it != g_tune.end()) c.tps = it->second;
    }
    if (batch_budget && k < 13) c.tps = batch_tps(k, fp64, batch_budget);
    if (force_tps & kNoLane) c.tps &= ~kLaneVec;
    else if (force_tps) c.tps = force_tps;
    if ((c.tps & kLaneVec) && !batch_budget && lane_candidate(P, fp64)) {
        c.lane = true;
        c.bs = 64;
        c.tps = 1;
        c.lds = lane_lds_bytes(P, fp64);
        c.lds_vec = true;
        return c;
    }
    // a lane choice tuned on another program of this width that this one cannot take
    if (c.tps & kLaneVec) c.tps = default_tps(k, fp64);
    const bool hbm = (c.tps & kHbmVec) && hbm_candidate(k);
    c.tps &= ~kHbmVec;
    if (narrow_wide(k) && c.tps < 64) c.tps = 64;
    if (count_mode && c.tps >= 64 && c.tps <= 256) c.bs = c.tps;
    if (k >= 13 && (!narrow_wide(k) || c.tps > 256)) {
        c.bs = 1024;
        c.tps = 1024;
    }
    c.lds = active_lds_bytes(P, c.bs, c.tps, true, fp64);
    c.lds_vec = c.lds <= kLdsLimit && !(narrow_wide(k) && c.tps <= 256) && !hbm;
    if (!c.lds_vec) c.lds = active_lds_bytes(P, c.bs, c.tps, false, fp64);
    return c;
}

static symft_status run_active(symft_program *h, const DevProg &D, bool fp64, uint64_t word_begin, uint64_t n_words,
                               uint64_t shots, uint64_t *out, uint64_t stride, uint32_t sections, double *p0,
                               uint64_t probe_shot0, uint64_t probe_n, uint64_t seed, hipStream_t st,
                               uint32_t force_tps = 0, const CountArgs *cnt = nullptr, double *amp = nullptr,
                               uint32_t amp_k = 0, const FixedScratch *fixed = nullptr) {
    ActiveConfig c = choose_active(D, fp64, force_tps, 0, cnt != nullptr);
    if (c.lds > kLdsLimit) return set_err(SYMFT_ECAPACITY, "program tables exceed the LDS budget of the active kernel");
    if (c.lane) {
        ActiveArgs A;
        std::memset(&A, 0, sizeof(A));
        A.P = D;
        A.seed = seed;
        A.word_begin = word_begin;
        A.n_words = n_words;
        A.shots = shots;
        A.out = out;
        A.row_stride = stride;
        A.sections = sections;
        A.tps = 1;
        A.p0_out = p0;
        A.amp_out = amp;
        A.amp_k = amp_k;
        A.probe_shot0 = probe_shot0;
        A.probe_n = probe_n;
        A.lds_vec = 1;
        A.lds_bytes = (uint32_t)c.lds;
        if (cnt) A.cnt = *cnt;
        // One workgroup per word, left to the hardware dispatcher: a persistent grid sized by the
        // occupancy query ran the C3 FP64 stream 1.5x slower (the query admitted one more 15.5 KB
        // workgroup per CU than ran at once, so a tenth of the workgroups waited for a whole pass).
        const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(n_words, kMaxGrid));
        const hipError_t e = launch_lane(A, fp64, grid, st);
        if (e != hipSuccess) return set_err(SYMFT_EHIP, std::string("lane kernel launch failed: ") + hipGetErrorString(e));
        return SYMFT_OK;
    }
    int per_cu = active_max_blocks_per_cu(fp64, c.bs, c.lds_vec, c.lds, cnt != nullptr);
    if (per_cu <= 0) per_cu = 1;
    uint64_t cap = (uint64_t)per_cu * (uint64_t)num_cus();
    // HBM-resident vectors: about 1024 threads of shot groups per CU
    if (!c.lds_vec) cap = std::min<uint64_t>(cap, (uint64_t)num_cus() * std::max<uint32_t>(2u, 1024u / c.bs));
    // Count mode with one shot group per workgroup: work units of 4 shots (a sixteenth of a word).  A
    // rejected shot ends its work early, so the units' costs differ; whole words assigned one per
    // workgroup left the launch waiting for its costliest words (POST: 33.4 ms with whole words, 31.1
    // with 16-shot units, 29.8 with 8, 28.9 with 4, 28.8 with 2).  With LDS vectors each unit is its own workgroup (the
    // dispatcher balances them); with HBM vectors, whose slices are per workgroup, resident workgroups
    // take units from a counter at the head of the scratch.
    const uint32_t part_log2 = (cnt && c.bs == c.tps && n_words < ((uint64_t)1 << (31 - kCountPartLog2))) ? kCountPartLog2 : 0u;
    const uint64_t units = n_words << part_log2;
    const bool queue = part_log2 && !c.lds_vec;
    const uint64_t qhdr = queue ? 256 : 0;
    if (fixed && !c.lds_vec) {
        // the vector slices of every workgroup (and the unit counter) must fit the caller's scratch
        const uint64_t per_wg = (uint64_t)(c.bs / c.tps) * ((uint64_t)1 << D.k_max) * (fp64 ? 16 : 8);
        if (per_wg + qhdr > fixed->bytes)
            return set_err(SYMFT_ECAPACITY, "one workgroup's vector scratch exceeds the fixed scratch (" +
                                                std::to_string(per_wg + qhdr) + " > " + std::to_string(fixed->bytes) + " bytes)");
        cap = std::min<uint64_t>(cap, (fixed->bytes - qhdr) / per_wg);
    }
    uint32_t grid = (uint32_t)std::max<uint64_t>(
        1, (part_log2 && c.lds_vec) ? std::min<uint64_t>(units, kMaxGrid) : std::min<uint64_t>(units, cap));
    ActiveArgs A;
    std::memset(&A, 0, sizeof(A));
    A.part_log2 = part_log2;
    A.P = D;
    A.seed = seed;
    A.word_begin = word_begin;
    A.n_words = n_words;
    A.shots = shots;
    A.out = out;
    A.row_stride = stride;
    A.sections = sections;
    A.tps = c.tps;
    A.p0_out = p0;
    A.amp_out = amp;
    A.amp_k = amp_k;
    A.probe_shot0 = probe_shot0;
    A.probe_n = probe_n;
    A.lds_vec = c.lds_vec ? 1 : 0;
    A.lds_bytes = (uint32_t)c.lds;
    if (cnt) A.cnt = *cnt;
    void *scratch = nullptr;
    if (!c.lds_vec) {
        const uint32_t G = c.bs / c.tps;
        A.scratch_stride = (uint64_t)1 << D.k_max;
        size_t bytes = qhdr + (size_t)grid * G * A.scratch_stride * (fp64 ? 16 : 8);
        unsigned char *base = nullptr;
        if (fixed) {
            base = (unsigned char *)fixed->ptr;
        } else {
            if (pool_alloc(&scratch, bytes, st) != hipSuccess) return set_err(SYMFT_ENOMEM, "vector scratch allocation failed");
            base = (unsigned char *)scratch;
        }
        A.scratch = base + qhdr;
        if (queue) A.unit_counter = (uint32_t *)base;
    }
    hipError_t e = launch_active(A, fp64, c.bs, grid, st);
    if (scratch) (void)hipFreeAsync(scratch, st);
    if (e != hipSuccess) return set_err(SYMFT_EHIP, std::string("active kernel launch failed: ") + hipGetErrorString(e));
    return SYMFT_OK;
}

// The wave-owned kernel: one 16-wave workgroup per CU, each wave one word of a 16-word tile.
static symft_status run_frame_wave(symft_program *h, const DevProg &D, uint64_t word_begin, uint64_t n_words,
                                   uint64_t shots, uint64_t *out, uint64_t stride, uint32_t sections, uint64_t seed,
                                   uint32_t cap_override, hipStream_t st, const CountArgs *cnt,
                                   const FixedScratch *fixed = nullptr) {
    const size_t lds = frame_wave_lds_bytes(D);
    if (lds > kLdsLimit) return set_err(SYMFT_ECAPACITY, "frame schedule exceeds the LDS budget of the wave kernel");
    int per_cu = frame_wave_max_blocks_per_cu(lds, cnt != nullptr);
    if (per_cu <= 0) per_cu = 1;
    const uint64_t tiles = (n_words + WV_TILE - 1) / WV_TILE;
    uint64_t cap = (uint64_t)per_cu * num_cus();
    WaveArgs A;
    std::memset(&A, 0, sizeof(A));
    A.word_entries = cap_override ? cap_override * D.n_cls : h->L.wv_word_entries;
    A.cap_override = cap_override;
    const uint64_t per_wg = (uint64_t)WV_TILE * std::max<uint32_t>(1, A.word_entries) * 4;
    if (fixed) {
        if (per_wg > fixed->bytes)
            return set_err(SYMFT_ECAPACITY, "one workgroup's flip-entry scratch exceeds the fixed scratch (" +
                                                std::to_string(per_wg) + " > " + std::to_string(fixed->bytes) + " bytes)");
        cap = std::min<uint64_t>(cap, fixed->bytes / per_wg);
    }
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(tiles, cap));
    void *scratch = nullptr;
    if (fixed) {
        A.scratch = (uint32_t *)fixed->ptr;
    } else {
        if (pool_alloc(&scratch, (size_t)grid * per_wg, st) != hipSuccess)
            return set_err(SYMFT_ENOMEM, "frame scratch allocation failed");
        A.scratch = (uint32_t *)scratch;
    }
    A.P = D;
    A.seed = seed;
    A.word_begin = word_begin;
    A.n_words = n_words;
    A.shots = shots;
    A.out = out;
    A.row_stride = stride;
    A.sections = sections;
    A.store16 = (((uintptr_t)out & 15u) == 0 && (stride & 1u) == 0) ? 1u : 0u;
    A.lds_bytes = (uint32_t)lds;
    if (cnt) A.cnt = *cnt;
    hipError_t e = launch_frame_wave(A, grid, st);
    if (scratch) (void)hipFreeAsync(scratch, st);
    if (e != hipSuccess) return set_err(SYMFT_EHIP, std::string("frame kernel launch failed: ") + hipGetErrorString(e));
    return SYMFT_OK;
}

// frame_kernel: 0 automatic (the step-synchronous kernel when its LDS fits,
// else the wave-owned one), 1 wave-owned, 2 step-synchronous (tile_words 16 /
// 32 or 0 = automatic); tile_words != 0 implies the step-synchronous kernel.
// Small calls of small schedules take the wave-owned kernel: it has no workgroup barriers, and at a few
// tiles per CU the step kernel's chain of barrier steps is the whole launch.  Measured per call, 16 to
// 4,096 words: d = 3 surface code (58 rows) 26-30 us against 31-34 us, d = 5 (266 rows) 35-40 against
// 39-43 us; at d = 11 (2,762 rows) the step kernel is faster at every size, and at 16,384 words for all
// three.
static const uint64_t kSmallFrameWords = 4096;
static bool frame_small_program(const DevProg &D) {
    return D.wv_ok && (uint64_t)D.n_rec + D.n_det + D.n_obs <= 512;
}

static symft_status run_frame(symft_program *h, const DevProg &D, uint64_t word_begin, uint64_t n_words, uint64_t shots,
                              uint64_t *out, uint64_t stride, uint32_t sections, uint64_t seed, uint32_t cap_override,
                              hipStream_t st, const CountArgs *cnt = nullptr, uint32_t tile_words = 0,
                              uint32_t frame_kernel = 0, const FixedScratch *fixed = nullptr) {
    if (tile_words != 0 && tile_words != 16 && tile_words != 32)
        return set_err(SYMFT_EINVAL, "frame_tile_words must be 0, 16 or 32");
    if (frame_kernel > 2) return set_err(SYMFT_EINVAL, "frame_kernel must be 0, 1 or 2");
    if (frame_kernel == 1 && tile_words) return set_err(SYMFT_EINVAL, "frame_tile_words applies to the step kernel only");
    if (frame_kernel == 1 && !D.wv_ok)
        return set_err(SYMFT_ECAPACITY, "the wave-owned frame kernel cannot run this schedule (LDS)");
    const bool step_fits = frame_lds_bytes(D, 16) <= kLdsLimit;
    const bool small = n_words <= kSmallFrameWords && frame_small_program(D);
    if (frame_kernel == 1 || (frame_kernel == 0 && !tile_words && D.wv_ok && (!step_fits || small)))
        return run_frame_wave(h, D, word_begin, n_words, shots, out, stride, sections, seed, cap_override, st, cnt,
                              fixed);
    // 32-word tiles halve the barrier steps per word; they need the slots of
    // 32 words in LDS and leave one workgroup per CU, so they are taken only
    // with at least two tiles per CU
    uint32_t tw = tile_words;
    if (!tw) tw = frame_lds_bytes(D, 32) <= kLdsLimit && (n_words + 31) / 32 >= 2 * (uint64_t)num_cus() ? 32 : 16;
    size_t lds = frame_lds_bytes(D, tw);
    if (lds > kLdsLimit) return set_err(SYMFT_ECAPACITY, "frame schedule exceeds the LDS budget");
    int per_cu = frame_max_blocks_per_cu(lds, tw);
    if (per_cu <= 0) per_cu = 1;
    uint64_t tiles = (n_words + tw - 1) / tw;
    uint64_t cap = (uint64_t)per_cu * (uint64_t)num_cus();
    FrameArgs A;
    std::memset(&A, 0, sizeof(A));
    A.word_entries = cap_override ? cap_override * D.n_cls : h->L.word_entries;
    A.cap_override = cap_override;
    const uint64_t per_wg = (uint64_t)frame_scratch_words(A.word_entries, tw) * 8;
    if (fixed) {
        if (per_wg > fixed->bytes)
            return set_err(SYMFT_ECAPACITY, "one workgroup's flip-entry scratch exceeds the fixed scratch (" +
                                                std::to_string(per_wg) + " > " + std::to_string(fixed->bytes) + " bytes)");
        cap = std::min<uint64_t>(cap, fixed->bytes / per_wg);
    }
    uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(tiles, cap));
    void *scratch = nullptr;
    if (fixed) {
        A.scratch = (uint64_t *)fixed->ptr;
    } else {
        if (pool_alloc(&scratch, (size_t)grid * per_wg, st) != hipSuccess)
            return set_err(SYMFT_ENOMEM, "frame scratch allocation failed");
        A.scratch = (uint64_t *)scratch;
    }
    A.P = D;
    A.seed = seed;
    A.word_begin = word_begin;
    A.n_words = n_words;
    A.shots = shots;
    A.out = out;
    A.row_stride = stride;
    A.sections = sections;
    A.store16 = (((uintptr_t)out & 15u) == 0 && (stride & 1u) == 0) ? 1u : 0u;
    A.lds_bytes = (uint32_t)lds;
    if (cnt) A.cnt = *cnt;
    hipError_t e = launch_frame(A, grid, st, tw);
    if (scratch) (void)hipFreeAsync(scratch, st);
    if (e != hipSuccess) return set_err(SYMFT_EHIP, std::string("frame kernel launch failed: ") + hipGetErrorString(e));
    return SYMFT_OK;
}

extern "C" {

const char *symft_last_error(void) { return g_err.c_str(); }

symft_status symft_compile(uint32_t n_qubits, const symft_op *ops, size_t n_ops, const void *opts, symft_program **out) {
    if (!out) return set_err(SYMFT_EINVAL, "out is NULL");
    *out = nullptr;
    symft_compile_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *(const symft_compile_opts *)opts;
    if (o.simplify > 1) return set_err(SYMFT_EINVAL, "simplify must be 0 or 1");
    if (o.components > 2) return set_err(SYMFT_EINVAL, "components must be 0, 1 or 2");
    symft_program *h = nullptr;
    try {
        h = new symft_program();
        h->comp_mode = o.components;
        std::string err;
        std::vector<symft_op> rewritten;
        uint64_t removed = 0;
        if (o.simplify && n_ops) {
            // the rewrite reads qubit and Pauli arrays, so check their presence first
            for (size_t i = 0; i < n_ops; ++i)
                if (ops[i].n && (!ops[i].qubits || (ops[i].kind == SYMFT_OP_ROT && !ops[i].paulis))) {
                    delete h;
                    return set_err(SYMFT_EINVAL, "op " + std::to_string(i) + ": qubits or paulis is NULL");
                }
            rewritten = simplify_rotations(ops, n_ops, removed);
        }
        int rc = compile_program(n_qubits, o.simplify && n_ops ? rewritten.data() : ops, n_ops, h->P, err);
        h->P.rot_removed = removed;
        if (rc) {
            delete h;
            return set_err(rc, err);
        }
        lower(h);
    } catch (const std::bad_alloc &) {
        delete h;
        return set_err(SYMFT_ENOMEM, "host allocation failed during compile");
    }
    *out = h;
    return SYMFT_OK;
}

void symft_program_free(symft_program *p) { delete p; }

symft_status symft_program_info(const symft_program *p, symft_info *info) {
    if (!p || !info) return set_err(SYMFT_EINVAL, "NULL argument");
    const Program &P = p->P;
    std::memset(info, 0, sizeof(*info));
    info->n_qubits = P.n_qubits;
    info->k_max = P.k_max;
    info->n_ops = P.n_ops;
    info->n_measurements = P.n_meas;
    info->n_records = P.n_rec;
    info->n_detectors = P.n_det;
    info->n_observables = P.n_obs;
    info->n_rows = P.n_rows();
    info->n_channels = P.chans.size();
    info->n_classes = P.classes.size();
    info->n_noise_symbols = P.n_noise_sym;
    double flops = 0, bytes = 0;
    for (const Instr &I : P.instrs) {
        info->n_instr[I.kind] += 1;
        if (I.kind != RANDOM_MEAS) {
            info->expr_noise_nnz += I.lam.noise.size();
            info->expr_meas_nnz += I.lam.meas.size();
        }
        const double N = std::ldexp(1.0, I.k_in);
        switch (I.kind) {
        case PROMOTE_ROT: flops += 4 * N; bytes += 8 * (N + 2 * N); break;
        case ACTIVE_DIAG_ROT: flops += 6 * N; bytes += 8 * 2 * N; break;
        case ACTIVE_PAIR_ROT: flops += 6 * N; bytes += 8 * 2 * N; break;
        case ACTIVE_DIAG_MEAS: flops += 4 * N + 2 * (N / 2); bytes += 8 * (N + N / 2); break;
        case ACTIVE_PAIR_MEAS: flops += 8 * N + 6 * (N / 2); bytes += 8 * (N + N / 2); break;
        default: break;
        }
    }
    info->dense_flops_per_shot = flops;
    info->dense_bytes_per_shot = bytes;
    info->frame_steps = p->F.n_steps;
    info->frame_slots = p->F.n_slots;
    info->frame_max_level = p->F.max_level;
    info->frame_noise_consumers = p->F.n_flips;
    info->rotations_removed = p->P.rot_removed;
    info->frame_pushes = p->F.n_pushes;
    info->frame_kernel = p->L.meta.fr_ok ? (frame_lds_bytes(p->L.meta, 16) <= kLdsLimit ? 2u : 1u) : 0u;
    info->frame_wave_batches = p->F.w_n_batches;
    info->frame_wave_flushes = p->F.w_n_flushes;
    info->frame_small_words =
        p->L.meta.fr_ok && info->frame_kernel == 2 && frame_small_program(p->L.meta) ? kSmallFrameWords : 0u;
    info->product_selected = p->product ? 1u : 0u;
    info->product_components = p->PP.n_comps;
    info->product_merges = p->PP.n_merges;
    info->product_vector_amplitudes = p->PP.vcap;
    info->product_flops_per_shot = p->PP.work_product;
    for (size_t i = 0; i < p->F.steps.size(); i += FR_STEP_WORDS)
        if (p->F.steps[i] == FR_NOISE) info->frame_noise_steps += 1;
    return SYMFT_OK;
}

symft_status symft_program_plan(const symft_program *p, int16_t *k_after_op, int8_t *meas_kind, int8_t *rot_kind) {
    if (!p) return set_err(SYMFT_EINVAL, "NULL program");
    const Program &P = p->P;
    // (an empty vector may hand out a null pointer, which memcpy must not see even for 0 bytes)
    if (k_after_op && !P.k_after_op.empty())
        std::memcpy(k_after_op, P.k_after_op.data(), P.k_after_op.size() * sizeof(int16_t));
    if (meas_kind && !P.meas_kind.empty()) std::memcpy(meas_kind, P.meas_kind.data(), P.meas_kind.size());
    if (rot_kind && !P.rot_kind.empty()) std::memcpy(rot_kind, P.rot_kind.data(), P.rot_kind.size());
    return SYMFT_OK;
}

symft_status symft_program_export(const symft_program *p, uint64_t *counts, int64_t *instr, double *theta,
                                  uint32_t *noise_refs, uint32_t *meas_refs, int64_t *chan, uint32_t *bmask) {
    if (!p || !counts) return set_err(SYMFT_EINVAL, "NULL argument");
    const Program &P = p->P;
    uint64_t nn = 0, nmr = 0, nb = 0;
    for (const Instr &I : P.instrs) {
        nn += I.lam.noise.size();
        nmr += I.lam.meas.size();
    }
    for (const Channel &c : P.chans) nb += c.bmask.size();
    counts[0] = P.instrs.size();
    counts[1] = nn;
    counts[2] = nmr;
    counts[3] = P.chans.size();
    counts[4] = nb;
    uint64_t on = 0, om = 0, ob = 0;
    for (size_t i = 0; i < P.instrs.size(); ++i) {
        const Instr &I = P.instrs[i];
        if (instr) {
            int64_t *r = instr + 13 * i;
            r[0] = I.kind; r[1] = I.k_in; r[2] = I.h; r[3] = I.mu; r[4] = I.eta; r[5] = I.lam.c;
            r[6] = I.a; r[7] = I.b; r[8] = I.meas;
            r[9] = (int64_t)on; r[10] = (int64_t)I.lam.noise.size();
            r[11] = (int64_t)om; r[12] = (int64_t)I.lam.meas.size();
        }
        if (theta) theta[i] = I.theta;
        if (noise_refs) std::copy(I.lam.noise.begin(), I.lam.noise.end(), noise_refs + on);
        if (meas_refs) std::copy(I.lam.meas.begin(), I.lam.meas.end(), meas_refs + om);
        on += I.lam.noise.size();
        om += I.lam.meas.size();
    }
    for (size_t c = 0; c < P.chans.size(); ++c) {
        const Channel &ch = P.chans[c];
        if (chan) {
            chan[4 * c] = ch.sym0; chan[4 * c + 1] = ch.nsym; chan[4 * c + 2] = ch.J; chan[4 * c + 3] = (int64_t)ob;
        }
        if (bmask) std::copy(ch.bmask.begin(), ch.bmask.end(), bmask + ob);
        ob += ch.bmask.size();
    }
    return SYMFT_OK;
}

symft_status symft_sample_ex(const symft_program *pc, const symft_sample_opts *opts, uint64_t shots, uint64_t seed,
                             uint64_t *records_out, void *stream) {
    symft_program *p = const_cast<symft_program *>(pc);
    if (!p) return set_err(SYMFT_EINVAL, "NULL program");
    symft_sample_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.shot_offset % 64) return set_err(SYMFT_EINVAL, "shot_offset must be a multiple of 64");
    if (o.precision > 1) return set_err(SYMFT_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
    if (shots == 0 || p->P.n_rows() == 0) return SYMFT_OK;  // nothing observable to write
    if (!records_out) return set_err(SYMFT_EINVAL, "records_out is NULL");
    const uint64_t n_words = (shots + 63) / 64;
    const uint64_t stride = o.row_stride_words ? o.row_stride_words : n_words;
    if (stride < n_words) return set_err(SYMFT_EINVAL, "row_stride_words smaller than the shot words");
    const uint32_t sections = o.sections ? o.sections : 7u;
    DevProg D;
    symft_status rc = device_prog(p, D);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t w0 = o.shot_offset / 64;
    if (D.fr_ok)
        return run_frame(p, D, w0, n_words, shots, records_out, stride, sections, seed, o.frame_entry_cap, st,
                         nullptr, o.frame_tile_words, o.frame_kernel);
    uint32_t force = 0;
    rc = active_choice(D, o.precision == 0, o.active_kernel, force);
    if (rc) return rc;
    return run_active(p, D, o.precision == 0, w0, n_words, shots, records_out, stride, sections, nullptr, 0, 0, seed, st,
                      force);
}

symft_status symft_sample(const symft_program *p, uint64_t shots, uint64_t seed, uint64_t *records_out, void *stream) {
    return symft_sample_ex(p, nullptr, shots, seed, records_out, stream);
}

}  // extern "C"

// ------------------------------------------------- allocation-free sampling
// The scratch of symft_sample_noalloc: every launch of that entry point takes
// its kernels' scratch (flip entries of the frame kernels, HBM vector slices
// of the active kernel) from this array instead of allocating, and caps its
// grid to fit.  Each device holds its own copy for the life of the process.
// In host code the name `scratch` stands for the host-side shadow of the
// symbol, not a device address: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is passed on.
static constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static constexpr int kNoAllocMaxDevices = 64;
static void *g_scratch_dev[kNoAllocMaxDevices];
static std::mutex g_scratch_mu;

// The device address of `scratch` on the current device, looked up on the
// first call on that device.
static symft_status noalloc_scratch(FixedScratch &out) {
    int dev = 0;
    if (const hipError_t e = hipGetDevice(&dev)) return hip_err("hipGetDevice failed", e);
    if (dev < 0 || dev >= kNoAllocMaxDevices) return set_err(SYMFT_ECAPACITY, "device index past the fixed scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_err("hipGetSymbolAddress of the fixed scratch failed", e);
        if (!ptr) return set_err(SYMFT_EHIP, "hipGetSymbolAddress returned no address for the fixed scratch");
        g_scratch_dev[dev] = ptr;
    }
    out.ptr = g_scratch_dev[dev];
    out.bytes = kNoAllocScratchBytes;
    return SYMFT_OK;
}

extern "C" {

symft_status symft_sample_noalloc(const symft_program *pc, const symft_sample_opts *opts, uint64_t shots,
                                  uint64_t seed, uint64_t *records_out, void *stream) {
    symft_program *p = const_cast<symft_program *>(pc);
    if (!p) return set_err(SYMFT_EINVAL, "NULL program");
    symft_sample_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.shot_offset % 64) return set_err(SYMFT_EINVAL, "shot_offset must be a multiple of 64");
    if (o.precision > 1) return set_err(SYMFT_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
    if (shots == 0 || p->P.n_rows() == 0) return SYMFT_OK;
    if (!records_out) return set_err(SYMFT_EINVAL, "records_out is NULL");
    const uint64_t n_words = (shots + 63) / 64;
    const uint64_t stride = o.row_stride_words ? o.row_stride_words : n_words;
    if (stride < n_words) return set_err(SYMFT_EINVAL, "row_stride_words smaller than the shot words");
    const uint32_t sections = o.sections ? o.sections : 7u;
    FixedScratch fx;
    symft_status rc = noalloc_scratch(fx);
    if (rc) return rc;
    DevProg D;
    rc = device_prog(p, D, false);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t w0 = o.shot_offset / 64;
    if (D.fr_ok)
        return run_frame(p, D, w0, n_words, shots, records_out, stride, sections, seed, o.frame_entry_cap, st,
                         nullptr, o.frame_tile_words, o.frame_kernel, &fx);
    uint32_t force = 0;
    rc = active_choice(D, o.precision == 0, o.active_kernel, force);
    if (rc) return rc;
    return run_active(p, D, o.precision == 0, w0, n_words, shots, records_out, stride, sections, nullptr, 0, 0, seed,
                      st, force, nullptr, nullptr, 0, &fx);
}

}  // extern "C"

// Device tables of an aggregate-count call: postselection bits per detector,
// expected-value bits per observable, and for each instruction the
// postselected detectors whose last record it makes (checked right after it).
// Uploaded once per (device, content) and kept with the program.
static symft_status count_tables(symft_program *h, const symft_count_opts &o, CountArgs &C,
                                 std::vector<uint32_t> *key_out = nullptr) {
    const Program &P = h->P;
    const size_t nd32 = std::max<size_t>(1, (P.n_det + 31) / 32), no32 = std::max<size_t>(1, (P.n_obs + 31) / 32);
    std::vector<uint32_t> tab(nd32 + no32, 0u);
    for (uint32_t i = 0; i < o.n_post; ++i) {
        const uint32_t d = o.post[i];
        if (d >= P.n_det) return set_err(SYMFT_EINVAL, "postselected detector index out of range");
        tab[d >> 5] |= 1u << (d & 31);
    }
    for (uint64_t b = 0; b < P.n_obs && o.obs_expected; ++b) {
        if (o.obs_expected[b] > 1) return set_err(SYMFT_EINVAL, "expected observable values must be 0 or 1");
        if (o.obs_expected[b]) tab[nd32 + (b >> 5)] |= 1u << (b & 31);
    }
    const size_t ni = P.instrs.size();
    std::vector<std::vector<uint32_t>> at(ni);
    for (uint64_t d = 0; d < P.n_det; ++d) {
        if (!((tab[d >> 5] >> (d & 31)) & 1u) || P.det_meas[d].empty()) continue;
        int64_t last = -1;
        for (uint32_t t : P.det_meas[d]) last = std::max<int64_t>(last, P.meas_instr[t]);
        if (last < 0 || (size_t)last >= ni) return set_err(SYMFT_EINVAL, "detector record without an instruction");
        at[(size_t)last].push_back((uint32_t)d);
    }
    // chk_off [ni + 1] -> entries; chk_mo [entries + 1] -> measurement ids
    const size_t o_off = tab.size();
    tab.resize(o_off + ni + 1);
    std::vector<uint32_t> mo, ms;
    for (size_t i = 0; i < ni; ++i) {
        tab[o_off + i] = (uint32_t)mo.size();
        for (uint32_t d : at[i]) {
            mo.push_back((uint32_t)ms.size());
            ms.insert(ms.end(), P.det_meas[d].begin(), P.det_meas[d].end());
        }
    }
    tab[o_off + ni] = (uint32_t)mo.size();
    mo.push_back((uint32_t)ms.size());
    const size_t o_mo = tab.size();
    tab.insert(tab.end(), mo.begin(), mo.end());
    const size_t o_ms = tab.size();
    tab.insert(tab.end(), ms.begin(), ms.end());
    tab.push_back(0u);
    int dev = 0;
    if (const hipError_t e = hipGetDevice(&dev)) return hip_err("hipGetDevice failed", e);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        auto key = std::make_pair(dev, tab);
        auto it = h->count_dev.find(key);
        if (it != h->count_dev.end()) {
            base = it->second;
        } else {
            if (hipMalloc(&base, tab.size() * 4) != hipSuccess) return set_err(SYMFT_ENOMEM, "count table allocation failed");
            if (hipMemcpy(base, tab.data(), tab.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
                (void)hipFree(base);
                return set_err(SYMFT_EHIP, "count table upload failed");
            }
            h->count_dev[key] = base;
        }
    }
    if (key_out) *key_out = tab;
    const uint32_t *b = (const uint32_t *)base;
    C.post = b;
    C.obs_exp = b + nd32;
    C.chk_off = b + o_off;
    C.chk_mo = b + o_mo;
    C.chk_meas = b + o_ms;
    C.on = 1;
    return SYMFT_OK;
}

extern "C" {

// Count path 2: the record kernel writes the detector and observable rows of
// every shot to scratch, and a reduction turns them into the flags.  The range
// runs in chunks of kViaRecordsChunk words, so the scratch holds the detector
// and observable rows of one chunk (record rows are never written: the
// kernel's base pointer is set n_rec rows before the scratch).
static constexpr uint32_t kViaRecords = 1u << 20;  // count-tuner choice: path 2
static constexpr uint64_t kViaRecordsChunk = 4096;

static symft_status counts_via_records(symft_program *p, const DevProg &D, bool fp64, uint64_t w0, uint64_t n_words,
                                       uint64_t shots, uint64_t seed, hipStream_t st, const CountArgs &C) {
    const Program &P = p->P;
    const uint64_t ch = std::min<uint64_t>(n_words, kViaRecordsChunk);
    const uint64_t drows = std::max<uint64_t>(1, P.n_det + P.n_obs);
    void *buf = nullptr;
    if (pool_alloc(&buf, (size_t)drows * ch * 8, st) != hipSuccess)
        return set_err(SYMFT_ENOMEM, "count row scratch allocation failed");
    symft_status rc = SYMFT_OK;
    for (uint64_t c0 = 0; c0 < n_words && rc == SYMFT_OK; c0 += ch) {
        const uint64_t cw = std::min(ch, n_words - c0);
        const uint64_t cshots = std::min<uint64_t>(shots - c0 * 64, cw * 64);
        // rows n_rec .. n_rows - 1 of a [n_rows][cw] array whose first n_rec rows are never touched
        uint64_t *base = (uint64_t *)((uintptr_t)buf - (uintptr_t)(P.n_rec * cw * 8));
        rc = run_active(p, D, fp64, w0 + c0, cw, cshots, base, cw, 6u, nullptr, 0, 0, seed, st);
        if (rc == SYMFT_OK) {
            hipError_t e = launch_flags_from_rows((const uint64_t *)buf, cw, cshots, 0, (uint32_t)P.n_det,
                                                  (uint32_t)P.n_obs, C, c0, n_words, st);
            if (e != hipSuccess) rc = set_err(SYMFT_EHIP, std::string("flag reduction launch failed: ") + hipGetErrorString(e));
        }
    }
    (void)hipFreeAsync(buf, st);
    return rc;
}

symft_status symft_sample_counts(const symft_program *pc, const symft_count_opts *opts, uint64_t shots, uint64_t seed,
                                 uint64_t *flags_out, uint64_t *counts_out, void *stream) {
    symft_program *p = const_cast<symft_program *>(pc);
    if (!p) return set_err(SYMFT_EINVAL, "NULL program");
    symft_count_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.shot_offset % 64) return set_err(SYMFT_EINVAL, "shot_offset must be a multiple of 64");
    if (o.precision > 1) return set_err(SYMFT_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
    if (o.n_post && !o.post) return set_err(SYMFT_EINVAL, "post is NULL");
    if (o.threads_per_shot && (o.threads_per_shot & (o.threads_per_shot - 1)))
        return set_err(SYMFT_EINVAL, "threads_per_shot must be a power of two");
    if (o.threads_per_shot && o.threads_per_shot != 1 &&
        (o.threads_per_shot < 4 || (o.threads_per_shot > 256 && o.threads_per_shot != 1024)))
        return set_err(SYMFT_EINVAL, "threads_per_shot must be 1 (the lane kernel), 4 .. 256, or 1024 at peak width >= 13");
    if (o.mode > 2) return set_err(SYMFT_EINVAL, "mode must be 0, 1 or 2");
    CountArgs C;
    std::memset(&C, 0, sizeof(C));
    std::vector<uint32_t> key;
    symft_status rc = count_tables(p, o, C, &key);
    if (rc) return rc;
    if (shots == 0) return SYMFT_OK;
    C.flags = flags_out;
    C.counts = (unsigned long long *)counts_out;
    DevProg D;
    rc = device_prog(p, D);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t w0 = o.shot_offset / 64, n_words = (shots + 63) / 64;
    if (D.fr_ok) return run_frame(p, D, w0, n_words, shots, nullptr, n_words, 0u, seed, 0, st, &C, 0, o.frame_kernel);
    const bool fp64 = o.precision == 0;
    if (D.k_max < 13 && o.threads_per_shot > 256)
        return set_err(SYMFT_EINVAL, "threads_per_shot above 256 needs peak width >= 13");
    uint32_t tps = o.threads_per_shot;
    if (tps == 1) {
        // the lane kernel
        if (!lane_candidate(D, fp64)) return set_err(SYMFT_ECAPACITY, "the lane kernel's state does not fit 64 KB of LDS");
        tps = 1u | kLaneVec;
    }
    uint32_t tuned = 0;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        auto it = p->count_tune.find({key, fp64});
        if (it != p->count_tune.end()) tuned = it->second;
    }
    // a caller's threads_per_shot names the count kernel; only the automatic choice takes the tuned records route
    if (o.mode == 2 || (o.mode == 0 && !o.threads_per_shot && (tuned & kViaRecords)))
        return counts_via_records(p, D, fp64, w0, n_words, shots, seed, st, C);
    if (!tps && !(tuned & kViaRecords)) tps = tuned;
    // untuned: one shot group per workgroup once vectors are wide enough to keep 256 lanes busy
    if (!tps && D.k_max >= 8 && D.k_max < 13 && active_lds_bytes(D, 256, 256, true, fp64) <= kLdsLimit) tps = 256;
    if (D.k_max >= 13 && !narrow_wide(D.k_max)) tps = 0;
    return run_active(p, D, fp64, w0, n_words, shots, nullptr, n_words, 0u, nullptr, 0, 0, seed, st, tps, &C);
}

symft_status symft_autotune_counts(const symft_program *pc, const symft_count_opts *opts, uint32_t *tps_out) {
    symft_program *p = const_cast<symft_program *>(pc);
    if (!p) return set_err(SYMFT_EINVAL, "NULL program");
    symft_count_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.precision > 1) return set_err(SYMFT_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
    if (o.n_post && !o.post) return set_err(SYMFT_EINVAL, "post is NULL");
    CountArgs C;
    std::memset(&C, 0, sizeof(C));
    std::vector<uint32_t> key;
    symft_status rc = count_tables(p, o, C, &key);
    if (rc) return rc;
    DevProg D;
    rc = device_prog(p, D);
    if (rc) return rc;
    const bool fp64 = o.precision == 0;
    if (D.fr_ok || (D.k_max >= 13 && !narrow_wide(D.k_max))) {
        if (tps_out) *tps_out = D.fr_ok ? 0 : 1024;
        return SYMFT_OK;
    }
    // 16384 words up to width 8: on 4096 a lane candidate whose count-mode LDS admits fewer workgroups
    // per CU than the record kernel's ran two passes to the records' one, and the records route won on
    // the sample while losing at full size
    const bool wide = narrow_wide(D.k_max);
    const uint64_t words = wide ? 1024 : D.k_max <= 8 ? 16384 : 4096;
    unsigned long long *cnt = nullptr;
    if (hipMalloc(&cnt, 16) != hipSuccess) return set_err(SYMFT_ENOMEM, "autotune buffer allocation failed");
    C.counts = cnt;
    hipStream_t st;
    if (hipStreamCreate(&st) != hipSuccess) {
        (void)hipFree(cnt);
        return set_err(SYMFT_EHIP, "stream creation failed");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    uint32_t best_tps = 0;
    for (uint32_t cand : {4u, 8u, 16u, 32u, 64u, 128u, 256u, 1024u, 64u | kHbmVec, 128u | kHbmVec, 256u | kHbmVec,
                          1u | kLaneVec}) {
        const uint32_t tps = cand & ~(kHbmVec | kLaneVec);
        if ((cand & kHbmVec) && !hbm_candidate(D.k_max)) continue;
        if ((cand & kLaneVec) && !lane_candidate(D, fp64)) continue;
        if (!(cand & kLaneVec)) {
            if (wide ? tps < 64 : tps > 256) continue;  // widths 13 and 14: 64 .. 256 threads, or 1024
            if (((uint32_t)1 << D.k_max) < tps / 4 && tps > 4) continue;  // most lanes would idle
            if (!wide && !(cand & kHbmVec) && active_lds_bytes(D, 256, tps, true, fp64) > kLdsLimit) continue;
        }
        // the first run warms caches and code; the faster of the next two counts
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && rc == SYMFT_OK; ++rep) {
            (void)hipEventRecord(e0, st);
            rc = run_active(p, D, fp64, 0, words, words * 64, nullptr, words, 0u, nullptr, 0, 0, 0x7E57ull, st, cand, &C);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float t = 0;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (rep) ms = std::min(ms, t);
        }
        if (rc) break;
        if (ms < best) {
            best = ms;
            best_tps = cand;
        }
    }
    // path 2: rows written by the record kernel, then reduced
    if (rc == SYMFT_OK && best_tps) {
        // the first run warms caches and code; the faster of the next two counts
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && rc == SYMFT_OK; ++rep) {
            (void)hipEventRecord(e0, st);
            rc = counts_via_records(p, D, fp64, 0, words, words * 64, 0x7E57ull, st, C);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float t = 0;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (rep) ms = std::min(ms, t);
        }
        if (rc == SYMFT_OK && ms < best) {
            best = ms;
            best_tps = choose_active(D, fp64, 0, 0, false).tps | kViaRecords;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    (void)hipFree(cnt);
    if (rc) return rc;
    if (best_tps) {
        std::lock_guard<std::mutex> lk(p->mu);
        p->count_tune[{key, fp64}] = best_tps;
    }
    if (tps_out) *tps_out = best_tps & ~(kHbmVec | kLaneVec | kViaRecords);
    return SYMFT_OK;
}

symft_status symft_probe(const symft_program *pc, uint64_t shot_begin, uint32_t n_shots, uint64_t seed,
                         uint32_t precision, double *p0_host) {
    symft_program *p = const_cast<symft_program *>(pc);
    if (!p || !p0_host) return set_err(SYMFT_EINVAL, "NULL argument");
    if (precision > 1) return set_err(SYMFT_EINVAL, "precision must be 0 or 1");
    if (n_shots == 0) return SYMFT_OK;
    DevProg D;
    symft_status rc = device_prog(p, D);
    if (rc) return rc;
    const uint64_t w0 = shot_begin / 64, w1 = (shot_begin + n_shots + 63) / 64;
    const uint64_t nw = w1 - w0;
    const size_t nm = std::max<size_t>(1, p->P.n_meas);
    double *dp0 = nullptr;
    uint64_t *drec = nullptr;
    const uint64_t rows = std::max<uint64_t>(1, p->P.n_rows());
    if (hipMalloc(&dp0, sizeof(double) * nm * n_shots) != hipSuccess) return set_err(SYMFT_ENOMEM, "probe allocation failed");
    if (hipMalloc(&drec, 8 * rows * nw) != hipSuccess) {
        (void)hipFree(dp0);
        return set_err(SYMFT_ENOMEM, "probe allocation failed");
    }
    (void)hipMemset(dp0, 0xff, sizeof(double) * nm * n_shots);  // NaN pattern
    rc = run_active(p, D, precision == 0, w0, nw, nw * 64, drec, nw, 7u, dp0, shot_begin, n_shots, seed, nullptr);
    if (rc == SYMFT_OK) {
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(p0_host, dp0, sizeof(double) * nm * n_shots, hipMemcpyDeviceToHost) != hipSuccess)
            rc = set_err(SYMFT_EHIP, "probe copy failed");
    }
    (void)hipFree(dp0);
    (void)hipFree(drec);
    return rc;
}

symft_status symft_probe_amplitudes(const symft_program *pc, uint64_t shot_begin, uint32_t n_shots, uint64_t seed,
                                    uint32_t precision, double *amp_host, uint32_t *k_end) {
    symft_program *p = const_cast<symft_program *>(pc);
    if (!p) return set_err(SYMFT_EINVAL, "NULL program");
    if (precision > 1) return set_err(SYMFT_EINVAL, "precision must be 0 or 1");
    const uint32_t k = p->P.k_after_op.empty() ? 0u : (uint32_t)std::max<int16_t>(0, p->P.k_after_op.back());
    if (k_end) *k_end = k;
    if (n_shots == 0 || !amp_host) return SYMFT_OK;
    if (p->P.k_max == 0) {
        for (uint64_t i = 0; i < n_shots; ++i) {
            amp_host[2 * i] = 1.0;
            amp_host[2 * i + 1] = 0.0;
        }
        return SYMFT_OK;
    }
    DevProg D;
    symft_status rc = device_prog(p, D, true, true);
    if (rc) return rc;
    const uint64_t w0 = shot_begin / 64, w1 = (shot_begin + n_shots + 63) / 64;
    const uint64_t nw = w1 - w0;
    const size_t namp = (size_t)n_shots * (2ull << k);
    double *damp = nullptr;
    uint64_t *drec = nullptr;
    const uint64_t rows = std::max<uint64_t>(1, p->P.n_rows());
    if (hipMalloc(&damp, sizeof(double) * namp) != hipSuccess) return set_err(SYMFT_ENOMEM, "probe allocation failed");
    if (hipMalloc(&drec, 8 * rows * nw) != hipSuccess) {
        (void)hipFree(damp);
        return set_err(SYMFT_ENOMEM, "probe allocation failed");
    }
    rc = run_active(p, D, precision == 0, w0, nw, nw * 64, drec, nw, 7u, nullptr, shot_begin, n_shots, seed, nullptr, 0,
                    nullptr, damp, k);
    if (rc == SYMFT_OK) {
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(amp_host, damp, sizeof(double) * namp, hipMemcpyDeviceToHost) != hipSuccess)
            rc = set_err(SYMFT_EHIP, "probe copy failed");
    }
    (void)hipFree(damp);
    (void)hipFree(drec);
    return rc;
}

symft_status symft_gap_check(uint64_t p32, const uint32_t *v, int32_t *g_out, uint64_t n, void *stream) {
    if (p32 == 0 || p32 > (uint64_t(1) << 32)) return set_err(SYMFT_EINVAL, "p32 must be in (0, 2^32]");
    if (n == 0) return SYMFT_OK;
    if (!v || !g_out) return set_err(SYMFT_EINVAL, "NULL argument");
    std::vector<uint64_t> Q(4097);
    gap_table(p32, Q.data());
    const GapFast F = gap_fast_constants(p32, Q.data());
    uint64_t *dQ = nullptr;
    if (hipMalloc(&dQ, Q.size() * 8) != hipSuccess) return set_err(SYMFT_ENOMEM, "gap table allocation failed");
    hipStream_t st = (hipStream_t)stream;
    symft_status rc = SYMFT_OK;
    if (hipMemcpy(dQ, Q.data(), Q.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        launch_gap_check(F, dQ, v, g_out, n, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        rc = set_err(SYMFT_EHIP, "gap check failed");
    (void)hipFree(dQ);
    return rc;
}

// ------------------------------------------------------------ autotune ----
// Times every threads-per-shot candidate that fits LDS on 4096 words of the
// program and keeps the fastest for (k_max, precision).  Records do not depend on the choice; only
// branch-probability rounding does.
static symft_status tune_program(symft_program *p, const DevProg &D, bool fp64, uint32_t *tps_out) {
    if ((D.k_max >= 13 && !narrow_wide(D.k_max)) || D.fr_ok) {
        if (tps_out) *tps_out = D.k_max >= 13 ? 1024 : 0;
        return SYMFT_OK;
    }
    // widths 13 and 14 run up to 1024 workgroups: time enough words to fill them
    const bool wide = narrow_wide(D.k_max);
    const uint64_t words = wide ? 1024 : 4096;
    uint64_t *out = nullptr;
    const uint64_t rows = std::max<uint64_t>(1, p->P.n_rows());
    if (hipMalloc(&out, 8 * rows * words) != hipSuccess) return set_err(SYMFT_ENOMEM, "autotune buffer allocation failed");
    hipStream_t st;
    if (hipStreamCreate(&st) != hipSuccess) {
        (void)hipFree(out);
        return set_err(SYMFT_EHIP, "stream creation failed");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    uint32_t best_tps = default_tps(D.k_max, fp64);
    symft_status rc = SYMFT_OK;
    const bool hbm_try = hbm_candidate(D.k_max);
    const bool lane_try = lane_candidate(D, fp64);
    for (uint32_t cand : {4u, 8u, 16u, 32u, 64u, 128u, 256u, 1024u, 64u | kHbmVec, 128u | kHbmVec, 256u | kHbmVec,
                          1u | kLaneVec}) {
        const uint32_t tps = cand & ~(kHbmVec | kLaneVec);
        if ((cand & kHbmVec) && !hbm_try) continue;
        if ((cand & kLaneVec) && !lane_try) continue;
        if (!(cand & kLaneVec)) {
            if (wide ? tps < 64 : tps > 256) continue;  // widths 13 and 14: 64 .. 256 threads, or 1024
            if (((uint32_t)1 << D.k_max) < tps / 4 && tps > 4) continue;  // most lanes would idle
            if (!wide && !(cand & kHbmVec) && active_lds_bytes(D, 256, tps, true, fp64) > kLdsLimit) continue;
        }
        // the first run warms caches and code; the faster of the next two counts
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && rc == SYMFT_OK; ++rep) {
            (void)hipEventRecord(e0, st);
            rc = run_active(p, D, fp64, 0, words, words * 64, out, words, 7u, nullptr, 0, 0, 0x7E57ull, st, cand);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float t = 0;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (rep) ms = std::min(ms, t);
        }
        if (rc) break;
        if (ms < best) {
            best = ms;
            best_tps = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    (void)hipFree(out);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[{D.k_max, fp64}] = best_tps;
    }
    if (tps_out) *tps_out = best_tps & ~(kHbmVec | kLaneVec);
    return SYMFT_OK;
}

symft_status symft_autotune(const symft_program *pc, uint32_t precision, uint32_t *tps_out) {
    symft_program *p = const_cast<symft_program *>(pc);
    if (!p) return set_err(SYMFT_EINVAL, "NULL program");
    if (precision > 1) return set_err(SYMFT_EINVAL, "precision must be 0 or 1");
    DevProg D;
    symft_status rc = device_prog(p, D);
    if (rc) return rc;
    return tune_program(p, D, precision == 0, tps_out);
}

// ------------------------------------------------------------- batching ----
struct BatchPlan {
    std::vector<const symft_program *> progs;
    std::vector<uint64_t> serials;  // progs' serial numbers (an address alone may be reused)
    std::vector<uint64_t> shots, seeds;
    std::vector<uint64_t *> outs;
    uint32_t precision = 0;
    int device = 0;
    ActiveArgs *d_calls = nullptr;
    BatchItem *d_items = nullptr;
    uint32_t *d_counter = nullptr;
    BatchArgs args;
    uint32_t grid = 0, lds = 0;
    // members on the lane kernel: queues of one-wave workgroups by LDS class (queue q counts at
    // d_counter + 16 (q + 1))
    struct LaneQueue {
        ActiveArgs *d_calls = nullptr;
        BatchItem *d_items = nullptr;
        BatchArgs args;
        uint32_t grid = 0, lds = 0;
    };
    std::vector<LaneQueue> lq;
    std::vector<size_t> others;  // programs sampled by their own launches
    // aggregate-count plans: the count tables' contents and the counters, compared with sig
    bool cm = false;
    std::vector<uint64_t> sig;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    bool same(const symft_program *const *p, const uint64_t *sh, const uint64_t *sd, uint64_t *const *o, size_t n,
              uint32_t prec, int dev) const {
        if (cm || n != progs.size() || prec != precision || dev != device) return false;
        for (size_t i = 0; i < n; ++i)
            if (p[i] != progs[i] || (p[i] && p[i]->serial != serials[i]) || sh[i] != shots[i] || sd[i] != seeds[i] ||
                o[i] != outs[i])
                return false;
        return true;
    }
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipFree(d_calls);
        (void)hipFree(d_items);
        (void)hipFree(d_counter);
        for (LaneQueue &q : lq) {
            (void)hipFree(q.d_calls);
            (void)hipFree(q.d_items);
        }
        lq.clear();
        exec = nullptr;
        graph = nullptr;
        d_calls = nullptr;
        d_items = nullptr;
        d_counter = nullptr;

    }
};

static std::mutex g_batch_mu;
static std::vector<BatchPlan *> g_plans;  // most recent first, a few kept

static void drop_batch_plans(const symft_program *p) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (size_t i = 0; i < g_plans.size();) {
        BatchPlan *B = g_plans[i];
        bool holds = false;
        for (size_t k = 0; k < B->progs.size(); ++k) holds |= B->progs[k] == p && B->serials[k] == p->serial;
        if (holds) {
            B->release();
            delete B;
            g_plans.erase(g_plans.begin() + (ptrdiff_t)i);
        } else {
            ++i;
        }
    }
}

// cnt (count plans): per program its count tables, flags and counters, and
// its first word; outs is then unused.
static symft_status build_plan(BatchPlan &B, const symft_program *const *progs, const uint64_t *shots,
                               const uint64_t *seeds, uint64_t *const *outs, size_t n, uint32_t precision,
                               const CountArgs *cnt = nullptr, const uint64_t *word0 = nullptr,
                               uint64_t budget = kBatchBudgets[0]) {
    const bool fp64 = precision == 0;
    B.cm = cnt != nullptr;
    B.progs.assign(progs, progs + n);
    B.serials.resize(n);
    for (size_t i = 0; i < n; ++i) B.serials[i] = progs[i] ? progs[i]->serial : 0;
    B.shots.assign(shots, shots + n);
    B.seeds.assign(seeds, seeds + n);
    if (!cnt) B.outs.assign(outs, outs + n);
    B.precision = precision;
    (void)hipGetDevice(&B.device);
    std::vector<ActiveArgs> calls;
    std::vector<double> cost;
    std::vector<uint64_t> words_of;
    size_t lds = 0;
    // lane members by LDS class: the queue's LDS is its largest member's, which sets its occupancy
    constexpr int kClasses = 4;
    const size_t kLaneClass[kClasses] = {8 * 1024, 16 * 1024, 24 * 1024, lane_batch_cap(fp64)};
    std::vector<ActiveArgs> lcalls[kClasses];
    std::vector<double> lcost[kClasses];
    std::vector<uint64_t> lwords_of[kClasses];
    size_t llds[kClasses] = {0, 0, 0, 0};
    for (size_t i = 0; i < n; ++i) {
        symft_program *p = const_cast<symft_program *>(progs[i]);
        if (!p || (!cnt && shots[i] && !outs[i])) return set_err(SYMFT_EINVAL, "NULL program or output in batch");
        DevProg D;
        symft_status rc = device_prog(p, D);
        if (rc) return rc;
        bool mine = shots[i] > 0 && !D.fr_ok;
        symft_info info;
        symft_program_info(p, &info);
        uint64_t n_instr = 0;
        for (uint64_t v : info.n_instr) n_instr += v;
        // estimated cost per word: the representation's flops and a per-instruction share
        const double wcost =
            (info.product_selected ? info.product_flops_per_shot : info.dense_flops_per_shot) + 200.0 * (double)n_instr + 64.0;
        if (mine && lane_candidate(D, fp64) && lane_lds_bytes(D, fp64) <= lane_batch_cap(fp64)) {
            // the lane kernel, in a queue of its own
            ActiveArgs A;
            std::memset(&A, 0, sizeof(A));
            A.P = D;
            A.seed = seeds[i];
            A.word_begin = word0 ? word0[i] : 0;
            A.n_words = (shots[i] + 63) / 64;
            A.shots = shots[i];
            A.out = cnt ? nullptr : outs[i];
            A.row_stride = A.n_words;
            A.sections = cnt ? 0u : 7u;
            if (cnt) A.cnt = cnt[i];
            A.tps = 1;
            A.lds_vec = 1;
            A.lds_bytes = (uint32_t)lane_lds_bytes(D, fp64);
            int q = 0;
            while (A.lds_bytes > kLaneClass[q]) ++q;
            llds[q] = std::max<size_t>(llds[q], A.lds_bytes);
            lcalls[q].push_back(A);
            lwords_of[q].push_back(A.n_words);
            lcost[q].push_back(wcost);
            continue;
        }
        ActiveConfig c;
        if (mine) {
            c = choose_active(D, fp64, 0, budget);
            mine = c.bs == 256 && c.lds_vec;
        }
        if (!mine) {
            if (shots[i]) B.others.push_back(i);
            continue;
        }
        ActiveArgs A;
        std::memset(&A, 0, sizeof(A));
        A.P = D;
        A.seed = seeds[i];
        A.word_begin = word0 ? word0[i] : 0;
        A.n_words = (shots[i] + 63) / 64;
        A.shots = shots[i];
        A.out = cnt ? nullptr : outs[i];
        A.row_stride = A.n_words;
        A.sections = cnt ? 0u : 7u;
        if (cnt) A.cnt = cnt[i];
        A.tps = c.tps;
        A.lds_vec = 1;
        A.lds_bytes = (uint32_t)c.lds;
        lds = std::max(lds, c.lds);
        calls.push_back(A);
        words_of.push_back(A.n_words);
        cost.push_back(wcost);
    }
    // the shot-group queue's counter and one per lane class, 64 bytes apart
    if (hipMalloc(&B.d_counter, sizeof(uint32_t) * 16 * (kClasses + 1)) != hipSuccess)
        return set_err(SYMFT_ENOMEM, "batch metadata allocation failed");
    for (int q = 0; q < kClasses; ++q) {
        if (lcalls[q].empty()) continue;
        // items of a few words for one-wave workgroups, by decreasing cost
        BatchPlan::LaneQueue Q;
        const int per_cu = std::max(1, lane_batch_max_blocks_per_cu(fp64, llds[q], B.cm));
        Q.grid = (uint32_t)(per_cu * num_cus());
        uint64_t total_words = 0;
        for (uint64_t w : lwords_of[q]) total_words += w;
        const uint64_t chunk = std::max<uint64_t>(1, std::min<uint64_t>(16, total_words / ((uint64_t)Q.grid * 4) + 1));
        std::vector<std::pair<double, BatchItem>> tmp;
        for (size_t ci = 0; ci < lcalls[q].size(); ++ci)
            for (uint64_t w0 = 0; w0 < lwords_of[q][ci]; w0 += chunk) {
                BatchItem it;
                it.call = (uint32_t)ci;
                it.pad = 0;
                it.w0 = w0;
                it.w1 = std::min(lwords_of[q][ci], w0 + chunk);
                tmp.push_back({lcost[q][ci] * (double)(it.w1 - it.w0), it});
            }
        std::stable_sort(tmp.begin(), tmp.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
        std::vector<BatchItem> litems;
        for (auto &x : tmp) litems.push_back(x.second);
        Q.grid = (uint32_t)std::min<uint64_t>(Q.grid, litems.size());
        Q.lds = (uint32_t)llds[q];
        B.lq.push_back(Q);
        BatchPlan::LaneQueue &R = B.lq.back();
        if (hipMalloc(&R.d_calls, sizeof(ActiveArgs) * lcalls[q].size()) != hipSuccess ||
            hipMalloc(&R.d_items, sizeof(BatchItem) * litems.size()) != hipSuccess)
            return set_err(SYMFT_ENOMEM, "batch metadata allocation failed");
        if (hipMemcpy(R.d_calls, lcalls[q].data(), sizeof(ActiveArgs) * lcalls[q].size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(R.d_items, litems.data(), sizeof(BatchItem) * litems.size(), hipMemcpyHostToDevice) != hipSuccess)
            return set_err(SYMFT_EHIP, "batch metadata upload failed");
        R.args.calls = R.d_calls;
        R.args.items = R.d_items;
        R.args.counter = B.d_counter + 16 * B.lq.size();
        R.args.n_items = (uint32_t)litems.size();
        R.args.pad = 0;
    }
    std::vector<BatchItem> items;
    if (!calls.empty()) {
        int per_cu = std::max(1, batch_max_blocks_per_cu(fp64, B.cm, lds));
        B.grid = (uint32_t)(per_cu * num_cus());
        uint64_t total_words = 0;
        for (uint64_t w : words_of) total_words += w;
        // about eight items per workgroup; an item never splits a word
        const uint64_t chunk = std::max<uint64_t>(1, std::min<uint64_t>(64, total_words / ((uint64_t)B.grid * 8) + 1));
        std::vector<std::pair<double, BatchItem>> tmp;
        for (size_t ci = 0; ci < calls.size(); ++ci)
            for (uint64_t w0 = 0; w0 < words_of[ci]; w0 += chunk) {
                BatchItem it;
                it.call = (uint32_t)ci;
                it.pad = 0;
                it.w0 = w0;
                it.w1 = std::min(words_of[ci], w0 + chunk);
                tmp.push_back({cost[ci] * (double)(it.w1 - it.w0), it});
            }
        std::stable_sort(tmp.begin(), tmp.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
        for (auto &x : tmp) items.push_back(x.second);
        B.grid = (uint32_t)std::min<uint64_t>(B.grid, items.size());
        B.lds = (uint32_t)lds;
        if (hipMalloc(&B.d_calls, sizeof(ActiveArgs) * calls.size()) != hipSuccess ||
            hipMalloc(&B.d_items, sizeof(BatchItem) * items.size()) != hipSuccess)
            return set_err(SYMFT_ENOMEM, "batch metadata allocation failed");
        if (hipMemcpy(B.d_calls, calls.data(), sizeof(ActiveArgs) * calls.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(B.d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess)
            return set_err(SYMFT_EHIP, "batch metadata upload failed");
    }
    B.args.calls = B.d_calls;
    B.args.items = B.d_items;
    B.args.counter = B.d_counter;
    B.args.n_items = (uint32_t)items.size();
    B.args.pad = 0;
    return SYMFT_OK;
}

// The plan's persistent kernel (after its counter reset), launched directly or
// through its captured graph.
// The plan's launches: the lane members' queues (by LDS class), then the shot-group members'.
static hipError_t launch_plan(BatchPlan &B, bool fp64, hipStream_t st) {
    hipError_t e = hipSuccess;
    for (const BatchPlan::LaneQueue &q : B.lq)
        if (e == hipSuccess && q.args.n_items) e = launch_lane_batch(q.args, fp64, B.cm, q.grid, q.lds, st);
    if (e == hipSuccess && B.args.n_items) e = launch_batch(B.args, fp64, B.cm, B.grid, B.lds, st);
    return e;
}

static symft_status run_plan(BatchPlan &B, bool fp64, uint32_t graph, hipStream_t st) {
    if (!B.args.n_items && B.lq.empty()) return SYMFT_OK;
    if (graph) {
        if (!B.exec) {
            // capture [counter resets, persistent kernels] once on a private stream
            hipStream_t cs;
            if (hipStreamCreate(&cs) != hipSuccess) return set_err(SYMFT_EHIP, "stream creation failed");
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) e = launch_plan(B, fp64, cs);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&B.exec, g, nullptr, nullptr, 0);
            B.graph = g;
            (void)hipStreamDestroy(cs);
            if (e != hipSuccess) return set_err(SYMFT_EHIP, std::string("batch graph capture failed: ") + hipGetErrorString(e));
        }
        hipError_t e = hipGraphLaunch(B.exec, st);
        if (e != hipSuccess) return set_err(SYMFT_EHIP, std::string("batch graph launch failed: ") + hipGetErrorString(e));
    } else {
        hipError_t e = launch_plan(B, fp64, st);
        if (e != hipSuccess) return set_err(SYMFT_EHIP, std::string("batch kernel launch failed: ") + hipGetErrorString(e));
    }
    return SYMFT_OK;
}

// Two direct launches of a plan on stream st; *ms is the second one's time.
static symft_status time_plan(BatchPlan &B, bool fp64, hipStream_t st, float *ms) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_err(SYMFT_EHIP, "event creation failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_err(SYMFT_EHIP, "event creation failed");
    }
    symft_status rc = run_plan(B, fp64, 0, st);
    if (rc == SYMFT_OK) (void)hipEventRecord(e0, st);
    if (rc == SYMFT_OK) rc = run_plan(B, fp64, 0, st);
    if (rc == SYMFT_OK) {
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            rc = set_err(SYMFT_EHIP, "batch timing failed");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// A new plan at the front of the cache, which keeps the four most recent.
static void keep_plan(BatchPlan *B) {
    g_plans.insert(g_plans.begin(), B);
    while (g_plans.size() > 4) {
        g_plans.back()->release();
        delete g_plans.back();
        g_plans.pop_back();
    }
}

symft_status symft_sample_batch(const symft_program *const *progs, const uint64_t *shots, const uint64_t *seeds,
                                uint64_t *const *records_out, size_t n, uint32_t precision, uint32_t graph,
                                void *stream) {
    if (n == 0) return SYMFT_OK;
    if (!progs || !shots || !seeds || !records_out) return set_err(SYMFT_EINVAL, "NULL argument");
    if (precision > 1) return set_err(SYMFT_EINVAL, "precision must be 0 or 1");
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchPlan *B = nullptr;
    for (size_t i = 0; i < g_plans.size(); ++i)
        if (g_plans[i]->same(progs, shots, seeds, records_out, n, precision, dev)) {
            B = g_plans[i];
            break;
        }
    if (!B) {
        // Plans for both LDS budgets; when they differ, each runs twice on the
        // caller's stream (its records are the batch's own, rewritten by the
        // launch below) and the faster second run is kept.
        float best_ms = 0;
        for (uint64_t budget : kBatchBudgets) {
            BatchPlan *C = new BatchPlan();
            symft_status rc = build_plan(*C, progs, shots, seeds, records_out, n, precision, nullptr, nullptr, budget);
            if (rc || (B && C->lds == B->lds)) {
                C->release();
                delete C;
                if (rc) {
                    if (B) {
                        B->release();
                        delete B;
                    }
                    return rc;
                }
                continue;
            }
            if (B) {
                if (!best_ms) {
                    // time the first plan now that there is a second to compare with
                    rc = time_plan(*B, precision == 0, st, &best_ms);
                    if (rc) return rc;
                }
                float ms = 0;
                rc = time_plan(*C, precision == 0, st, &ms);
                if (rc) {
                    C->release();
                    delete C;
                    B->release();
                    delete B;
                    return rc;
                }
                if (ms < best_ms) {
                    std::swap(B, C);
                    best_ms = ms;
                }
                C->release();
                delete C;
            } else {
                B = C;
            }
        }
        keep_plan(B);
    }
    const symft_status rc = run_plan(*B, precision == 0, graph, st);
    if (rc) return rc;
    for (size_t i : B->others) {
        symft_sample_opts o;
        std::memset(&o, 0, sizeof(o));
        o.precision = precision;
        symft_status rc = symft_sample_ex(progs[i], &o, shots[i], seeds[i], records_out[i], stream);
        if (rc) return rc;
    }
    return SYMFT_OK;
}

symft_status symft_sample_counts_batch(const symft_program *const *progs, const uint64_t *shots, const uint64_t *seeds,
                                       const symft_count_opts *opts, uint64_t *const *flags_out, uint64_t *counts_out,
                                       size_t n, uint32_t precision, uint32_t graph, void *stream) {
    if (n == 0) return SYMFT_OK;
    if (!progs || !shots || !seeds) return set_err(SYMFT_EINVAL, "NULL argument");
    if (precision > 1) return set_err(SYMFT_EINVAL, "precision must be 0 or 1");
    std::vector<CountArgs> cnt(n);
    std::vector<uint64_t> word0(n, 0);
    std::vector<uint64_t> sig;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    (void)hipGetDevice(&dev);
    sig.push_back(n);
    sig.push_back(precision);
    sig.push_back((uint64_t)dev);
    for (size_t i = 0; i < n; ++i) {
        symft_program *p = const_cast<symft_program *>(progs[i]);
        if (!p) return set_err(SYMFT_EINVAL, "NULL program in batch");
        symft_count_opts o;
        std::memset(&o, 0, sizeof(o));
        if (opts) o = opts[i];
        if (o.shot_offset % 64) return set_err(SYMFT_EINVAL, "shot_offset must be a multiple of 64");
        if (o.n_post && !o.post) return set_err(SYMFT_EINVAL, "post is NULL");
        std::memset(&cnt[i], 0, sizeof(CountArgs));
        std::vector<uint32_t> key;
        symft_status rc = count_tables(p, o, cnt[i], &key);
        if (rc) return rc;
        cnt[i].flags = flags_out ? flags_out[i] : nullptr;
        cnt[i].counts = counts_out ? (unsigned long long *)(counts_out + 2 * i) : nullptr;
        word0[i] = o.shot_offset / 64;
        sig.insert(sig.end(), {(uint64_t)(uintptr_t)p, p->serial, shots[i], seeds[i],
                               (uint64_t)(uintptr_t)cnt[i].flags, (uint64_t)(uintptr_t)cnt[i].counts, word0[i],
                               (uint64_t)key.size()});
        sig.insert(sig.end(), key.begin(), key.end());
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchPlan *B = nullptr;
    for (size_t i = 0; i < g_plans.size(); ++i)
        if (g_plans[i]->cm && g_plans[i]->sig == sig) {
            B = g_plans[i];
            break;
        }
    if (!B) {
        B = new BatchPlan();
        symft_status rc = build_plan(*B, progs, shots, seeds, nullptr, n, precision, cnt.data(), word0.data());
        if (rc) {
            B->release();
            delete B;
            return rc;
        }
        B->sig = sig;
        keep_plan(B);
    }
    const symft_status rc = run_plan(*B, precision == 0, graph, st);
    if (rc) return rc;
    for (size_t i : B->others) {
        symft_count_opts o;
        std::memset(&o, 0, sizeof(o));
        if (opts) o = opts[i];
        o.precision = precision;
        symft_status r2 = symft_sample_counts(progs[i], &o, shots[i], seeds[i], flags_out ? flags_out[i] : nullptr,
                                              counts_out ? counts_out + 2 * i : nullptr, stream);
        if (r2) return r2;
    }
    return SYMFT_OK;
}

}  // extern "C"
