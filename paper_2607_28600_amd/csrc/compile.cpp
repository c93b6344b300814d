// compile.cpp -- one host pass: symbolic Clifford-Pauli frame factorization
// (paper Sec. 3) interleaved with adaptive stabilizer-coordinate planning
// (paper Sec. 4), emitting the seven sampling instructions (Sec. 5).
//
// Frames.  The Clifford frame C is kept as the inverse images C^dag X_q C and
// C^dag Z_q C (signed Paulis), so pulling a Pauli back is a product of
// images.  The symbolic Pauli frame E is kept per qubit as two affine
// expressions EX_q, EZ_q (bitsets over symbols): the sign a frame factor F^e
// puts on a pulled-back Pauli Q is omega(F, Q) e, and omega is bilinear in
// the symplectic bits, so lambda(Q) = XOR_{q: Q.z_q} EX_q  XOR_{q: Q.x_q} EZ_q.
// A noise channel contributes one symbol per nonzero (qubit, x|z) component
// of its branches (the chosen Pauli's symplectic bits); a branch is then a bit
// pattern over those symbols.  The planner's symbolic corrections after a
// measurement (paper Sec. 4.2) are Pauli factors raised to an affine
// expression and enter the same frame, since they act on every later
// pulled-back operation exactly like a frame factor.
//
// Planner.  A signed stabilizer-destabilizer tableau over the pulled-back
// frame, first k coordinates active.  Pivot rules: the lowest dormant
// coordinate whose Zbar anticommutes with P (swapped to position k for a
// promotion); the highest set bit of a for pair instructions; the highest set
// bit of b for active-diagonal measurements; after an active measurement the
// pivot pair becomes the first dormant coordinate.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/symft.h"
#include "program.hpp"

namespace symft {
namespace {

// ---------------------------------------------------------------- Paulis --
struct PauliV {
    std::vector<uint64_t> x, z;
    int e = 0;  // i^e X^x Z^z
    explicit PauliV(int W = 0) : x(W, 0), z(W, 0) {}
};

inline int popc(uint64_t v) { return __builtin_popcountll(v); }

inline int anti(const PauliV &a, const PauliV &b) {
    int s = 0;
    for (size_t i = 0; i < a.x.size(); ++i) s += popc(a.x[i] & b.z[i]) + popc(a.z[i] & b.x[i]);
    return s & 1;
}

// a <- a * b
inline void rmul(PauliV &a, const PauliV &b) {
    int s = 0;
    for (size_t i = 0; i < a.x.size(); ++i) s += popc(a.z[i] & b.x[i]);
    a.e = (a.e + b.e + 2 * (s & 1)) & 3;
    for (size_t i = 0; i < a.x.size(); ++i) {
        a.x[i] ^= b.x[i];
        a.z[i] ^= b.z[i];
    }
}

inline bool bit(const std::vector<uint64_t> &v, uint32_t q) { return (v[q >> 6] >> (q & 63)) & 1u; }

// ------------------------------------------------------------- bitsets ---
struct Bits {
    std::vector<uint64_t> w;
    void init(size_t nbits) { w.assign((nbits + 63) / 64, 0); }
    void flip(uint32_t i) { w[i >> 6] ^= uint64_t(1) << (i & 63); }
    void xor_in(const Bits &o) {
        for (size_t i = 0; i < w.size(); ++i) w[i] ^= o.w[i];
    }
    void clear() { std::fill(w.begin(), w.end(), 0); }
};

struct Compiler {
    uint32_t n = 0, W = 0;
    // symbol space: 0 = constant 1, [1, 1+Nn) noise, [1+Nn, 1+Nn+M) measurements
    uint32_t Nn = 0, M = 0, S = 0;
    std::vector<PauliV> imgX, imgZ;  // C^dag X_q C, C^dag Z_q C
    std::vector<Bits> EX, EZ;        // symbolic frame per qubit
    std::vector<PauliV> Zb, Xb;      // planner tableau
    int k = 0;
    Program *P = nullptr;
    std::string err;

    uint32_t sym_meas(uint32_t t) const { return 1 + Nn + t; }

    void init_frames() {
        W = (n + 63) / 64;
        imgX.assign(n, PauliV(W));
        imgZ.assign(n, PauliV(W));
        Zb.assign(n, PauliV(W));
        Xb.assign(n, PauliV(W));
        for (uint32_t q = 0; q < n; ++q) {
            imgX[q].x[q >> 6] |= uint64_t(1) << (q & 63);
            imgZ[q].z[q >> 6] |= uint64_t(1) << (q & 63);
            Zb[q].z[q >> 6] |= uint64_t(1) << (q & 63);
            Xb[q].x[q >> 6] |= uint64_t(1) << (q & 63);
        }
        rel_of.assign(S, {});
        EX.resize(n);
        EZ.resize(n);
        for (uint32_t q = 0; q < n; ++q) {
            EX[q].init(S);
            EZ[q].init(S);
        }
    }

    // ------------------------------------------------- Clifford frame ---
    // C_t = g C_{t-1}: new image of P is the old image of g^dag P g.
    void gate1(uint32_t kind, uint32_t q) {
        switch (kind) {
        case SYMFT_OP_H: std::swap(imgX[q], imgZ[q]); break;
        case SYMFT_OP_S: {  // S^dag X S = -i X Z
            PauliV t = imgX[q];
            rmul(t, imgZ[q]);
            t.e = (t.e + 3) & 3;
            imgX[q] = t;
            break;
        }
        case SYMFT_OP_S_DAG: {  // S X S^dag = i X Z
            PauliV t = imgX[q];
            rmul(t, imgZ[q]);
            t.e = (t.e + 1) & 3;
            imgX[q] = t;
            break;
        }
        case SYMFT_OP_X: imgZ[q].e = (imgZ[q].e + 2) & 3; break;
        case SYMFT_OP_Y:
            imgX[q].e = (imgX[q].e + 2) & 3;
            imgZ[q].e = (imgZ[q].e + 2) & 3;
            break;
        case SYMFT_OP_Z: imgX[q].e = (imgX[q].e + 2) & 3; break;
        default: break;
        }
    }
    void gate2(uint32_t kind, uint32_t a, uint32_t b) {
        switch (kind) {
        case SYMFT_OP_CX:  // X_a -> X_a X_b, Z_b -> Z_a Z_b
            rmul(imgX[a], imgX[b]);
            {
                PauliV t = imgZ[a];
                rmul(t, imgZ[b]);
                imgZ[b] = t;
            }
            break;
        case SYMFT_OP_CZ: {  // X_a -> X_a Z_b, X_b -> Z_a X_b
            PauliV xa = imgX[a];
            rmul(xa, imgZ[b]);
            PauliV xb = imgZ[a];
            rmul(xb, imgX[b]);
            imgX[a] = xa;
            imgX[b] = xb;
            break;
        }
        case SYMFT_OP_SWAP:
            std::swap(imgX[a], imgX[b]);
            std::swap(imgZ[a], imgZ[b]);
            break;
        default: break;
        }
    }
    // C^dag P C for P = (-1)^neg prod letters
    PauliV pull_back(const uint32_t *qs, const uint8_t *lets, uint32_t cnt, bool neg) {
        PauliV r(W);
        int e = neg ? 2 : 0;
        for (uint32_t j = 0; j < cnt; ++j)
            if (lets[j] == 2) e += 1;  // Y = i X Z
        r.e = e & 3;
        for (uint32_t j = 0; j < cnt; ++j)
            if (lets[j] == 1 || lets[j] == 2) rmul(r, imgX[qs[j]]);
        for (uint32_t j = 0; j < cnt; ++j)
            if (lets[j] == 2 || lets[j] == 3) rmul(r, imgZ[qs[j]]);
        return r;
    }

    // ----------------------------------------------- symbolic frame -----
    void frame_add_symbol(const PauliV &F, uint32_t sym) {
        for (uint32_t q = 0; q < n; ++q) {
            if (bit(F.x, q)) EX[q].flip(sym);
            if (bit(F.z, q)) EZ[q].flip(sym);
        }
    }
    void frame_add_expr(const PauliV &F, const Bits &e) {
        for (uint32_t q = 0; q < n; ++q) {
            if (bit(F.x, q)) EX[q].xor_in(e);
            if (bit(F.z, q)) EZ[q].xor_in(e);
        }
    }
    void lambda_of(const PauliV &Q, Bits &out) {
        out.clear();
        for (uint32_t q = 0; q < n; ++q) {
            if (bit(Q.z, q)) out.xor_in(EX[q]);
            if (bit(Q.x, q)) out.xor_in(EZ[q]);
        }
    }
    void to_expr(const Bits &b, Expr &e) {
        e.c = 0;
        e.noise.clear();
        e.meas.clear();
        for (size_t i = 0; i < b.w.size(); ++i) {
            uint64_t v = b.w[i];
            while (v) {
                uint32_t id = uint32_t(i * 64 + __builtin_ctzll(v));
                v &= v - 1;
                if (id == 0) e.c = 1;
                else if (id <= Nn) e.noise.push_back(id - 1);
                else e.meas.push_back(id - 1 - Nn);
            }
        }
    }

    // ------------------------------------- relative sign expressions -----
    // Every deterministic measurement t gives the identity
    //     lambda_t ^ m_t ^ eta_t = 0
    // over the symbols, so XOR-ing it into a later sign expression leaves the
    // expression's value unchanged.  A greedy pass rewrites each new sign
    // relative to earlier records this way while that lowers its weight, which
    // keeps signs local (paper Sec. 6: exogenous/causal split and shared
    // partial expressions).
    std::vector<std::vector<uint32_t>> rel;     // symbol ids of each identity (0 = constant)
    std::vector<std::vector<uint32_t>> rel_of;  // symbol id -> identities containing it
    std::vector<int> cnt;
    std::vector<uint32_t> touched;

    void add_relation(const Bits &lam, uint32_t t, int eta) {
        std::vector<uint32_t> ids;
        for (size_t i = 0; i < lam.w.size(); ++i) {
            uint64_t v = lam.w[i];
            while (v) {
                ids.push_back(uint32_t(i * 64 + __builtin_ctzll(v)));
                v &= v - 1;
            }
        }
        auto toggle = [&](uint32_t id) {
            auto it = std::lower_bound(ids.begin(), ids.end(), id);
            if (it != ids.end() && *it == id) ids.erase(it);
            else ids.insert(it, id);
        };
        toggle(sym_meas(t));
        if (eta) toggle(0);
        const uint32_t r = (uint32_t)rel.size();
        for (uint32_t id : ids)
            if (id) rel_of[id].push_back(r);
        rel.push_back(std::move(ids));
        cnt.push_back(0);
    }

    void reduce(Bits &lam) {
        auto has = [&](uint32_t id) { return (lam.w[id >> 6] >> (id & 63)) & 1u; };
        int w = 0;
        for (size_t i = 0; i < lam.w.size(); ++i) w += popc(lam.w[i]);
        w -= (int)has(0);
        for (int iter = 0; iter < 256; ++iter) {
            touched.clear();
            for (size_t i = 0; i < lam.w.size(); ++i) {
                uint64_t v = lam.w[i];
                while (v) {
                    uint32_t id = uint32_t(i * 64 + __builtin_ctzll(v));
                    v &= v - 1;
                    if (!id) continue;
                    for (uint32_t r : rel_of[id]) {
                        if (cnt[r]++ == 0) touched.push_back(r);
                    }
                }
            }
            int best = -1, best_w = w;
            for (uint32_t r : touched) {
                int len = (int)rel[r].size() - (rel[r][0] == 0 ? 1 : 0);
                int nw = w + len - 2 * cnt[r];
                if (nw < best_w || (nw == best_w && best >= 0 && r > (uint32_t)best)) {
                    if (nw < w) { best = (int)r; best_w = nw; }
                }
            }
            for (uint32_t r : touched) cnt[r] = 0;
            if (best < 0) break;
            for (uint32_t id : rel[best]) lam.flip(id);
            w = best_w;
        }
    }

    // ------------------------------------------------------- planner ----
    struct Dec {
        std::vector<uint8_t> zc, xc;  // omega with Zbar_j, Xbar_j
        uint32_t a = 0, b = 0;
        bool d = false;
        int mu = 0;  // P = i^mu Xbar_A^a Zbar_A^b Xbar_D^d Zbar_D^c
    };
    Dec decompose(const PauliV &Pq) {
        Dec D;
        D.zc.assign(n, 0);
        D.xc.assign(n, 0);
        PauliV r(W);
        for (uint32_t j = 0; j < n; ++j) {
            D.zc[j] = (uint8_t)anti(Pq, Zb[j]);
            D.xc[j] = (uint8_t)anti(Pq, Xb[j]);
            if ((int)j < k) {
                if (D.zc[j]) D.a |= 1u << j;
                if (D.xc[j]) D.b |= 1u << j;
            } else if (D.zc[j]) {
                D.d = true;
            }
        }
        for (int j = 0; j < k; ++j)
            if (D.zc[j]) rmul(r, Xb[j]);
        for (int j = 0; j < k; ++j)
            if (D.xc[j]) rmul(r, Zb[j]);
        for (uint32_t j = k; j < n; ++j)
            if (D.zc[j]) rmul(r, Xb[j]);
        for (uint32_t j = k; j < n; ++j)
            if (D.xc[j]) rmul(r, Zb[j]);
        D.mu = (Pq.e - r.e) & 3;
        return D;
    }
    int lowest_dormant(const Dec &D) {
        for (uint32_t j = k; j < n; ++j)
            if (D.zc[j]) return (int)j;
        return -1;
    }
    // every generator except the pivot pair that anticommutes with P takes a factor G
    void pivot_update(const Dec &D, int h, const PauliV &G) {
        for (uint32_t j = 0; j < n; ++j) {
            if ((int)j == h) continue;
            if (D.zc[j]) rmul(Zb[j], G);
            if (D.xc[j]) rmul(Xb[j], G);
        }
    }
    void swap_pair(int i, int j) {
        if (i == j) return;
        std::swap(Zb[i], Zb[j]);
        std::swap(Xb[i], Xb[j]);
    }
    void move_pair(int h, int dst) {
        for (int j = h; j < dst; ++j) swap_pair(j, j + 1);
    }

    void emit(Instr in) { P->instrs.push_back(std::move(in)); }

    void plan_rotation(const PauliV &Q, Bits &lam, double theta, int op) {
        reduce(lam);
        Dec D = decompose(Q);
        Instr in;
        in.theta = theta;
        in.k_in = (uint8_t)k;
        in.op = op;
        to_expr(lam, in.lam);
        if (D.d) {
            int h = lowest_dormant(D);
            PauliV Zh = Zb[h];
            pivot_update(D, h, Zh);
            Xb[h] = Q;
            swap_pair(h, k);
            in.kind = PROMOTE_ROT;
            k += 1;
            P->rot_kind[op] = 1;
            emit(std::move(in));
        } else if (D.a == 0 && D.b == 0) {
            P->rot_kind[op] = 0;  // global phase: no instruction
        } else if (D.a == 0) {
            in.kind = ACTIVE_DIAG_ROT;
            in.b = D.b;
            in.mu = (uint8_t)D.mu;
            P->rot_kind[op] = 2;
            emit(std::move(in));
        } else {
            in.kind = ACTIVE_PAIR_ROT;
            in.a = D.a;
            in.b = D.b;
            in.mu = (uint8_t)D.mu;
            in.h = (uint8_t)(31 - __builtin_clz(D.a));
            P->rot_kind[op] = 3;
            emit(std::move(in));
        }
        if ((uint32_t)k > P->k_max) P->k_max = (uint32_t)k;
    }

    // measurement t of pulled-back Q with sign expression lam
    void plan_measurement(const PauliV &Q, Bits &lam, uint32_t t, int op) {
        Bits raw = lam;
        reduce(lam);
        Dec D = decompose(Q);
        Instr in;
        in.k_in = (uint8_t)k;
        in.meas = (int32_t)t;
        in.op = op;
        to_expr(lam, in.lam);
        Bits corr;  // correction exponent m_t + lam (+ eta)
        if (D.d) {
            int h = lowest_dormant(D);
            PauliV Zh = Zb[h];
            pivot_update(D, h, Zh);
            Xb[h] = Zh;
            Zb[h] = Q;
            in.kind = RANDOM_MEAS;
            corr = lam;
            corr.flip(sym_meas(t));
            frame_add_expr(Xb[h], corr);
            P->meas_kind[t] = 0;
        } else if (D.a == 0 && D.b == 0) {
            in.kind = DET_MEAS;
            in.eta = (uint8_t)(D.mu == 0 ? 0 : 1);
            P->meas_kind[t] = 1;
            add_relation(raw, t, in.eta);
        } else if (D.a == 0) {
            int h = 31 - __builtin_clz(D.b);
            in.kind = ACTIVE_DIAG_MEAS;
            in.b = D.b;
            in.h = (uint8_t)h;
            in.eta = (uint8_t)(D.mu == 0 ? 0 : 1);
            PauliV Xh = Xb[h];
            pivot_update(D, h, Xh);
            Zb[h] = Q;
            if (in.eta) Zb[h].e = (Zb[h].e + 2) & 3;  // Zbar_h <- (-1)^eta P
            corr = lam;
            corr.flip(sym_meas(t));
            if (in.eta) corr.flip(0);
            frame_add_expr(Xb[h], corr);
            move_pair(h, k - 1);
            k -= 1;
            P->meas_kind[t] = 2;
        } else {
            int h = 31 - __builtin_clz(D.a);
            in.kind = ACTIVE_PAIR_MEAS;
            in.a = D.a;
            in.b = D.b;
            in.h = (uint8_t)h;
            in.mu = (uint8_t)D.mu;
            PauliV Zh = Zb[h];
            pivot_update(D, h, Zh);
            Xb[h] = Zh;
            Zb[h] = Q;
            corr = lam;
            corr.flip(sym_meas(t));
            frame_add_expr(Xb[h], corr);
            move_pair(h, k - 1);
            k -= 1;
            P->meas_kind[t] = 3;
        }
        P->meas_instr[t] = (int32_t)P->instrs.size();
        emit(std::move(in));
    }
};

struct OpView {
    const symft_op *o;
};

int fail(std::string &err, int code, const std::string &msg) {
    err = msg;
    return code;
}

}  // namespace

int compile_program(uint32_t n_qubits, const void *ops_v, size_t n_ops, Program &out, std::string &err) {
    const symft_op *ops = static_cast<const symft_op *>(ops_v);
    if (n_qubits == 0) return fail(err, SYMFT_EINVAL, "n_qubits must be positive");
    if (n_ops && !ops) return fail(err, SYMFT_EINVAL, "ops is NULL");
    Program &P = out;
    P = Program();
    P.n_qubits = n_qubits;
    P.n_ops = n_ops;

    // ---- pass 1: validate, count measurements / records / channels / symbols
    uint64_t nm = 0, nr = 0, nd = 0, nobs = 0;
    uint32_t nsym = 0;
    std::vector<uint8_t> seen(n_qubits, 0);
    for (size_t i = 0; i < n_ops; ++i) {
        const symft_op &o = ops[i];
        if (o.n && !o.qubits) return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": qubits is NULL");
        for (uint32_t j = 0; j < o.n; ++j)
            if (o.qubits[j] >= n_qubits)
                return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": qubit out of range");
        switch (o.kind) {
        case SYMFT_OP_H: case SYMFT_OP_S: case SYMFT_OP_S_DAG: case SYMFT_OP_X: case SYMFT_OP_Y: case SYMFT_OP_Z:
        case SYMFT_OP_TICK:
            break;
        case SYMFT_OP_CX: case SYMFT_OP_CZ: case SYMFT_OP_SWAP:
            if (o.n % 2) return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": two-qubit gate needs pairs");
            for (uint32_t j = 0; j < o.n; j += 2)
                if (o.qubits[j] == o.qubits[j + 1])
                    return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": repeated qubit in a pair");
            break;
        case SYMFT_OP_R:
            if (o.arg != 0.0) return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": a reset has no record to flip");
            nm += o.n;
            break;
        case SYMFT_OP_M: case SYMFT_OP_MR:
            if (!(o.arg >= 0.0 && o.arg <= 1.0))
                return fail(err, SYMFT_EPROB, "op " + std::to_string(i) + ": readout-flip probability outside [0,1]");
            nm += o.n;
            nr += o.n;
            if (o.arg > 0.0) nsym += o.n;
            break;
        case SYMFT_OP_X_ERROR: case SYMFT_OP_DEPOLARIZE1: case SYMFT_OP_DEPOLARIZE2:
            if (!(o.arg >= 0.0 && o.arg <= 1.0))
                return fail(err, SYMFT_EPROB, "op " + std::to_string(i) + ": probability outside [0,1]");
            if (o.kind == SYMFT_OP_DEPOLARIZE2) {
                if (o.n % 2) return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": DEPOLARIZE2 needs pairs");
                for (uint32_t j = 0; j < o.n; j += 2)
                    if (o.qubits[j] == o.qubits[j + 1])
                        return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": repeated qubit in a pair");
                nsym += 2 * o.n;
            } else {
                nsym += (o.kind == SYMFT_OP_X_ERROR ? 1 : 2) * o.n;
            }
            break;
        case SYMFT_OP_PAULI_CHANNEL: {
            if (o.n_branches && (!o.probs || !o.branch_paulis))
                return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": channel arrays are NULL");
            double tot = 0;
            for (uint32_t j = 0; j < o.n_branches; ++j) {
                if (!(o.probs[j] >= 0.0)) return fail(err, SYMFT_EPROB, "op " + std::to_string(i) + ": negative probability");
                tot += o.probs[j];
                for (uint32_t q = 0; q < o.n; ++q)
                    if (o.branch_paulis[j * o.n + q] > 3) return fail(err, SYMFT_EINVAL, "bad Pauli letter");
            }
            if (tot > 1.0 + 1e-12) return fail(err, SYMFT_EPROB, "op " + std::to_string(i) + ": channel total exceeds 1");
            if (o.n > 16) return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": channel support above 16 qubits");
            if (o.n_branches > 64) return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": more than 64 branches");
            nsym += 2 * o.n;
            break;
        }
        case SYMFT_OP_ROT: case SYMFT_OP_MPP: case SYMFT_OP_FEEDBACK: {
            if (o.n && !o.paulis) return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": paulis is NULL");
            for (uint32_t j = 0; j < o.n; ++j) {
                if (o.paulis[j] < 1 || o.paulis[j] > 3) return fail(err, SYMFT_EINVAL, "bad Pauli letter");
                if (seen[o.qubits[j]]) return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": repeated qubit in a Pauli");
                seen[o.qubits[j]] = 1;
            }
            for (uint32_t j = 0; j < o.n; ++j) seen[o.qubits[j]] = 0;
            if (o.kind == SYMFT_OP_MPP) {
                if (!(o.arg >= 0.0 && o.arg <= 1.0))
                    return fail(err, SYMFT_EPROB, "op " + std::to_string(i) + ": readout-flip probability outside [0,1]");
                nm += 1;
                nr += 1;
                if (o.arg > 0.0) nsym += 1;
            }
            if (o.kind == SYMFT_OP_ROT && !std::isfinite(o.arg)) return fail(err, SYMFT_EINVAL, "non-finite angle");
            break;
        }
        case SYMFT_OP_DETECTOR: nd += 1; break;
        case SYMFT_OP_OBSERVABLE: if (o.obs_id + 1 > nobs) nobs = o.obs_id + 1; break;
        default: return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": unknown kind");
        }
        if (o.kind == SYMFT_OP_FEEDBACK || o.kind == SYMFT_OP_DETECTOR || o.kind == SYMFT_OP_OBSERVABLE)
            if (o.n_recs && !o.recs) return fail(err, SYMFT_EINVAL, "op " + std::to_string(i) + ": recs is NULL");
    }
    P.n_meas = nm;
    P.n_rec = nr;
    P.n_det = nd;
    P.n_obs = nobs;

    Compiler K;
    K.n = n_qubits;
    K.Nn = nsym;
    K.M = (uint32_t)nm;
    K.S = 1 + nsym + (uint32_t)nm;
    K.P = &P;
    K.init_frames();
    P.meas_instr.assign(nm, -1);
    P.meas_row.assign(nm, -1);
    P.meas_kind.assign(nm, -1);
    P.rot_kind.assign(n_ops, 0);
    P.k_after_op.assign(n_ops, 0);
    P.det_meas.clear();
    P.obs_meas.assign(nobs, {});
    std::vector<uint32_t> rec_meas;  // record -> measurement
    rec_meas.reserve(nr);

    Bits lam, fb;
    lam.init(K.S);
    fb.init(K.S);
    uint32_t t = 0, sym = 0;
    auto resolve = [&](int64_t r, size_t i, uint32_t &m_out) -> int {
        int64_t rr = r < 0 ? (int64_t)rec_meas.size() + r : r;
        if (rr < 0 || rr >= (int64_t)rec_meas.size())
            return fail(err, SYMFT_EACAUSAL, "op " + std::to_string(i) + ": record " + std::to_string(r) + " not yet measured");
        m_out = rec_meas[(size_t)rr];
        return 0;
    };
    size_t cur_op = 0;
    auto add_channel = [&](const uint32_t *qs, uint32_t nq, const std::vector<std::vector<uint8_t>> &branches,
                           const std::vector<double> &probs, bool uniform, double p_event) {
        Channel ch;
        ch.op = (int32_t)cur_op;
        ch.J = (uint32_t)branches.size();
        ch.uniform = uniform ? 1 : 0;
        // symbols: per qubit, x then z, when some branch has that component
        std::vector<std::pair<uint32_t, int>> comps;  // (qubit index within channel, 0=x 1=z)
        for (uint32_t j = 0; j < nq; ++j) {
            bool hx = false, hz = false;
            for (auto &b : branches) {
                hx |= (b[j] == 1 || b[j] == 2);
                hz |= (b[j] == 2 || b[j] == 3);
            }
            if (hx) comps.push_back({j, 0});
            if (hz) comps.push_back({j, 1});
        }
        ch.sym0 = sym;
        ch.nsym = (uint32_t)comps.size();
        for (auto &b : branches) {
            uint32_t m = 0;
            for (size_t c = 0; c < comps.size(); ++c) {
                uint8_t L = b[comps[c].first];
                bool on = comps[c].second == 0 ? (L == 1 || L == 2) : (L == 2 || L == 3);
                if (on) m |= 1u << c;
            }
            ch.bmask.push_back(m);
        }
        for (size_t c = 0; c < comps.size(); ++c) {
            uint32_t q = qs[comps[c].first];
            const PauliV &F = comps[c].second == 0 ? K.imgX[q] : K.imgZ[q];
            K.frame_add_symbol(F, 1 + sym + (uint32_t)c);
        }
        sym += (uint32_t)comps.size();
        // event threshold and branch thresholds (draw contract)
        double f = std::ldexp(p_event, 32);
        ch.p32 = p_event >= 1.0 ? (uint64_t(1) << 32) : (f <= 0.0 ? 0 : (uint64_t)std::floor(f));
        if (!uniform) {
            double cum = 0;
            for (uint32_t j = 0; j < ch.J; ++j) {
                cum += probs[j];
                double g = p_event > 0 ? std::ldexp(cum / p_event, 32) : 4294967296.0;
                ch.thr.push_back(g >= 4294967296.0 ? (uint64_t(1) << 32) : (uint64_t)std::floor(g));
            }
            if (ch.J) ch.thr[ch.J - 1] = uint64_t(1) << 32;
        }
        P.chans.push_back(std::move(ch));
    };

    // Readout flip of probability p (paper Sec. 6: an exogenous symbol): a
    // one-branch channel whose symbol s enters only the sign of the measured
    // Pauli, so a flipped measurement of P is one of -P.  Returns s.
    auto add_readout_flip = [&](double p) -> uint32_t {
        Channel ch;
        ch.op = (int32_t)cur_op;
        ch.J = 1;
        ch.uniform = 1;
        ch.sym0 = sym;
        ch.nsym = 1;
        ch.bmask.push_back(1u);
        const double f = std::ldexp(p, 32);
        ch.p32 = p >= 1.0 ? (uint64_t(1) << 32) : (f <= 0.0 ? 0 : (uint64_t)std::floor(f));
        P.chans.push_back(std::move(ch));
        return 1 + sym++;
    };

    static const uint8_t D2[15][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 0}, {1, 1}, {1, 2}, {1, 3}, {2, 0},
                                      {2, 1}, {2, 2}, {2, 3}, {3, 0}, {3, 1}, {3, 2}, {3, 3}};
    for (size_t i = 0; i < n_ops; ++i) {
        const symft_op &o = ops[i];
        cur_op = i;
        switch (o.kind) {
        case SYMFT_OP_H: case SYMFT_OP_S: case SYMFT_OP_S_DAG: case SYMFT_OP_X: case SYMFT_OP_Y: case SYMFT_OP_Z:
            for (uint32_t j = 0; j < o.n; ++j) K.gate1(o.kind, o.qubits[j]);
            break;
        case SYMFT_OP_CX: case SYMFT_OP_CZ: case SYMFT_OP_SWAP:
            for (uint32_t j = 0; j < o.n; j += 2) K.gate2(o.kind, o.qubits[j], o.qubits[j + 1]);
            break;
        case SYMFT_OP_R: case SYMFT_OP_M: case SYMFT_OP_MR:
            for (uint32_t j = 0; j < o.n; ++j) {
                uint32_t q = o.qubits[j];
                uint8_t z = 3;
                const uint32_t flip = (o.kind != SYMFT_OP_R && o.arg > 0.0) ? add_readout_flip(o.arg) : 0u;
                PauliV Q = K.pull_back(&q, &z, 1, false);
                K.lambda_of(Q, lam);
                if (flip) lam.flip(flip);
                if (o.kind != SYMFT_OP_R) {
                    P.meas_row[t] = (int64_t)rec_meas.size();
                    rec_meas.push_back(t);
                }
                K.plan_measurement(Q, lam, t, (int)i);
                if (o.kind != SYMFT_OP_M) {  // reset: X^{m_t} feedback on the true outcome m_t + s
                    uint8_t x = 1;
                    PauliV F = K.pull_back(&q, &x, 1, false);
                    fb.clear();
                    fb.flip(K.sym_meas(t));
                    if (flip) fb.flip(flip);
                    K.frame_add_expr(F, fb);
                }
                ++t;
            }
            break;
        case SYMFT_OP_MPP: {
            const uint32_t flip = o.arg > 0.0 ? add_readout_flip(o.arg) : 0u;
            PauliV Q = K.pull_back(o.qubits, o.paulis, o.n, o.negate != 0);
            K.lambda_of(Q, lam);
            if (flip) lam.flip(flip);
            P.meas_row[t] = (int64_t)rec_meas.size();
            rec_meas.push_back(t);
            K.plan_measurement(Q, lam, t, (int)i);
            ++t;
            break;
        }
        case SYMFT_OP_ROT: {
            PauliV Q = K.pull_back(o.qubits, o.paulis, o.n, o.negate != 0);
            K.lambda_of(Q, lam);
            K.plan_rotation(Q, lam, o.arg, (int)i);
            break;
        }
        case SYMFT_OP_FEEDBACK: {
            fb.clear();
            for (uint32_t j = 0; j < o.n_recs; ++j) {
                uint32_t m;
                int rc = resolve(o.recs[j], i, m);
                if (rc) return rc;
                fb.flip(K.sym_meas(m));
            }
            PauliV F = K.pull_back(o.qubits, o.paulis, o.n, false);
            K.frame_add_expr(F, fb);
            break;
        }
        case SYMFT_OP_X_ERROR:
            for (uint32_t j = 0; j < o.n; ++j)
                add_channel(&o.qubits[j], 1, {{1}}, {o.arg}, true, o.arg);
            break;
        case SYMFT_OP_DEPOLARIZE1:
            for (uint32_t j = 0; j < o.n; ++j)
                add_channel(&o.qubits[j], 1, {{1}, {2}, {3}}, {}, true, o.arg);
            break;
        case SYMFT_OP_DEPOLARIZE2: {
            std::vector<std::vector<uint8_t>> br;
            for (auto &d : D2) br.push_back({d[0], d[1]});
            for (uint32_t j = 0; j < o.n; j += 2) add_channel(&o.qubits[j], 2, br, {}, true, o.arg);
            break;
        }
        case SYMFT_OP_PAULI_CHANNEL: {
            std::vector<std::vector<uint8_t>> br;
            std::vector<double> pr;
            double tot = 0;
            for (uint32_t j = 0; j < o.n_branches; ++j) {
                br.push_back(std::vector<uint8_t>(o.branch_paulis + j * o.n, o.branch_paulis + (j + 1) * o.n));
                pr.push_back(o.probs[j]);
                tot += o.probs[j];
            }
            add_channel(o.qubits, o.n, br, pr, false, tot);
            break;
        }
        case SYMFT_OP_DETECTOR: {
            std::vector<uint32_t> ms;
            for (uint32_t j = 0; j < o.n_recs; ++j) {
                uint32_t m;
                int rc = resolve(o.recs[j], i, m);
                if (rc) return rc;
                ms.push_back(m);
            }
            P.det_meas.push_back(std::move(ms));
            P.det_op.push_back((int32_t)i);
            break;
        }
        case SYMFT_OP_OBSERVABLE: {
            for (uint32_t j = 0; j < o.n_recs; ++j) {
                uint32_t m;
                int rc = resolve(o.recs[j], i, m);
                if (rc) return rc;
                P.obs_meas[o.obs_id].push_back(m);
            }
            break;
        }
        default: break;
        }
        P.k_after_op[i] = (int16_t)K.k;
        if (P.k_max > 30) return fail(err, SYMFT_ECAPACITY, "peak active width above 30");
    }
    P.n_noise_sym = sym;

    // probability classes by first occurrence of P32; ranks in circuit order
    for (size_t c = 0; c < P.chans.size(); ++c) {
        Channel &ch = P.chans[c];
        if (ch.p32 == 0) {
            ch.cls = -1;
            continue;
        }
        int f = -1;
        for (size_t j = 0; j < P.classes.size(); ++j)
            if (P.classes[j].p32 == ch.p32) {
                f = (int)j;
                break;
            }
        if (f < 0) {
            f = (int)P.classes.size();
            NoiseClass nc;
            nc.p32 = ch.p32;
            P.classes.push_back(nc);
        }
        ch.cls = f;
        ch.rank = (int64_t)P.classes[f].chans.size();
        P.classes[f].chans.push_back((int32_t)c);
    }
    for (auto &nc : P.classes) {
        nc.Q.resize(4097);
        gap_table(nc.p32, nc.Q.data());
    }
    return 0;
}

// Commutation-aware simplification before planning (paper Sec. 6), in its
// conservative circuit-level form: R_P(a) ... R_P(b) with nothing between
// them touching P's qubits and no detector between them is R_P(a + b) at the
// first place (every op between commutes with P, acting on other qubits), and
// nothing at all when a + b is a multiple of 2 pi.  A rotation that reaches,
// the same way, a measurement of +-P is a phase per outcome and goes too.
std::vector<symft_op> simplify_rotations(const symft_op *ops, size_t n_ops, uint64_t &removed) {
    std::vector<symft_op> out(ops, ops + n_ops);
    removed = 0;
    // sorted (qubit, letter) pairs; empty for a body the compiler would reject
    // (bad letter, repeated qubit), so that such an op is never fused away
    auto body = [](const symft_op &o) {
        std::vector<std::pair<uint32_t, uint8_t>> b;
        for (uint32_t j = 0; j < o.n; ++j) {
            if (o.paulis[j] < 1 || o.paulis[j] > 3) return std::vector<std::pair<uint32_t, uint8_t>>{};
            b.push_back({o.qubits[j], o.paulis[j]});
        }
        std::sort(b.begin(), b.end());
        for (size_t j = 1; j < b.size(); ++j)
            if (b[j].first == b[j - 1].first) return std::vector<std::pair<uint32_t, uint8_t>>{};
        return b;
    };
    const double two_pi = 6.283185307179586;
    for (size_t i = 0; i < n_ops; ++i) {
        if (out[i].kind != SYMFT_OP_ROT || out[i].n == 0) continue;
        const auto bi = body(out[i]);
        if (bi.empty()) continue;
        double theta = out[i].negate ? -out[i].arg : out[i].arg;
        bool fused = false, absorbed = false;
        for (size_t j = i + 1; j < n_ops; ++j) {
            const symft_op &o = out[j];
            if (o.kind == SYMFT_OP_DETECTOR) break;
            if (o.kind == SYMFT_OP_ROT && o.n == bi.size() && body(o) == bi) {
                theta += o.negate ? -o.arg : o.arg;
                out[j] = symft_op{};
                out[j].kind = SYMFT_OP_TICK;
                ++removed;
                fused = true;
                continue;
            }
            bool touch = false;
            for (uint32_t t = 0; t < o.n && !touch; ++t)
                for (const auto &q : bi)
                    if (o.qubits[t] == q.first) {
                        touch = true;
                        break;
                    }
            if (!touch) continue;
            // The rotation commutes up to this op.  A measurement of +-P next
            // (MPP of the same body; M, MR or R of the qubit when P = Z_q)
            // sees R_P only as a phase per outcome, so the rotation goes.
            if (o.kind == SYMFT_OP_MPP) {
                absorbed = o.n == bi.size() && body(o) == bi;
            } else if ((o.kind == SYMFT_OP_M || o.kind == SYMFT_OP_MR || o.kind == SYMFT_OP_R) && bi.size() == 1 &&
                       bi[0].second == 3) {
                absorbed = true;  // touch means one of its qubits is P's
            }
            break;
        }
        if (absorbed) {
            out[i] = symft_op{};
            out[i].kind = SYMFT_OP_TICK;
            ++removed;
            continue;
        }
        if (!fused) continue;
        if (std::fabs(std::remainder(theta, two_pi)) < 1e-12) {
            out[i] = symft_op{};
            out[i].kind = SYMFT_OP_TICK;
            ++removed;
        } else {
            out[i].negate = 0;
            out[i].arg = theta;
        }
    }
    return out;
}

void gap_table(uint64_t p32, uint64_t *Q) {
    Q[0] = uint64_t(1) << 32;
    for (int g = 0; g < 4096; ++g) {
        unsigned __int128 prod = (unsigned __int128)Q[g] * ((uint64_t(1) << 32) - p32);
        Q[g + 1] = (uint64_t)(prod >> 32);
    }
}

}  // namespace symft
