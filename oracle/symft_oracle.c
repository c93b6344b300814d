/*
 * symft_oracle.c -- plain, slow CPU oracle for the SymFT per-shot sampling stage.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; the two meet only
 * at the seeded circuit descriptions built in Python.
 *
 * What it computes (the plain definition of the sampled distribution, paper
 * Sec. 2): every shot starts in |0^n> and applies the circuit's operations in
 * order -- Clifford gates, Pauli rotations R_P(theta) = cos(theta/2) I -
 * i sin(theta/2) P, stochastic Pauli channels, projective Pauli measurements
 * (outcome 0 <-> +1 eigenvalue) and record-parity-controlled Pauli feedback.
 *
 * How it represents the state: a signed stabilizer-destabilizer tableau
 * (Zbar_1..Zbar_n, Xbar_1..Xbar_n) whose first k coordinates are active, plus
 * an explicit FP64 active vector alpha in C^(2^k), so that
 *     psi = sum_x alpha_x Xbar_1^x1 ... Xbar_k^xk |0bar>
 * (paper Sec. 4, eq. for the active basis and the representation invariant).
 * Unlike the paper's planner it carries CONCRETE signs: Clifford gates, noise
 * Paulis and feedback Paulis conjugate every tableau generator (signs
 * included) and leave alpha unchanged, since the global phase is dropped.
 * Rotations and measurements use the active/dormant decomposition
 * P = mu Xbar_A^a Zbar_A^b Xbar_D^d Zbar_D^c (paper Sec. 4) and the paper's
 * case analysis (Sec. 4.1 rotations, Sec. 4.2 measurements); where the paper
 * propagates a symbolic Pauli correction after a measurement, this oracle
 * instead stores the measured eigenspace directly, i.e. the new dormant
 * stabilizer is (-1)^m P.
 *
 * Readout flips (paper Sec. 6 lists them among the exogenous symbols): an M,
 * MR or MPP with probability p > 0 owns one one-branch channel per record; a
 * fired flip reports the complement of the true outcome and leaves the state
 * of the true outcome.  That instrument is exactly a measurement of -P with
 * the outcome reported as is, which is how it runs here, so the measurement's
 * own draw decides the reported bit; a reset acts on the true outcome.
 *
 * Pivot rules (they only change the basis, never a probability or record):
 *   - dormant pivot: the lowest dormant coordinate whose Zbar anticommutes
 *     with P; a promoted coordinate is then swapped to position k (0-based);
 *   - pair instructions: the highest set bit of a;
 *   - active-diagonal measurement: the highest set bit of b;
 *   - after an active measurement the pivot pair becomes the first dormant
 *     coordinate and the active coordinates above it shift down by one.
 *
 * Random draws follow the counter-based Philox4x32-10 draw contract (Salmon
 * et al., SC'11), implemented here from its published definition:
 *   key = (seed mod 2^32, seed >> 32); counter top byte = domain.
 *   domain 1 (gap) / 2 (branch): per (probability class c, 64-shot word w)
 *     a geometric walk over positions rank*64+lane, with the exact-integer
 *     table Q[0]=2^32, Q[g+1]=floor(Q[g](2^32-P32)/2^32), g <= 4096;
 *   domain 3: RandomMeas bits per (measurement t, word w);
 *   domain 4: a 53-bit uniform u per (measurement t, shot s); the recorded bit
 *     is 0 iff u < Pr(m = 0).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (published definition)                                */
/* ------------------------------------------------------------------ */
static void philox4x32_10(const uint32_t ctr_in[4], uint32_t key0, uint32_t key1, uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key0, k1 = key1;
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* exported for the known-answer test */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    philox4x32_10(ctr, key[0], key[1], out);
}

#define DOM_GAP 1u
#define DOM_BRANCH 2u
#define DOM_RMEAS 3u
#define DOM_ACTIVE 4u
#define GAP_CAP 4096

static void draw_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4]) {
    uint32_t ctr[4] = {c0, c1, c2, c3};
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

/* RandomMeas bit for measurement t, shot s (domain 3). */
static int rmeas_bit(uint64_t seed, uint64_t t, uint64_t s) {
    uint64_t w = s >> 6;
    uint32_t o[4];
    draw_block(seed, (uint32_t)(t >> 1), (uint32_t)w, 0u, (DOM_RMEAS << 24) | (uint32_t)(w >> 32), o);
    uint64_t word = (uint64_t)o[2 * (t & 1)] | ((uint64_t)o[2 * (t & 1) + 1] << 32);
    return (int)((word >> (s & 63)) & 1u);
}

/* 53-bit uniform for active measurement t, shot s (domain 4). */
static double active_u(uint64_t seed, uint64_t t, uint64_t s) {
    uint32_t o[4];
    draw_block(seed, (uint32_t)t, (uint32_t)s, (uint32_t)(s >> 32), DOM_ACTIVE << 24, o);
    uint64_t v = ((uint64_t)o[0] << 21) + (uint64_t)(o[1] >> 11);
    return ldexp((double)v, -53);
}

/* ------------------------------------------------------------------ */
/* Pauli rows: i^e X^x Z^z, bit-packed                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int n, W;       /* qubits, 64-bit words per bit vector */
    int rows;       /* number of rows */
    uint64_t *x, *z; /* rows*W each */
    uint8_t *e;      /* phase exponent mod 4 */
} Rows;

static void rows_alloc(Rows *r, int n, int rows) {
    r->n = n;
    r->W = (n + 63) / 64;
    r->rows = rows;
    r->x = (uint64_t *)calloc((size_t)rows * r->W, sizeof(uint64_t));
    r->z = (uint64_t *)calloc((size_t)rows * r->W, sizeof(uint64_t));
    r->e = (uint8_t *)calloc((size_t)rows, 1);
}
static void rows_free(Rows *r) { free(r->x); free(r->z); free(r->e); }
static void rows_copy(Rows *dst, const Rows *src) {
    memcpy(dst->x, src->x, (size_t)src->rows * src->W * 8);
    memcpy(dst->z, src->z, (size_t)src->rows * src->W * 8);
    memcpy(dst->e, src->e, (size_t)src->rows);
}
static inline int getb(const uint64_t *v, int q) { return (int)((v[q >> 6] >> (q & 63)) & 1u); }
static inline void flipb(uint64_t *v, int q) { v[q >> 6] ^= (uint64_t)1 << (q & 63); }
static inline void setb(uint64_t *v, int q, int b) {
    if (getb(v, q) != b) flipb(v, q);
}

/* a standalone Pauli */
typedef struct { uint64_t *x, *z; int e; } Pauli;

static int dot(const uint64_t *a, const uint64_t *b, int W) {
    int s = 0;
    for (int i = 0; i < W; ++i) s += __builtin_popcountll(a[i] & b[i]);
    return s;
}
/* commutation indicator omega(A,B) = x_A.z_B + z_A.x_B mod 2 (paper Sec. 3) */
static int omega(const uint64_t *ax, const uint64_t *az, const uint64_t *bx, const uint64_t *bz, int W) {
    return (dot(ax, bz, W) + dot(az, bx, W)) & 1;
}
/* dst <- dst * src, with (i^e1 X^x1 Z^z1)(i^e2 X^x2 Z^z2) = i^(e1+e2+2 z1.x2) X^(x1^x2) Z^(z1^z2) */
static void mul_right(uint64_t *dx, uint64_t *dz, int *de, const uint64_t *sx, const uint64_t *sz, int se, int W) {
    int e = *de + se + 2 * (dot(dz, sx, W) & 1);
    for (int i = 0; i < W; ++i) { dx[i] ^= sx[i]; dz[i] ^= sz[i]; }
    *de = e & 3;
}

/* ------------------------------------------------------------------ */
/* Clifford conjugation of one row: P -> U P U^dagger                   */
/* ------------------------------------------------------------------ */
enum {
    OK_H = 1, OK_S, OK_SDAG, OK_X, OK_Y, OK_Z, OK_CX, OK_CZ, OK_SWAP,
    OK_R, OK_M, OK_MR, OK_XERR, OK_DEP1, OK_DEP2, OK_CHAN, OK_ROT, OK_MPP, OK_FEEDBACK,
    OK_DET, OK_OBS, OK_TICK
};

static void conj_row(int kind, int qa, int qb, uint64_t *x, uint64_t *z, int *e) {
    int xa = getb(x, qa), za = getb(z, qa);
    switch (kind) {
    case OK_H: /* X <-> Z, X^x Z^z -> Z^x X^z = (-1)^(xz) X^z Z^x */
        setb(x, qa, za); setb(z, qa, xa); *e = (*e + 2 * (xa & za)) & 3; break;
    case OK_S: /* S X S^dag = iXZ, S Z S^dag = Z */
        setb(z, qa, za ^ xa); *e = (*e + xa) & 3; break;
    case OK_SDAG: /* S^dag X S = -iXZ */
        setb(z, qa, za ^ xa); *e = (*e + 3 * xa) & 3; break;
    case OK_X: *e = (*e + 2 * za) & 3; break;
    case OK_Y: *e = (*e + 2 * (xa ^ za)) & 3; break;
    case OK_Z: *e = (*e + 2 * xa) & 3; break;
    case OK_CX: { /* X_c -> X_c X_t, Z_t -> Z_c Z_t */
        int xb = getb(x, qb), zb = getb(z, qb);
        setb(x, qb, xb ^ xa); setb(z, qa, za ^ zb); break;
    }
    case OK_CZ: { /* X_a -> X_a Z_b, X_b -> Z_a X_b */
        int xb = getb(x, qb), zb = getb(z, qb);
        setb(z, qa, za ^ xb); setb(z, qb, zb ^ xa); *e = (*e + 2 * (xa & xb)) & 3; break;
    }
    case OK_SWAP: {
        int xb = getb(x, qb), zb = getb(z, qb);
        setb(x, qa, xb); setb(z, qa, zb); setb(x, qb, xa); setb(z, qb, za); break;
    }
    default: break;
    }
}

/* exported for the exhaustive gate test: conjugates one Pauli on n<=64 qubits */
void orc_conjugate(int kind, int qa, int qb, uint64_t *x, uint64_t *z, int *e) {
    conj_row(kind, qa, qb, x, z, e);
}

/* ------------------------------------------------------------------ */
/* Circuit description (decoded from the tape built by oracle.py)      */
/* ------------------------------------------------------------------ */
typedef struct {
    int kind;
    int nq;
    int *q;
    uint8_t *let;    /* Pauli letters for ROT/MPP/FEEDBACK (1=X,2=Y,3=Z) */
    int negate;
    double arg;
    int nrec;
    int64_t *recs;
    int obs;
    int nbr;         /* PAULI_CHANNEL */
    double *probs;
    uint8_t *blet;   /* nbr*nq letters 0..3 */
    int chan0;       /* first channel index of a noise op */
    int meas0;       /* first measurement index of a measurement op */
    int rec0;        /* first visible record index */
} OOp;

typedef struct {
    int op;          /* op index */
    int qa, qb;      /* qubits for X_ERROR/DEP1 (qa), DEP2 (qa,qb), CHAN: -1 */
    int kind;        /* OK_XERR / OK_DEP1 / OK_DEP2 / OK_CHAN */
    uint64_t p32;    /* event threshold, <= 2^32 */
    int cls;         /* probability class, -1 if it never fires */
    int64_t rank;    /* position within its class */
    int uniform;     /* branch choice (v*J)>>32 */
    int J;           /* number of branches */
    uint64_t *thr;   /* non-uniform thresholds, J entries */
} OChan;

typedef struct {
    uint64_t p32;
    int64_t n;       /* channels in the class */
    uint64_t *Q;     /* GAP_CAP+1 entries */
} OClass;

typedef struct {
    int n;
    int n_ops;
    OOp *ops;
    int n_chan;
    OChan *ch;
    int n_cls;
    OClass *cls;
    int n_meas, n_rec, n_det, n_obs;
    int *rec_meas;   /* visible record -> measurement index */
    int *det_op;     /* detector -> op index */
    int *obs_ops_n;  /* per observable: number of OBS ops */
    int **obs_ops;
} OCirc;

static int is_noise(int k) { return k == OK_XERR || k == OK_DEP1 || k == OK_DEP2 || k == OK_CHAN; }

/* Channels an op owns: noise ops their Pauli channels; a recorded measurement
 * with a readout-flip probability (arg > 0) one flip per record it writes
 * (paper Sec. 6: readout flips are exogenous symbols). */
static int op_channels(const OOp *o) {
    switch (o->kind) {
    case OK_XERR: case OK_DEP1: return o->nq;
    case OK_DEP2: return o->nq / 2;
    case OK_CHAN: return 1;
    case OK_M: case OK_MR: return o->arg > 0 ? o->nq : 0;
    case OK_MPP: return o->arg > 0 ? 1 : 0;
    default: return 0;
    }
}

/* Tape layout (int64): n_ops, then per op:
 *   kind, nq, q[nq], negate, n_let, let[n_let], nrec, recs[nrec], obs, nbr, blet[nbr*nq]
 * doubles, consumed in order: arg for every op, then probs[nbr] for PAULI_CHANNEL. */
/* Largest register: the per-shot Pauli scratch rows (nx, nz, tmp) are fixed
 * arrays of 64 words. */
#define ORC_MAX_QUBITS 4096

/* NULL when n_qubits is outside [1, ORC_MAX_QUBITS] or an op names a qubit
 * outside [0, n_qubits). */
void *orc_circuit_new(int n_qubits, const int64_t *tape, const double *dargs) {
    if (n_qubits < 1 || n_qubits > ORC_MAX_QUBITS || !tape || !dargs) return NULL;
    {
        /* bounds pass over the tape before anything is allocated */
        size_t ti = 0;
        const int64_t n_ops = tape[ti++];
        if (n_ops < 0) return NULL;
        for (int64_t i = 0; i < n_ops; ++i) {
            ti++; /* kind */
            const int64_t nq = tape[ti++];
            if (nq < 0) return NULL;
            for (int64_t j = 0; j < nq; ++j)
                if (tape[ti + (size_t)j] < 0 || tape[ti + (size_t)j] >= n_qubits) return NULL;
            ti += (size_t)nq;
            ti++; /* negate */
            const int64_t nl = tape[ti++];
            if (nl < 0) return NULL;
            ti += (size_t)nl;
            const int64_t nrec = tape[ti++];
            if (nrec < 0) return NULL;
            ti += (size_t)nrec;
            ti++; /* obs */
            const int64_t nbr = tape[ti++];
            if (nbr < 0) return NULL;
            ti += (size_t)(nbr * nq);
        }
    }
    OCirc *C = (OCirc *)calloc(1, sizeof(OCirc));
    C->n = n_qubits;
    size_t ti = 0, di = 0;
    C->n_ops = (int)tape[ti++];
    C->ops = (OOp *)calloc((size_t)C->n_ops, sizeof(OOp));
    int nch = 0, nm = 0, nr = 0, nd = 0, nobs = 0;
    for (int i = 0; i < C->n_ops; ++i) {
        OOp *o = &C->ops[i];
        o->kind = (int)tape[ti++];
        o->nq = (int)tape[ti++];
        o->q = (int *)malloc(sizeof(int) * (size_t)(o->nq + 1));
        for (int j = 0; j < o->nq; ++j) o->q[j] = (int)tape[ti++];
        o->negate = (int)tape[ti++];
        int nl = (int)tape[ti++];
        o->let = (uint8_t *)malloc((size_t)nl + 1);
        for (int j = 0; j < nl; ++j) o->let[j] = (uint8_t)tape[ti++];
        o->nrec = (int)tape[ti++];
        o->recs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(o->nrec + 1));
        for (int j = 0; j < o->nrec; ++j) o->recs[j] = tape[ti++];
        o->obs = (int)tape[ti++];
        o->nbr = (int)tape[ti++];
        o->blet = (uint8_t *)malloc((size_t)o->nbr * o->nq + 1);
        for (int j = 0; j < o->nbr * o->nq; ++j) o->blet[j] = (uint8_t)tape[ti++];
        o->arg = dargs[di++];
        o->probs = (double *)malloc(sizeof(double) * (size_t)(o->nbr + 1));
        for (int j = 0; j < o->nbr; ++j) o->probs[j] = dargs[di++];
        o->chan0 = nch;
        o->meas0 = nm;
        o->rec0 = nr;
        nch += op_channels(o);
        switch (o->kind) {
        case OK_R: nm += o->nq; break;
        case OK_M: case OK_MR: nm += o->nq; nr += o->nq; break;
        case OK_MPP: nm += 1; nr += 1; break;
        case OK_DET: nd += 1; break;
        case OK_OBS: if (o->obs + 1 > nobs) nobs = o->obs + 1; break;
        default: break;
        }
    }
    C->n_chan = nch; C->n_meas = nm; C->n_rec = nr; C->n_det = nd; C->n_obs = nobs;
    C->rec_meas = (int *)malloc(sizeof(int) * (size_t)(nr + 1));
    C->det_op = (int *)malloc(sizeof(int) * (size_t)(nd + 1));
    C->obs_ops_n = (int *)calloc((size_t)nobs + 1, sizeof(int));
    C->obs_ops = (int **)calloc((size_t)nobs + 1, sizeof(int *));
    for (int b = 0; b < nobs; ++b) C->obs_ops[b] = (int *)malloc(sizeof(int) * (size_t)C->n_ops);
    C->ch = (OChan *)calloc((size_t)nch + 1, sizeof(OChan));
    int ci = 0, di2 = 0;
    for (int i = 0; i < C->n_ops; ++i) {
        OOp *o = &C->ops[i];
        if (o->kind == OK_M || o->kind == OK_MR) {
            for (int j = 0; j < o->nq; ++j) C->rec_meas[o->rec0 + j] = o->meas0 + j;
        } else if (o->kind == OK_MPP) {
            C->rec_meas[o->rec0] = o->meas0;
        } else if (o->kind == OK_DET) {
            C->det_op[di2++] = i;
        } else if (o->kind == OK_OBS) {
            C->obs_ops[o->obs][C->obs_ops_n[o->obs]++] = i;
        }
        int cnt = op_channels(o);
        for (int j = 0; j < cnt; ++j) {
            OChan *c = &C->ch[ci++];
            c->op = i;
            c->kind = o->kind;
            c->qa = -1; c->qb = -1;
            double ptot;
            if (o->kind == OK_DEP2) { c->qa = o->q[2 * j]; c->qb = o->q[2 * j + 1]; }
            else if (o->kind != OK_CHAN && o->kind != OK_MPP) { c->qa = o->q[j]; }
            if (!is_noise(o->kind)) {
                /* readout flip: one branch of probability arg */
                ptot = o->arg;
                c->uniform = 1;
                c->J = 1;
            } else if (o->kind == OK_CHAN) {
                /* general channel: total in branch order, integer thresholds */
                ptot = 0.0;
                for (int b = 0; b < o->nbr; ++b) ptot += o->probs[b];
                c->uniform = 0;
                c->J = o->nbr;
                c->thr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(o->nbr + 1));
                double cum = 0.0;
                for (int b = 0; b < o->nbr; ++b) {
                    cum += o->probs[b];
                    double f = ptot > 0 ? ldexp(cum / ptot, 32) : 4294967296.0;
                    uint64_t t = f >= 4294967296.0 ? ((uint64_t)1 << 32) : (uint64_t)floor(f);
                    c->thr[b] = t;
                }
                if (o->nbr > 0) c->thr[o->nbr - 1] = (uint64_t)1 << 32;
            } else {
                ptot = o->arg;
                c->uniform = 1;
                c->J = o->kind == OK_XERR ? 1 : (o->kind == OK_DEP1 ? 3 : 15);
            }
            double f = ldexp(ptot, 32);
            c->p32 = ptot >= 1.0 ? ((uint64_t)1 << 32) : (f <= 0.0 ? 0 : (uint64_t)floor(f));
        }
    }
    /* probability classes by first occurrence of P32 */
    C->cls = (OClass *)calloc((size_t)nch + 1, sizeof(OClass));
    C->n_cls = 0;
    for (int i = 0; i < nch; ++i) {
        OChan *c = &C->ch[i];
        if (c->p32 == 0) { c->cls = -1; continue; }
        int f = -1;
        for (int k = 0; k < C->n_cls; ++k)
            if (C->cls[k].p32 == c->p32) { f = k; break; }
        if (f < 0) {
            f = C->n_cls++;
            C->cls[f].p32 = c->p32;
            C->cls[f].n = 0;
        }
        c->cls = f;
        c->rank = C->cls[f].n++;
    }
    for (int k = 0; k < C->n_cls; ++k) {
        OClass *K = &C->cls[k];
        K->Q = (uint64_t *)malloc(sizeof(uint64_t) * (GAP_CAP + 1));
        K->Q[0] = (uint64_t)1 << 32;
        for (int g = 0; g < GAP_CAP; ++g) {
            unsigned __int128 prod = (unsigned __int128)K->Q[g] * (((uint64_t)1 << 32) - K->p32);
            K->Q[g + 1] = (uint64_t)(prod >> 32);
        }
    }
    return C;
}

void orc_circuit_free(void *h) {
    OCirc *C = (OCirc *)h;
    if (!C) return;
    for (int i = 0; i < C->n_ops; ++i) {
        free(C->ops[i].q); free(C->ops[i].let); free(C->ops[i].recs);
        free(C->ops[i].blet); free(C->ops[i].probs);
    }
    for (int i = 0; i < C->n_chan; ++i) free(C->ch[i].thr);
    for (int k = 0; k < C->n_cls; ++k) free(C->cls[k].Q);
    for (int b = 0; b < C->n_obs; ++b) free(C->obs_ops[b]);
    free(C->obs_ops); free(C->obs_ops_n);
    free(C->ops); free(C->ch); free(C->cls); free(C->rec_meas); free(C->det_op);
    free(C);
}

void orc_circuit_info(void *h, int64_t *info) {
    OCirc *C = (OCirc *)h;
    info[0] = C->n_meas; info[1] = C->n_rec; info[2] = C->n_det; info[3] = C->n_obs;
    info[4] = C->n_chan; info[5] = C->n_cls;
}

/* class/rank/p32 of each channel (for tests of the noise sampler) */
void orc_channel_info(void *h, int64_t *cls, int64_t *rank, uint64_t *p32) {
    OCirc *C = (OCirc *)h;
    for (int i = 0; i < C->n_chan; ++i) { cls[i] = C->ch[i].cls; rank[i] = C->ch[i].rank; p32[i] = C->ch[i].p32; }
}

/* ------------------------------------------------------------------ */
/* Noise events of one 64-shot word (domains 1 and 2)                   */
/* ------------------------------------------------------------------ */
/* G = max { g in [0, GAP_CAP] : v < Q[g] }  (Q non-increasing, Q[0] = 2^32 > v) */
static int gap_of(const uint64_t *Q, uint32_t v) {
    int lo = 0, hi = GAP_CAP; /* invariant: v < Q[lo] */
    if ((uint64_t)v < Q[hi]) return hi;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if ((uint64_t)v < Q[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

/* fired[c][lane] = branch index or -1; fills for one word */
static void word_events(const OCirc *C, uint64_t seed, uint64_t w, int16_t *fired /* n_chan*64 */,
                        int64_t **rank_to_chan) {
    for (int i = 0; i < C->n_chan * 64; ++i) fired[i] = -1;
    for (int c = 0; c < C->n_cls; ++c) {
        const OClass *K = &C->cls[c];
        int64_t end = K->n * 64;
        int64_t pos = 0;
        uint64_t j = 0, ev = 0;
        uint32_t blk[4];
        while (pos < end) {
            if ((j & 3) == 0)
                draw_block(seed, (uint32_t)(j >> 2), (uint32_t)w, (uint32_t)c, (DOM_GAP << 24) | (uint32_t)(w >> 32), blk);
            uint32_t v = blk[j & 3];
            ++j;
            int G = gap_of(K->Q, v);
            if (G == GAP_CAP) { pos += GAP_CAP; continue; }
            int64_t at = pos + G;
            pos = at + 1;
            if (at >= end) break;
            int64_t rank = at >> 6;
            int lane = (int)(at & 63);
            int ch = (int)rank_to_chan[c][rank];
            const OChan *X = &C->ch[ch];
            uint32_t bb[4];
            draw_block(seed, (uint32_t)(ev >> 2), (uint32_t)w, (uint32_t)c, (DOM_BRANCH << 24) | (uint32_t)(w >> 32), bb);
            uint32_t u = bb[ev & 3];
            ++ev;
            int br;
            if (X->uniform) {
                br = (int)(((uint64_t)u * (uint64_t)X->J) >> 32);
            } else {
                br = X->J - 1;
                for (int b = 0; b < X->J; ++b)
                    if ((uint64_t)u < X->thr[b]) { br = b; break; }
            }
            fired[(size_t)ch * 64 + lane] = (int16_t)br;
        }
    }
}

static int64_t **build_rank_maps(const OCirc *C) {
    int64_t **m = (int64_t **)calloc((size_t)C->n_cls + 1, sizeof(int64_t *));
    for (int c = 0; c < C->n_cls; ++c) m[c] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C->cls[c].n + 1));
    for (int i = 0; i < C->n_chan; ++i)
        if (C->ch[i].cls >= 0) m[C->ch[i].cls][C->ch[i].rank] = i;
    return m;
}
static void free_rank_maps(const OCirc *C, int64_t **m) {
    for (int c = 0; c < C->n_cls; ++c) free(m[c]);
    free(m);
}

/* ------------------------------------------------------------------ */
/* One shot: tableau + active vector                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    int n, W, k, kcap;
    Rows T;            /* rows 0..n-1 = Zbar_j, n..2n-1 = Xbar_j */
    double complex *a, *b;
    uint8_t *m;        /* all measurement outcomes */
    /* scratch */
    uint64_t *px, *pz, *rx, *rz;
    int *zc, *xc;
    /* trace (optional) */
    int trace;
    int8_t *t_kind;    /* per measurement: 0 random 1 det 2 diag 3 pair */
    double *t_p0;      /* per measurement: Pr(m=0) */
    int8_t *t_rot;     /* per op: rotation kind 0 none 1 promote 2 diag 3 pair */
    int16_t *t_k;      /* per op: k after the op */
} Shot;

static void shot_init(Shot *S, const OCirc *C) {
    memset(S, 0, sizeof(*S));
    S->n = C->n;
    S->W = (C->n + 63) / 64;
    rows_alloc(&S->T, C->n, 2 * C->n);
    S->kcap = 4;
    S->a = (double complex *)malloc(sizeof(double complex) << S->kcap);
    S->b = (double complex *)malloc(sizeof(double complex) << S->kcap);
    S->m = (uint8_t *)malloc((size_t)C->n_meas + 1);
    S->px = (uint64_t *)malloc(8 * (size_t)S->W); S->pz = (uint64_t *)malloc(8 * (size_t)S->W);
    S->rx = (uint64_t *)malloc(8 * (size_t)S->W); S->rz = (uint64_t *)malloc(8 * (size_t)S->W);
    S->zc = (int *)malloc(sizeof(int) * (size_t)C->n);
    S->xc = (int *)malloc(sizeof(int) * (size_t)C->n);
}
static void shot_free(Shot *S) {
    rows_free(&S->T); free(S->a); free(S->b); free(S->m);
    free(S->px); free(S->pz); free(S->rx); free(S->rz); free(S->zc); free(S->xc);
}
static void shot_reset(Shot *S) {
    int n = S->n, W = S->W;
    memset(S->T.x, 0, (size_t)2 * n * W * 8);
    memset(S->T.z, 0, (size_t)2 * n * W * 8);
    memset(S->T.e, 0, (size_t)2 * n);
    for (int j = 0; j < n; ++j) {
        flipb(S->T.z + (size_t)j * W, j);       /* Zbar_j = Z_j */
        flipb(S->T.x + (size_t)(n + j) * W, j); /* Xbar_j = X_j */
    }
    S->k = 0;
    S->a[0] = 1.0;
}
static void ensure_cap(Shot *S, int k) {
    if (k <= S->kcap) return;
    while (S->kcap < k) S->kcap++;
    S->a = (double complex *)realloc(S->a, sizeof(double complex) << S->kcap);
    S->b = (double complex *)realloc(S->b, sizeof(double complex) << S->kcap);
}

#define ZROW(S, j) ((size_t)(j) * (S)->W)
#define XROW(S, j) ((size_t)((S)->n + (j)) * (S)->W)

static void tab_conj_gate(Shot *S, int kind, int qa, int qb) {
    for (int r = 0; r < 2 * S->n; ++r) {
        int e = S->T.e[r];
        conj_row(kind, qa, qb, S->T.x + (size_t)r * S->W, S->T.z + (size_t)r * S->W, &e);
        S->T.e[r] = (uint8_t)e;
    }
}
/* apply a Pauli operator N to the state: every generator G -> N G N^dag = (-1)^omega G */
static void tab_apply_pauli(Shot *S, const uint64_t *nx, const uint64_t *nz) {
    for (int r = 0; r < 2 * S->n; ++r)
        if (omega(nx, nz, S->T.x + (size_t)r * S->W, S->T.z + (size_t)r * S->W, S->W))
            S->T.e[r] = (uint8_t)((S->T.e[r] + 2) & 3);
}
static void tab_row_mul(Shot *S, int dst, int src) {
    int e = S->T.e[dst];
    mul_right(S->T.x + (size_t)dst * S->W, S->T.z + (size_t)dst * S->W, &e,
              S->T.x + (size_t)src * S->W, S->T.z + (size_t)src * S->W, S->T.e[src], S->W);
    S->T.e[dst] = (uint8_t)e;
}
static void tab_row_set(Shot *S, int dst, const uint64_t *x, const uint64_t *z, int e) {
    memcpy(S->T.x + (size_t)dst * S->W, x, 8 * (size_t)S->W);
    memcpy(S->T.z + (size_t)dst * S->W, z, 8 * (size_t)S->W);
    S->T.e[dst] = (uint8_t)(e & 3);
}
static void tab_row_copy(Shot *S, int dst, int src) {
    tab_row_set(S, dst, S->T.x + (size_t)src * S->W, S->T.z + (size_t)src * S->W, S->T.e[src]);
}
static void tab_swap_pairs(Shot *S, int i, int j) {
    if (i == j) return;
    int W = S->W;
    uint64_t tmp[64];
    uint8_t te;
    int rows[2][2] = {{i, j}, {S->n + i, S->n + j}};
    for (int t = 0; t < 2; ++t) {
        int r1 = rows[t][0], r2 = rows[t][1];
        memcpy(tmp, S->T.x + (size_t)r1 * W, 8 * (size_t)W);
        memcpy(S->T.x + (size_t)r1 * W, S->T.x + (size_t)r2 * W, 8 * (size_t)W);
        memcpy(S->T.x + (size_t)r2 * W, tmp, 8 * (size_t)W);
        memcpy(tmp, S->T.z + (size_t)r1 * W, 8 * (size_t)W);
        memcpy(S->T.z + (size_t)r1 * W, S->T.z + (size_t)r2 * W, 8 * (size_t)W);
        memcpy(S->T.z + (size_t)r2 * W, tmp, 8 * (size_t)W);
        te = S->T.e[r1]; S->T.e[r1] = S->T.e[r2]; S->T.e[r2] = te;
    }
}
/* move coordinate pair h to position dst (dst >= h), shifting h+1..dst down by one */
static void tab_move_pair(Shot *S, int h, int dst) {
    for (int j = h; j < dst; ++j) tab_swap_pairs(S, j, j + 1);
}

/* Build the Pauli of a ROT/MPP/FEEDBACK op into px,pz and return its phase exponent. */
static int op_pauli(Shot *S, const OOp *o) {
    memset(S->px, 0, 8 * (size_t)S->W);
    memset(S->pz, 0, 8 * (size_t)S->W);
    int e = o->negate ? 2 : 0;
    for (int j = 0; j < o->nq; ++j) {
        int q = o->q[j], L = o->let[j];
        if (L == 1 || L == 2) flipb(S->px, q);
        if (L == 2 || L == 3) flipb(S->pz, q);
        if (L == 2) e += 1; /* Y = i X Z; distinct qubits commute, so X^x Z^z ordering adds no sign */
    }
    return e & 3;
}

/*
 * Active/dormant decomposition (paper Sec. 4):  P = mu Xbar_A^a Zbar_A^b Xbar_D^d Zbar_D^c.
 * zc[j] = omega(P, Zbar_j) (a for active j, d for dormant), xc[j] = omega(P, Xbar_j) (b / c).
 * Returns mu as a power of i; flags whether any dormant zc is set.
 */
static int decompose(Shot *S, int pe, int *has_d, uint32_t *amask, uint32_t *bmask) {
    int n = S->n, W = S->W, k = S->k;
    *has_d = 0; *amask = 0; *bmask = 0;
    for (int j = 0; j < n; ++j) {
        S->zc[j] = omega(S->px, S->pz, S->T.x + ZROW(S, j), S->T.z + ZROW(S, j), W);
        S->xc[j] = omega(S->px, S->pz, S->T.x + XROW(S, j), S->T.z + XROW(S, j), W);
        if (j < k) {
            if (S->zc[j]) *amask |= 1u << j;
            if (S->xc[j]) *bmask |= 1u << j;
        } else if (S->zc[j]) {
            *has_d = 1;
        }
    }
    /* product in the written order: Xbar_A^a, Zbar_A^b, Xbar_D^d, Zbar_D^c */
    memset(S->rx, 0, 8 * (size_t)W);
    memset(S->rz, 0, 8 * (size_t)W);
    int re = 0;
    for (int j = 0; j < k; ++j)
        if (S->zc[j]) mul_right(S->rx, S->rz, &re, S->T.x + XROW(S, j), S->T.z + XROW(S, j), S->T.e[n + j], W);
    for (int j = 0; j < k; ++j)
        if (S->xc[j]) mul_right(S->rx, S->rz, &re, S->T.x + ZROW(S, j), S->T.z + ZROW(S, j), S->T.e[j], W);
    for (int j = k; j < n; ++j)
        if (S->zc[j]) mul_right(S->rx, S->rz, &re, S->T.x + XROW(S, j), S->T.z + XROW(S, j), S->T.e[n + j], W);
    for (int j = k; j < n; ++j)
        if (S->xc[j]) mul_right(S->rx, S->rz, &re, S->T.x + ZROW(S, j), S->T.z + ZROW(S, j), S->T.e[j], W);
    for (int i = 0; i < W; ++i)
        if (S->rx[i] != S->px[i] || S->rz[i] != S->pz[i]) {
            fprintf(stderr, "symft oracle: tableau no longer spans the Pauli group\n");
            abort();
        }
    return (pe - re) & 3;
}

static const double complex IPOW[4] = {1.0, I, -1.0, -I};

static inline int parity32(uint32_t v) { return __builtin_popcount(v) & 1; }

/* Dormant-pivot coordinate change shared by promotion and random measurement:
 * every generator other than the pivot pair that anticommutes with P is
 * multiplied by Zbar_h (paper Sec. 4.1, dormant-nondiagonal case). */
static void dormant_pivot_update(Shot *S, int h) {
    int n = S->n;
    for (int j = 0; j < n; ++j) {
        if (j == h) continue;
        if (S->zc[j]) tab_row_mul(S, j, h);
        if (S->xc[j]) tab_row_mul(S, n + j, h);
    }
}

static void do_rotation(Shot *S, int pe, double theta, int op_index) {
    int has_d; uint32_t a, b;
    int mu = decompose(S, pe, &has_d, &a, &b);
    int n = S->n, k = S->k;
    double c = cos(theta / 2), s = sin(theta / 2);
    int kind;
    if (has_d) {
        int h = -1;
        for (int j = k; j < n; ++j) if (S->zc[j]) { h = j; break; }
        dormant_pivot_update(S, h);
        tab_row_set(S, n + h, S->px, S->pz, pe);  /* Xbar_h <- P */
        tab_swap_pairs(S, h, k);
        ensure_cap(S, k + 1);
        size_t N = (size_t)1 << k;
        for (size_t x = 0; x < N; ++x) {
            double complex v = S->a[x];
            S->a[x] = c * v;
            S->a[x + N] = -I * s * v;
        }
        S->k = k + 1;
        kind = 1;
    } else if (a == 0 && b == 0) {
        kind = 0; /* acts as +-1 on the represented state: global phase */
    } else if (a == 0) {
        size_t N = (size_t)1 << k;
        double sg = (mu == 0) ? 1.0 : -1.0; /* mu is real here */
        for (size_t x = 0; x < N; ++x) {
            double sig = sg * (parity32(b & (uint32_t)x) ? -1.0 : 1.0);
            S->a[x] *= (c - I * sig * s);
        }
        kind = 2;
    } else {
        size_t N = (size_t)1 << k;
        double complex m = IPOW[mu];
        for (size_t x = 0; x < N; ++x) {
            uint32_t y = (uint32_t)x ^ a;
            double sg = parity32(b & y) ? -1.0 : 1.0;
            S->b[x] = c * S->a[x] - I * s * m * sg * S->a[y];
        }
        memcpy(S->a, S->b, sizeof(double complex) * N);
        kind = 3;
    }
    if (S->trace) S->t_rot[op_index] = (int8_t)kind;
}

static inline uint32_t insert_bit(uint32_t z, int h, int v) {
    uint32_t lo = z & ((1u << h) - 1u);
    uint32_t hi = z >> h;
    return lo | ((uint32_t)v << h) | (hi << (h + 1));
}

static int top_bit(uint32_t v) { return 31 - __builtin_clz(v); }

/* Returns the outcome bit; t = global measurement index, sh = shot index. */
static int do_measure(Shot *S, int pe, uint64_t seed, int t, uint64_t sh) {
    int has_d; uint32_t a, b;
    int mu = decompose(S, pe, &has_d, &a, &b);
    int n = S->n, k = S->k;
    int m, kind;
    double p0 = NAN;
    if (has_d) {
        /* dormant-nondiagonal: uniformly random, vector unchanged (Sec. 4.2) */
        m = rmeas_bit(seed, (uint64_t)t, sh);
        int h = -1;
        for (int j = k; j < n; ++j) if (S->zc[j]) { h = j; break; }
        dormant_pivot_update(S, h);
        tab_row_copy(S, n + h, h);                    /* Xbar_h <- old Zbar_h */
        tab_row_set(S, h, S->px, S->pz, pe + 2 * m);  /* Zbar_h <- (-1)^m P  */
        kind = 0;
        p0 = 0.5;
    } else if (a == 0 && b == 0) {
        /* dormant-diagonal: P acts as mu = (-1)^eta */
        m = (mu == 0) ? 0 : 1;
        kind = 1;
        p0 = m ? 0.0 : 1.0;
    } else if (a == 0) {
        /* active-diagonal: P|x> = (-1)^(b.x + eta)|x> */
        int eta = (mu == 0) ? 0 : 1;
        size_t N = (size_t)1 << k;
        double s0 = 0, s1 = 0;
        for (size_t x = 0; x < N; ++x) {
            double w = creal(S->a[x]) * creal(S->a[x]) + cimag(S->a[x]) * cimag(S->a[x]);
            if (parity32(b & (uint32_t)x) ^ eta) s1 += w; else s0 += w;
        }
        p0 = s0 / (s0 + s1);
        double u = active_u(seed, (uint64_t)t, sh);
        m = (u < p0) ? 0 : 1;
        int h = top_bit(b);
        int v = m ^ eta;
        double norm = 1.0 / sqrt(m ? s1 : s0);
        uint32_t bl = b & ~(1u << h);
        for (size_t z = 0; z < N / 2; ++z) {
            uint32_t uu = insert_bit((uint32_t)z, h, v);
            uint32_t x = uu ^ ((uint32_t)parity32(bl & uu) << h);
            S->b[z] = S->a[x] * norm;
        }
        memcpy(S->a, S->b, sizeof(double complex) * (N / 2));
        /* generators anticommuting with P take a factor Xbar_h; then Zbar_h <- (-1)^m P */
        for (int j = 0; j < n; ++j) {
            if (j == h) continue;
            if (S->zc[j]) tab_row_mul(S, j, n + h);
            if (S->xc[j]) tab_row_mul(S, n + j, n + h);
        }
        tab_row_set(S, h, S->px, S->pz, pe + 2 * m);
        tab_move_pair(S, h, k - 1);
        S->k = k - 1;
        kind = 2;
    } else {
        /* active-nondiagonal: paired amplitudes beta_z(y) */
        size_t N = (size_t)1 << k;
        int h = top_bit(a);
        double complex mc = conj(IPOW[mu]);
        double s0 = 0, s1 = 0;
        for (size_t z = 0; z < N / 2; ++z) {
            uint32_t u0 = insert_bit((uint32_t)z, h, 0);
            double sg = parity32(b & u0) ? -1.0 : 1.0;
            double complex b0 = (S->a[u0] + mc * sg * S->a[u0 ^ a]) / sqrt(2.0);
            double complex b1 = (S->a[u0] - mc * sg * S->a[u0 ^ a]) / sqrt(2.0);
            s0 += creal(b0) * creal(b0) + cimag(b0) * cimag(b0);
            s1 += creal(b1) * creal(b1) + cimag(b1) * cimag(b1);
        }
        p0 = s0 / (s0 + s1);
        double u = active_u(seed, (uint64_t)t, sh);
        m = (u < p0) ? 0 : 1;
        double norm = 1.0 / sqrt(m ? s1 : s0);
        double ys = m ? -1.0 : 1.0;
        for (size_t z = 0; z < N / 2; ++z) {
            uint32_t u0 = insert_bit((uint32_t)z, h, 0);
            double sg = parity32(b & u0) ? -1.0 : 1.0;
            S->b[z] = (S->a[u0] + ys * mc * sg * S->a[u0 ^ a]) / sqrt(2.0) * norm;
        }
        memcpy(S->a, S->b, sizeof(double complex) * (N / 2));
        dormant_pivot_update(S, h);                   /* same rule: G -> G Zbar_h */
        tab_row_copy(S, n + h, h);                    /* Xbar_h <- old Zbar_h */
        tab_row_set(S, h, S->px, S->pz, pe + 2 * m);  /* Zbar_h <- (-1)^m P */
        tab_move_pair(S, h, k - 1);
        S->k = k - 1;
        kind = 3;
    }
    S->m[t] = (uint8_t)m;
    if (S->trace) { S->t_kind[t] = (int8_t)kind; S->t_p0[t] = p0; }
    return m;
}

static void set_single_z(Shot *S, int q) {
    memset(S->px, 0, 8 * (size_t)S->W);
    memset(S->pz, 0, 8 * (size_t)S->W);
    flipb(S->pz, q);
}
static void apply_x_on(Shot *S, int q) {
    uint64_t nx[64] = {0}, nz[64] = {0};
    flipb(nx, q);
    tab_apply_pauli(S, nx, nz);
}

static int rec_value(const OCirc *C, const Shot *S, int64_t r) {
    return S->m[C->rec_meas[r]];
}

/* letters of a uniform channel branch: D1 order X,Y,Z; D2 lexicographic over
 * {I,X,Y,Z}^2 without II with I<X<Y<Z */
static void branch_letters(const OChan *X, int br, int *la, int *lb) {
    if (X->kind == OK_XERR) { *la = 1; *lb = 0; }
    else if (X->kind == OK_DEP1) { *la = br + 1; *lb = 0; }
    else { int v = br + 1; *la = v / 4; *lb = v % 4; }
}

static void letter_into(uint64_t *x, uint64_t *z, int q, int L) {
    if (L == 1 || L == 2) flipb(x, q);
    if (L == 2 || L == 3) flipb(z, q);
}

/* Simulate shot `sh` (lane = sh % 64) given the word's fired table. */
static void run_shot(const OCirc *C, Shot *S, uint64_t seed, uint64_t sh, const int16_t *fired) {
    shot_reset(S);
    int lane = (int)(sh & 63);
    int W = S->W;
    uint64_t nx[64], nz[64];
    for (int i = 0; i < C->n_ops; ++i) {
        const OOp *o = &C->ops[i];
        switch (o->kind) {
        case OK_H: case OK_S: case OK_SDAG: case OK_X: case OK_Y: case OK_Z:
            for (int j = 0; j < o->nq; ++j) tab_conj_gate(S, o->kind, o->q[j], -1);
            break;
        case OK_CX: case OK_CZ: case OK_SWAP:
            for (int j = 0; j + 1 < o->nq; j += 2) tab_conj_gate(S, o->kind, o->q[j], o->q[j + 1]);
            break;
        case OK_R: case OK_M: case OK_MR:
            for (int j = 0; j < o->nq; ++j) {
                /* a fired readout flip: the reported bit is the outcome of -Z, the true one its complement */
                int f = op_channels(o) && fired[(size_t)(o->chan0 + j) * 64 + lane] >= 0;
                set_single_z(S, o->q[j]);
                int m = do_measure(S, 2 * f, seed, o->meas0 + j, sh);
                if (o->kind != OK_M && (m ^ f)) apply_x_on(S, o->q[j]); /* reset: flip back to |0> */
            }
            break;
        case OK_MPP: {
            int f = op_channels(o) && fired[(size_t)o->chan0 * 64 + lane] >= 0;
            int pe = op_pauli(S, o);
            do_measure(S, (pe + 2 * f) & 3, seed, o->meas0, sh);
            break;
        }
        case OK_ROT: {
            int pe = op_pauli(S, o);
            do_rotation(S, pe, o->arg, i);
            break;
        }
        case OK_FEEDBACK: {
            int par = 0;
            for (int j = 0; j < o->nrec; ++j) par ^= rec_value(C, S, o->recs[j]);
            if (par) {
                op_pauli(S, o);
                tab_apply_pauli(S, S->px, S->pz);
            }
            break;
        }
        case OK_XERR: case OK_DEP1: case OK_DEP2: case OK_CHAN: {
            int cnt = o->kind == OK_DEP2 ? o->nq / 2 : (o->kind == OK_CHAN ? 1 : o->nq);
            for (int j = 0; j < cnt; ++j) {
                int ci = o->chan0 + j;
                int br = fired[(size_t)ci * 64 + lane];
                if (br < 0) continue;
                const OChan *X = &C->ch[ci];
                memset(nx, 0, 8 * (size_t)W);
                memset(nz, 0, 8 * (size_t)W);
                if (X->kind == OK_CHAN) {
                    for (int t = 0; t < o->nq; ++t) letter_into(nx, nz, o->q[t], o->blet[br * o->nq + t]);
                } else {
                    int la, lb;
                    branch_letters(X, br, &la, &lb);
                    letter_into(nx, nz, X->qa, la);
                    if (X->kind == OK_DEP2) letter_into(nx, nz, X->qb, lb);
                }
                tab_apply_pauli(S, nx, nz);
            }
            break;
        }
        default: break;
        }
        if (S->trace) S->t_k[i] = (int16_t)S->k;
    }
}

static void write_bits(const OCirc *C, const Shot *S, uint64_t *out, int64_t n_words, int64_t wi, int lane) {
    uint64_t bit = (uint64_t)1 << lane;
    int64_t row = 0;
    for (int r = 0; r < C->n_rec; ++r, ++row)
        if (rec_value(C, S, r)) out[row * n_words + wi] |= bit;
    for (int d = 0; d < C->n_det; ++d, ++row) {
        const OOp *o = &C->ops[C->det_op[d]];
        int par = 0;
        for (int j = 0; j < o->nrec; ++j) par ^= rec_value(C, S, o->recs[j]);
        if (par) out[row * n_words + wi] |= bit;
    }
    for (int b = 0; b < C->n_obs; ++b, ++row) {
        int par = 0;
        for (int t = 0; t < C->obs_ops_n[b]; ++t) {
            const OOp *o = &C->ops[C->obs_ops[b][t]];
            for (int j = 0; j < o->nrec; ++j) par ^= rec_value(C, S, o->recs[j]);
        }
        if (par) out[row * n_words + wi] |= bit;
    }
}

/*
 * Sample shots [shot_begin, shot_begin + n_shots) (shot_begin % 64 == 0) into
 * out[row][word] (record-major, bit s%64 of word s/64 - shot_begin/64; rows are
 * visible records, then detectors, then observables).  `word_stride` is the
 * row stride of out in words.  Words are processed in parallel.
 */
int orc_sample(void *h, uint64_t seed, uint64_t shot_begin, uint64_t n_shots, uint64_t *out,
               int64_t word_stride, int threads) {
    OCirc *C = (OCirc *)h;
    if (shot_begin % 64) return -1;
    int64_t n_words = (int64_t)((n_shots + 63) / 64);
    int64_t rows = C->n_rec + C->n_det + C->n_obs;
    for (int64_t r = 0; r < rows; ++r) memset(out + r * word_stride, 0, 8 * (size_t)n_words);
    int64_t **rmap = build_rank_maps(C);
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel
#endif
    {
        Shot S;
        shot_init(&S, C);
        int16_t *fired = (int16_t *)malloc(sizeof(int16_t) * ((size_t)C->n_chan * 64 + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t wi = 0; wi < n_words; ++wi) {
            uint64_t w = shot_begin / 64 + (uint64_t)wi;
            word_events(C, seed, w, fired, rmap);
            for (int lane = 0; lane < 64; ++lane) {
                uint64_t sh = w * 64 + (uint64_t)lane;
                if (sh >= shot_begin + n_shots) break;
                run_shot(C, &S, seed, sh, fired);
                write_bits(C, &S, out, word_stride, wi, lane);
            }
        }
        free(fired);
        shot_free(&S);
    }
    free_rank_maps(C, rmap);
    return 0;
}

/*
 * Trace of one shot: per measurement kind (0 random, 1 deterministic,
 * 2 active-diagonal, 3 active-pair), outcome and Pr(m=0); per op the rotation
 * kind (0 none, 1 promote, 2 active-diagonal, 3 active-pair) and k after the
 * op; per channel the fired branch (-1 none).
 */
int orc_trace(void *h, uint64_t seed, uint64_t sh, int8_t *kind, uint8_t *m, double *p0,
              int8_t *rot, int16_t *kk, int16_t *fired_out) {
    OCirc *C = (OCirc *)h;
    int64_t **rmap = build_rank_maps(C);
    int16_t *fired = (int16_t *)malloc(sizeof(int16_t) * ((size_t)C->n_chan * 64 + 1));
    word_events(C, seed, sh / 64, fired, rmap);
    Shot S;
    shot_init(&S, C);
    S.trace = 1;
    S.t_kind = kind; S.t_p0 = p0; S.t_rot = rot; S.t_k = kk;
    for (int i = 0; i < C->n_ops; ++i) rot[i] = 0;
    run_shot(C, &S, seed, sh, fired);
    for (int t = 0; t < C->n_meas; ++t) m[t] = S.m[t];
    for (int i = 0; i < C->n_chan; ++i) fired_out[i] = fired[(size_t)i * 64 + (sh & 63)];
    shot_free(&S);
    free(fired);
    free_rank_maps(C, rmap);
    return 0;
}

/*
 * Final state of one shot: *k_out = active width after the last op; amp
 * (nullable, 2 * 2^k doubles as (re, im)) = the active vector alpha; tab_x /
 * tab_z (nullable, 2n rows of W = ceil(n / 64) words: Zbar_1..Zbar_n then
 * Xbar_1..Xbar_n) and tab_e (2n phase exponents, row = i^e X^x Z^z) = the
 * signed tableau, so that psi = sum_x alpha_x Xbar_1^x1 ... Xbar_k^xk |0bar>.
 */
int orc_final_state(void *h, uint64_t seed, uint64_t sh, int *k_out, double *amp, uint64_t *tab_x, uint64_t *tab_z,
                    int *tab_e) {
    OCirc *C = (OCirc *)h;
    int64_t **rmap = build_rank_maps(C);
    int16_t *fired = (int16_t *)malloc(sizeof(int16_t) * ((size_t)C->n_chan * 64 + 1));
    word_events(C, seed, sh / 64, fired, rmap);
    Shot S;
    shot_init(&S, C);
    run_shot(C, &S, seed, sh, fired);
    *k_out = S.k;
    if (amp)
        for (size_t x = 0; x < ((size_t)1 << S.k); ++x) {
            amp[2 * x] = creal(S.a[x]);
            amp[2 * x + 1] = cimag(S.a[x]);
        }
    size_t nw = (size_t)2 * S.n * S.W;
    if (tab_x) memcpy(tab_x, S.T.x, 8 * nw);
    if (tab_z) memcpy(tab_z, S.T.z, 8 * nw);
    if (tab_e)
        for (int r = 0; r < 2 * S.n; ++r) tab_e[r] = S.T.e[r] & 3;
    shot_free(&S);
    free(fired);
    free_rank_maps(C, rmap);
    return 0;
}

/* Per-word noise-event count of each channel over shots [shot_begin, +n_words*64):
 * counts[c] += events, branch_counts[c*16+j] += events in branch j. */
int orc_noise_counts(void *h, uint64_t seed, uint64_t word_begin, uint64_t n_words, uint64_t *counts,
                     uint64_t *branch_counts) {
    OCirc *C = (OCirc *)h;
    int64_t **rmap = build_rank_maps(C);
    int16_t *fired = (int16_t *)malloc(sizeof(int16_t) * ((size_t)C->n_chan * 64 + 1));
    for (uint64_t w = word_begin; w < word_begin + n_words; ++w) {
        word_events(C, seed, w, fired, rmap);
        for (int c = 0; c < C->n_chan; ++c)
            for (int l = 0; l < 64; ++l) {
                int br = fired[(size_t)c * 64 + l];
                if (br >= 0) { counts[c]++; if (br < 16) branch_counts[(size_t)c * 16 + br]++; }
            }
    }
    free(fired);
    free_rank_maps(C, rmap);
    return 0;
}

/* exported draw helpers for contract tests */
int orc_rmeas_bit(uint64_t seed, uint64_t t, uint64_t s) { return rmeas_bit(seed, t, s); }
double orc_active_u(uint64_t seed, uint64_t t, uint64_t s) { return active_u(seed, t, s); }
void orc_gap_table(uint64_t p32, uint64_t *Q) {
    Q[0] = (uint64_t)1 << 32;
    for (int g = 0; g < GAP_CAP; ++g) {
        unsigned __int128 prod = (unsigned __int128)Q[g] * (((uint64_t)1 << 32) - p32);
        Q[g + 1] = (uint64_t)(prod >> 32);
    }
}
