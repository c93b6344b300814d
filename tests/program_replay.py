"""FP64 replay of an exported SymFT program on the CPU (test harness only).

It applies the seven instruction semantics of the paper (Sec. 4.1 / 4.2 / 5)
to one shot, given that shot's noise branches and draws, so that the host
compiler's output (pulled-back Paulis, pivots, mu, eta and every sign
expression) can be checked against the oracle on the CPU before any kernel
runs.  It is not the oracle and not the product path: the draws it consumes
are the oracle's, and its result is compared with the oracle's records.
"""
from __future__ import annotations

import numpy as np

import oracle


def _insert(z, h, v):
    lo = z & ((1 << h) - 1)
    return lo | (v << h) | ((z >> h) << (h + 1))


def _par(v):
    return bin(v).count("1") & 1


def replay_shot(exp, circ, seed, shot, fired, return_state=False):
    instr, theta = exp["instr"], exp["theta"]
    noise_refs, meas_refs = exp["noise"], exp["meas"]
    chan, bmask = exp["chan"], exp["bmask"]
    n_sym = int((chan[:, 0] + chan[:, 1]).max()) if len(chan) else 0
    sym = np.zeros(max(n_sym, 1), dtype=np.uint8)
    for c, b in enumerate(fired):
        b = int(b)
        if b >= 0:
            s0, ns, J, off = (int(v) for v in chan[c])
            m = int(bmask[off + b])
            for i in range(ns):
                if (m >> i) & 1:
                    sym[s0 + i] = 1
    n_meas = circ.num_measurements
    mvals = np.zeros(n_meas, dtype=np.uint8)
    p0s = np.full(n_meas, np.nan)
    a = np.ones(1, dtype=complex)
    for i in range(len(instr)):
        kind, k, h, mu, eta, lc, am, bm, t, no, nl, mo, ml = (int(v) for v in instr[i])
        lam = lc
        for s in noise_refs[no:no + nl]:
            lam ^= int(sym[s])
        for u in meas_refs[mo:mo + ml]:
            lam ^= int(mvals[u])
        c, s = np.cos(theta[i] / 2), np.sin(theta[i] / 2)
        N = 1 << k
        if kind == 1:  # PromoteRot
            sg = -1 if lam else 1
            a = np.concatenate([c * a, -1j * sg * s * a])
        elif kind == 2:  # ActiveDiagRot
            muv = 1 if mu == 0 else -1
            for x in range(N):
                sig = (-1) ** lam * muv * (-1) ** _par(bm & x)
                a[x] *= (c - 1j * sig * s)
        elif kind == 3:  # ActivePairRot
            muv = 1j ** mu
            new = a.copy()
            for x in range(N):
                y = x ^ am
                new[x] = c * a[x] - 1j * (-1) ** lam * s * muv * (-1) ** _par(bm & y) * a[y]
            a = new
        elif kind == 4:  # RandomMeas
            mvals[t] = oracle.rmeas_bit(seed, t, shot)
            p0s[t] = 0.5
        elif kind == 5:  # DetMeas
            mvals[t] = lam ^ eta
            p0s[t] = 0.0 if mvals[t] else 1.0
        elif kind == 6:  # ActiveDiagMeas
            w = np.abs(a) ** 2
            cls = np.array([_par(bm & x) for x in range(N)])
            S = [w[cls == 0].sum(), w[cls == 1].sum()]
            flip = lam ^ eta
            p0 = S[flip] / (S[0] + S[1])
            m = 0 if oracle.active_u(seed, t, shot) < p0 else 1
            y = m ^ flip
            bl = bm & ~(1 << h)
            new = np.zeros(N // 2, dtype=complex)
            for z in range(N // 2):
                u = _insert(z, h, y)
                x = u ^ (_par(bl & u) << h)
                new[z] = a[x] / np.sqrt(S[y])
            a = new
            mvals[t] = m
            p0s[t] = p0
        elif kind == 7:  # ActivePairMeas
            mc = np.conj(1j ** mu)
            beta = np.zeros((2, N // 2), dtype=complex)
            for z in range(N // 2):
                u0 = _insert(z, h, 0)
                for yy in (0, 1):
                    beta[yy, z] = (a[u0] + mc * (-1) ** (_par(bm & u0) ^ yy) * a[u0 ^ am]) / np.sqrt(2)
            S = (np.abs(beta) ** 2).sum(axis=1)
            p0 = S[lam] / S.sum()
            m = 0 if oracle.active_u(seed, t, shot) < p0 else 1
            y = m ^ lam
            a = beta[y] / np.sqrt(S[y])
            mvals[t] = m
            p0s[t] = p0
    if return_state:
        return mvals, p0s, a
    return mvals, p0s


def rows_from_measurements(circ, mvals):
    recs = []
    t = 0
    for o in circ.ops:
        if o.name in ("R", "M", "MR"):
            for _ in o.targets:
                if o.name != "R":
                    recs.append(int(mvals[t]))
                t += 1
        elif o.name == "MPP":
            recs.append(int(mvals[t]))
            t += 1
    from oracle.dense import records_to_rows
    return records_to_rows(circ, recs)
