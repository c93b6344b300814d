"""Seeded near-Clifford circuits with a controlled peak active width.

Shape (stand-in for the paper's near-Clifford workloads, whose circuit files
are not available): n qubits, `layers` layers of random Clifford gates (a
random permutation pairs the first 2*n_cx qubits into CNOTs of random
orientation; each remaining qubit gets H, S or nothing), DEPOLARIZE1(p) after
H/S and DEPOLARIZE2(p) after every CNOT; pi/8 rotations exp(-i pi/8 P)
(theta = pi/4) and Pauli-product measurements at random layer boundaries;
after a measurement, with probability 1/2, a feedback Pauli on 1-3 qubits
conditioned on the parity of 1-2 of the last 8 records.

Steering the active width.  Random Pauli products on a scrambled register
would almost surely promote a fresh coordinate at every rotation and never
return one, so the generator keeps unsigned, forward-propagated bookkeeping
of the Paulis it has placed (propagation through H, S and CNOT only; no
signs, no amplitudes):
  * "closers": each opened rotation's Pauli, propagated forward; measuring it
    later returns that coordinate;
  * "known stabilizers": measured Paulis (and the initial Z_q), propagated
    forward while nothing anticommuting has been measured since.
A new rotation is drawn (weight 2..6) to commute with all open closers, so
that every coordinate stays returnable.  Further rotations about an open
closer (or a product of two) act inside the active space; rotations about a
known stabilizer that anticommutes with an open closer act diagonally.
Measurements either return a coordinate (measure a closer, or a known
stabilizer that anticommutes with open closers), re-measure a known
stabilizer that commutes with every closer, or measure a fresh weight-1..4
Pauli drawn to commute with all open closers.  None of this bookkeeping is
checked here; the planned peak width is measured downstream, and the seeds
in ``seeds.json`` are the ones whose width hits the target.
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np

from .circuit import Circuit

THETA_PI8 = np.pi / 4  # exp(-i pi/8 P) = R_P(pi/4)


class _Tracked:
    """Unsigned Paulis as bool rows, propagated forward through Cliffords."""

    def __init__(self, n: int):
        self.n = n
        self.x = np.zeros((0, n), dtype=bool)
        self.z = np.zeros((0, n), dtype=bool)

    def add(self, x: np.ndarray, z: np.ndarray) -> int:
        self.x = np.vstack([self.x, x[None, :]])
        self.z = np.vstack([self.z, z[None, :]])
        return self.x.shape[0] - 1

    def h(self, q):
        self.x[:, q], self.z[:, q] = self.z[:, q].copy(), self.x[:, q].copy()

    def s(self, q):
        self.z[:, q] ^= self.x[:, q]

    def cx(self, c, t):
        self.x[:, t] ^= self.x[:, c]
        self.z[:, c] ^= self.z[:, t]


def _anti(x1, z1, x2, z2) -> bool:
    return bool((np.count_nonzero(x1 & z2) + np.count_nonzero(z1 & x2)) & 1)


def _to_pauli(x, z) -> List[Tuple[int, str]]:
    out = []
    for q in range(len(x)):
        if x[q] and z[q]:
            out.append((q, "Y"))
        elif x[q]:
            out.append((q, "X"))
        elif z[q]:
            out.append((q, "Z"))
    return out


def _rand_paulis(rng, n, wmin, wmax, count):
    """`count` random Paulis with weight uniform in [wmin, wmax] and letters uniform in X, Y, Z."""
    w = rng.integers(wmin, min(wmax, n) + 1, size=count)
    keys = rng.random((count, n))
    order = np.argsort(keys, axis=1)
    chosen = np.zeros((count, n), dtype=bool)
    ranks = np.empty_like(order)
    np.put_along_axis(ranks, order, np.arange(n)[None, :].repeat(count, 0), axis=1)
    chosen = ranks < w[:, None]
    L = rng.integers(1, 4, size=(count, n))
    x = chosen & ((L == 1) | (L == 2))
    z = chosen & ((L == 2) | (L == 3))
    return x, z


def _rand_pauli(rng, n, wmin, wmax):
    w = int(rng.integers(wmin, min(wmax, n) + 1))
    qs = rng.choice(n, w, replace=False)
    x = np.zeros(n, dtype=bool)
    z = np.zeros(n, dtype=bool)
    for q in qs:
        L = int(rng.integers(1, 4))
        x[q] = L in (1, 2)
        z[q] = L in (2, 3)
    return x, z


def near_clifford(n: int, layers: int, n_rot: int, n_meas: int, k_target: int, p: float, seed: int,
                  n_cx: Optional[int] = None, feedback_prob: float = 0.5,
                  active_rot_prob: float = 0.35, front_load: bool = False) -> Circuit:
    rng = np.random.default_rng(seed)
    if n_cx is None:
        n_cx = min(5, n // 4)
    circ = Circuit(n)
    # events at layer boundaries: 'R' rotations and 'M' measurements
    if front_load:
        rot_at = np.sort(rng.integers(0, max(1, layers // 3), n_rot))
    else:
        rot_at = np.sort(rng.integers(0, layers, n_rot))
    meas_at = np.sort(rng.integers(0, layers + 1, n_meas))
    events: List[Tuple[int, int, str]] = [(int(l), 0, "R") for l in rot_at] + [(int(l), 1, "M") for l in meas_at]
    events.sort()

    closers = _Tracked(n)       # rows = open rotation Paulis (propagated)
    open_ids: List[int] = []    # rows of `closers` still open
    stabs = _Tracked(n)         # known stabilizers (propagated)
    valid: List[bool] = []
    for q in range(n):
        x = np.zeros(n, dtype=bool)
        z = np.zeros(n, dtype=bool)
        z[q] = True
        stabs.add(x, z)
        valid.append(True)

    def layer():
        perm = rng.permutation(n)
        cx = []
        for i in range(n_cx):
            a, b = int(perm[2 * i]), int(perm[2 * i + 1])
            if rng.random() < 0.5:
                a, b = b, a
            cx += [a, b]
        hs, ss = [], []
        for q in perm[2 * n_cx:]:
            r = rng.random()
            if r < 1 / 3:
                hs.append(int(q))
            elif r < 2 / 3:
                ss.append(int(q))
        if cx:
            circ.append("CX", cx)
            for i in range(0, len(cx), 2):
                closers.cx(cx[i], cx[i + 1])
                stabs.cx(cx[i], cx[i + 1])
            circ.append("DEPOLARIZE2", cx, arg=p)
        if hs:
            circ.append("H", hs)
            for q in hs:
                closers.h(q)
                stabs.h(q)
        if ss:
            circ.append("S", ss)
            for q in ss:
                closers.s(q)
                stabs.s(q)
        if hs or ss:
            circ.append("DEPOLARIZE1", hs + ss, arg=p)

    def draw_commuting(wmin, wmax):
        """A random Pauli that commutes with every open closer (batched rejection)."""
        if not open_ids:
            return _rand_pauli(rng, n, wmin, wmax)
        ox = closers.x[open_ids].astype(np.int32)
        oz = closers.z[open_ids].astype(np.int32)
        for _ in range(4096):
            x, z = _rand_paulis(rng, n, wmin, wmax, 4096)
            anti = (x.astype(np.int32) @ oz.T + z.astype(np.int32) @ ox.T) & 1
            ok = np.flatnonzero(~anti.any(axis=1))
            if ok.size:
                return x[ok[0]].copy(), z[ok[0]].copy()
        raise RuntimeError("no commuting Pauli found")

    def commutes_with_open(x, z) -> bool:
        for i in open_ids:
            if _anti(x, z, closers.x[i], closers.z[i]):
                return False
        return True

    def invalidate_against(x, z):
        for j in range(len(valid)):
            if valid[j] and _anti(x, z, stabs.x[j], stabs.z[j]):
                valid[j] = False

    def record_stab(x, z):
        invalidate_against(x, z)
        stabs.add(x.copy(), z.copy())
        valid.append(True)

    def add_feedback():
        if rng.random() >= feedback_prob:
            return
        nr = circ.num_records
        lo = max(0, nr - 8)
        cnt = int(rng.integers(1, 3))
        recs = sorted(set(int(r) for r in rng.integers(lo, nr, cnt)))
        fx, fz = _rand_pauli(rng, n, 1, 3)
        circ.feedback(_to_pauli(fx, fz), recs)

    def diag_candidates():
        out = []
        for j in range(len(valid)):
            if not valid[j]:
                continue
            sx, sz = stabs.x[j], stabs.z[j]
            if any(_anti(sx, sz, closers.x[i], closers.z[i]) for i in open_ids):
                out.append(j)
        return out

    ei = 0
    for L in range(layers + 1):
        while ei < len(events) and events[ei][0] == L:
            _, _, kind = events[ei]
            ei += 1
            if kind == "R":
                want_open = len(open_ids) < k_target and (not open_ids or rng.random() >= active_rot_prob)
                if want_open:
                    x, z = draw_commuting(2, 6)
                    circ.rot(_to_pauli(x, z), THETA_PI8)
                    open_ids.append(closers.add(x, z))
                elif open_ids:
                    cands = diag_candidates()
                    if cands and rng.random() < 0.4:
                        j = int(rng.choice(cands))
                        circ.rot(_to_pauli(stabs.x[j], stabs.z[j]), THETA_PI8)
                    else:
                        i = int(rng.choice(open_ids))
                        x, z = closers.x[i].copy(), closers.z[i].copy()
                        if len(open_ids) > 1 and rng.random() < 0.5:
                            i2 = int(rng.choice([o for o in open_ids if o != i]))
                            x ^= closers.x[i2]
                            z ^= closers.z[i2]
                        circ.rot(_to_pauli(x, z), THETA_PI8)
                else:
                    x, z = _rand_pauli(rng, n, 2, 6)
                    circ.rot(_to_pauli(x, z), THETA_PI8)
                    open_ids.append(closers.add(x, z))
            else:
                r = rng.random()
                close_bias = len(open_ids) / max(k_target, 1)
                if open_ids and r < 0.55 * close_bias:
                    cands = diag_candidates()
                    if cands and rng.random() < 0.4:
                        j = int(rng.choice(cands))
                        sx, sz = stabs.x[j].copy(), stabs.z[j].copy()
                        circ.mpp(_to_pauli(sx, sz))
                        anti = [i for i in open_ids if _anti(sx, sz, closers.x[i], closers.z[i])]
                        drop = anti[0]
                        for i in anti[1:]:
                            closers.x[i] ^= closers.x[drop]
                            closers.z[i] ^= closers.z[drop]
                        open_ids.remove(drop)
                        invalidate_against(sx, sz)
                        valid[j] = True
                    else:
                        i = int(rng.choice(open_ids))
                        x, z = closers.x[i].copy(), closers.z[i].copy()
                        circ.mpp(_to_pauli(x, z))
                        open_ids.remove(i)
                        record_stab(x, z)
                else:
                    det = [j for j in range(len(valid)) if valid[j] and commutes_with_open(stabs.x[j], stabs.z[j])]
                    if det and rng.random() < 0.2:
                        j = int(rng.choice(det))
                        circ.mpp(_to_pauli(stabs.x[j], stabs.z[j]))
                    else:
                        x, z = draw_commuting(1, 4)
                        circ.mpp(_to_pauli(x, z))
                        record_stab(x, z)
                add_feedback()
        if L < layers:
            layer()
    return circ


# -- the benchmark workloads -----------------------------------------------

def c3(seed: int = 3) -> Circuit:
    """n=20, 400 layers, 24 pi/8 rotations (weight 2..6), 60 measurements, p=5e-4, peak width 8."""
    return near_clifford(20, 400, 24, 60, 8, 5e-4, seed)


def c4_params(i: int):
    """Program i of the 128-program batch: (n, k_target, shots) with shots log-uniform in [2^10, 2^18]."""
    n = 12 + (i % 29)
    k = 1 + (i % 12)
    u = np.random.default_rng(4000 + i).random()
    shots = 64 * max(1, int(round(2 ** (10 + 8 * u) / 64)))
    return n, k, shots


def c4_program(i: int, seed: int) -> Circuit:
    n, k, _ = c4_params(i)
    return near_clifford(n, 100, 2 * k + 4, 2 * k + 12, k, 5e-4, seed)


def c5(seed: int = 5, k_target: int = 14) -> Circuit:
    """n=48, 400 layers, 80 pi/8 rotations, 200 measurements with feedback, p=5e-4."""
    return near_clifford(48, 400, 80, 200, k_target, 5e-4, seed, n_cx=8, front_load=(k_target > 14))
