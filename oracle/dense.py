"""Plain dense state-vector / density-matrix brute force (test infrastructure only).

This is the paper's circuit semantics (Sec. 2) written out directly on a
2^n vector, for n <= 12: Clifford gates as matrices, R_P(theta) =
cos(theta/2) I - i sin(theta/2) P, projectors (I + (-1)^m P)/2 (m = 0 for the
+1 eigenvalue), stochastic Pauli channels and record-parity feedback.  It is
independent of the tableau oracle and pins it: given the noise branches and
outcomes a tableau shot took, ``replay`` recomputes every Pr(m = 0) by
projection.  ``exact_record_distribution`` enumerates the outcome tree (with
density matrices for noise) to give exact record probabilities for small
circuits.  Qubit q is bit q of the basis index.

Readout flips (an M / MR / MPP with ``arg`` = p > 0; paper Sec. 6 counts them
among the exogenous symbols) are taken by their plain definition: the state
is projected on the true outcome and, with probability p, the complement of
that outcome is recorded; a reset acts on the true outcome.  Each flip is one
channel, in circuit order with the noise channels.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Sequence, Tuple

import numpy as np

_I2 = np.eye(2, dtype=complex)
_X = np.array([[0, 1], [1, 0]], dtype=complex)
_Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
_Z = np.array([[1, 0], [0, -1]], dtype=complex)
_H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
_S = np.array([[1, 0], [0, 1j]], dtype=complex)
PAULI_MATS = {"I": _I2, "X": _X, "Y": _Y, "Z": _Z}
GATE_1Q = {"H": _H, "S": _S, "S_DAG": _S.conj().T, "X": _X, "Y": _Y, "Z": _Z}


def _cx():
    m = np.zeros((4, 4), dtype=complex)
    # basis |c t>, index = 2*c + t
    for c in (0, 1):
        for t in (0, 1):
            m[2 * c + (t ^ c), 2 * c + t] = 1
    return m


GATE_2Q = {
    "CX": _cx(),
    "CZ": np.diag([1, 1, 1, -1]).astype(complex),
    "SWAP": np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=complex),
}

D1_BRANCHES = ("X", "Y", "Z")
D2_BRANCHES = tuple(a + b for a in "IXYZ" for b in "IXYZ" if a + b != "II")


def apply_1q(psi: np.ndarray, n: int, U: np.ndarray, q: int) -> np.ndarray:
    t = psi.reshape((2,) * n)
    ax = n - 1 - q
    t = np.moveaxis(np.tensordot(U, t, axes=([1], [ax])), 0, ax)
    return t.reshape(-1)


def apply_2q(psi: np.ndarray, n: int, U: np.ndarray, qa: int, qb: int) -> np.ndarray:
    """U acts on |a b> with index 2*a + b."""
    t = psi.reshape((2,) * n)
    aa, ab = n - 1 - qa, n - 1 - qb
    U4 = U.reshape(2, 2, 2, 2)
    t = np.tensordot(U4, t, axes=([2, 3], [aa, ab]))
    t = np.moveaxis(t, [0, 1], [aa, ab])
    return t.reshape(-1)


def pauli_apply(psi: np.ndarray, n: int, pauli: Sequence[Tuple[int, str]], negate: bool = False) -> np.ndarray:
    out = psi.copy()
    for q, s in pauli:
        out = apply_1q(out, n, PAULI_MATS[s], q)
    return -out if negate else out


def pauli_matrix(n: int, pauli: Sequence[Tuple[int, str]], negate: bool = False) -> np.ndarray:
    M = np.eye(2 ** n, dtype=complex)
    cols = [pauli_apply(M[:, j], n, pauli, negate) for j in range(2 ** n)]
    return np.stack(cols, axis=1)


def _noise_branches(op) -> List[Tuple[Tuple[int, ...], Tuple[float, ...], Tuple[str, ...]]]:
    """Channels of one noise op: (qubits, branch probabilities, branch letters)."""
    out = []
    if op.name == "X_ERROR":
        for q in op.targets:
            out.append(((q,), (op.arg,), ("X",)))
    elif op.name == "DEPOLARIZE1":
        for q in op.targets:
            out.append(((q,), (op.arg / 3,) * 3, D1_BRANCHES))
    elif op.name == "DEPOLARIZE2":
        for i in range(0, len(op.targets), 2):
            out.append(((op.targets[i], op.targets[i + 1]), (op.arg / 15,) * 15, D2_BRANCHES))
    elif op.name == "PAULI_CHANNEL":
        out.append((tuple(op.targets), tuple(p for p, _ in op.branches), tuple(s for _, s in op.branches)))
    return out


def _apply_letters(psi, n, qubits, letters):
    for q, s in zip(qubits, letters):
        if s != "I":
            psi = apply_1q(psi, n, PAULI_MATS[s], q)
    return psi


def replay(circ, fired: Sequence[int], outcomes: Sequence[int]) -> Dict[str, np.ndarray]:
    """Re-run one shot on a dense vector with the given noise branches (per
    channel, -1 = none) and measurement outcomes (all measurements, resets
    included).  Returns Pr(m=0) of every measurement and the final state."""
    n = circ.n_qubits
    psi = np.zeros(2 ** n, dtype=complex)
    psi[0] = 1.0
    p0s: List[float] = []
    recs: List[int] = []
    t = 0
    ch = 0

    def flip_fired(op):
        # the op's next readout-flip channel, if it has them
        nonlocal ch
        if op.name == "R" or op.arg <= 0:
            return 0
        f = int(fired[ch]) >= 0
        ch += 1
        return int(f)

    def measure(psi, P, negate=False, flip=0):
        # `outcomes` holds reported bits; the true outcome is the reported one
        # XOR the flip, and Pr(m = 0) is returned for the reported bit
        nonlocal t
        Ppsi = pauli_apply(psi, n, P, negate)
        plus = (psi + Ppsi) / 2
        p0 = float(np.vdot(plus, plus).real)
        m = int(outcomes[t]) ^ flip
        proj = plus if m == 0 else (psi - Ppsi) / 2
        pr = float(np.vdot(proj, proj).real)
        if pr <= 1e-14:
            raise AssertionError(f"measurement {t}: outcome {m} has probability {pr}")
        p0s.append(1.0 - p0 if flip else p0)
        t += 1
        return proj / np.sqrt(pr), m

    for op in circ.ops:
        nm = op.name
        if nm in GATE_1Q:
            for q in op.targets:
                psi = apply_1q(psi, n, GATE_1Q[nm], q)
        elif nm in GATE_2Q:
            for i in range(0, len(op.targets), 2):
                psi = apply_2q(psi, n, GATE_2Q[nm], op.targets[i], op.targets[i + 1])
        elif nm in ("R", "M", "MR"):
            for q in op.targets:
                f = flip_fired(op)
                psi, m = measure(psi, ((q, "Z"),), flip=f)
                if nm != "R":
                    recs.append(m ^ f)
                if nm != "M" and m:
                    psi = apply_1q(psi, n, _X, q)
        elif nm == "MPP":
            f = flip_fired(op)
            psi, m = measure(psi, op.pauli, op.negate, flip=f)
            recs.append(m ^ f)
        elif nm == "ROT":
            c, s = np.cos(op.arg / 2), np.sin(op.arg / 2)
            psi = c * psi - 1j * s * pauli_apply(psi, n, op.pauli, op.negate)
        elif nm == "FEEDBACK":
            if sum(recs[r] for r in op.recs) % 2:
                psi = pauli_apply(psi, n, op.pauli)
        elif nm in ("X_ERROR", "DEPOLARIZE1", "DEPOLARIZE2", "PAULI_CHANNEL"):
            for qubits, _, letters in _noise_branches(op):
                b = int(fired[ch])
                ch += 1
                if b >= 0:
                    psi = _apply_letters(psi, n, qubits, letters[b])
    return {"p0": np.asarray(p0s), "state": psi, "records": np.asarray(recs, dtype=np.uint8)}


def exact_record_distribution(circ, cutoff: float = 1e-15) -> Dict[Tuple[int, ...], float]:
    """Exact probability of every visible record tuple (density matrices for
    noise, an explicit outcome tree for measurements).  Small circuits only."""
    n = circ.n_qubits
    dim = 2 ** n
    rho0 = np.zeros((dim, dim), dtype=complex)
    rho0[0, 0] = 1
    cache_pm: Dict = {}

    def pmat(P, negate=False):
        key = (tuple(P), negate)
        if key not in cache_pm:
            cache_pm[key] = pauli_matrix(n, P, negate)
        return cache_pm[key]

    def unitary_1q(U, q):
        M = np.eye(dim, dtype=complex)
        return np.stack([apply_1q(M[:, j], n, U, q) for j in range(dim)], axis=1)

    def unitary_2q(U, a, b):
        M = np.eye(dim, dtype=complex)
        return np.stack([apply_2q(M[:, j], n, U, a, b) for j in range(dim)], axis=1)

    result: Dict[Tuple[int, ...], float] = {}

    def rec(i, rho, prob, recs):
        if prob < cutoff:
            return
        while i < len(circ.ops):
            op = circ.ops[i]
            nm = op.name
            if nm in GATE_1Q:
                for q in op.targets:
                    U = unitary_1q(GATE_1Q[nm], q)
                    rho = U @ rho @ U.conj().T
            elif nm in GATE_2Q:
                for j in range(0, len(op.targets), 2):
                    U = unitary_2q(GATE_2Q[nm], op.targets[j], op.targets[j + 1])
                    rho = U @ rho @ U.conj().T
            elif nm == "ROT":
                P = pmat(op.pauli, op.negate)
                U = np.cos(op.arg / 2) * np.eye(dim) - 1j * np.sin(op.arg / 2) * P
                rho = U @ rho @ U.conj().T
            elif nm in ("X_ERROR", "DEPOLARIZE1", "DEPOLARIZE2", "PAULI_CHANNEL"):
                for qubits, probs, letters in _noise_branches(op):
                    new = (1 - sum(probs)) * rho
                    for p, L in zip(probs, letters):
                        P = pmat(tuple((q, s) for q, s in zip(qubits, L) if s != "I"))
                        new = new + p * (P @ rho @ P.conj().T)
                    rho = new
            elif nm == "FEEDBACK":
                if sum(recs[r] for r in op.recs) % 2:
                    P = pmat(op.pauli)
                    rho = P @ rho @ P.conj().T
            elif nm in ("R", "M", "MR", "MPP"):
                if nm == "MPP":
                    Ps = [(op.pauli, op.negate, None)]
                else:
                    Ps = [(((q, "Z"),), False, q) for q in op.targets]
                # expand this op's measurements one by one (branching)
                def branch(j, rho, prob, recs):
                    if j == len(Ps):
                        rec(i + 1, rho, prob, recs)
                        return
                    P, neg, q = Ps[j]
                    PM = pmat(P, neg)
                    pf = op.arg if nm != "R" else 0.0  # readout flip of the recorded bit
                    for m in (0, 1):
                        Pi = (np.eye(dim) + (-1) ** m * PM) / 2
                        r2 = Pi @ rho @ Pi
                        pm = float(np.trace(r2).real)
                        if pm * prob < cutoff:
                            continue
                        r2 = r2 / pm
                        if nm in ("R", "MR") and m:
                            Xq = pmat(((q, "X"),))
                            r2 = Xq @ r2 @ Xq
                        if nm == "R":
                            branch(j + 1, r2, prob * pm, recs)
                            continue
                        for f, pr in ((0, 1.0 - pf), (1, pf)):
                            if pr > 0:
                                branch(j + 1, r2, prob * pm * pr, recs + [m ^ f])
                branch(0, rho, prob, recs)
                return
            i += 1
        key = tuple(recs)
        result[key] = result.get(key, 0.0) + prob

    rec(0, rho0, 1.0, [])
    return result


def records_to_rows(circ, recs: Sequence[int]) -> np.ndarray:
    """Visible records -> full row vector (records, detectors, observables)."""
    rows = list(int(r) for r in recs)
    for op in circ.ops:
        if op.name == "DETECTOR":
            rows.append(sum(recs[r] for r in op.recs) % 2)
    n_obs = circ.num_observables
    obs = [0] * n_obs
    for op in circ.ops:
        if op.name == "OBSERVABLE_INCLUDE":
            obs[op.obs] ^= sum(recs[r] for r in op.recs) % 2
    return np.asarray(rows + obs, dtype=np.uint8)


def enumerate_paulis(nq: int):
    for letters in itertools.product("IXYZ", repeat=nq):
        yield "".join(letters)
