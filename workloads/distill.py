"""15-to-1 magic-state distillation on the [[15,1,3]] quantum Reed-Muller code
(textbook construction; stands in for the paper's distillation circuits,
whose files are external).

Qubit q carries the index i = q + 1 in 1..15.  X stabilizers: for each bit b
of i, the product of X over the qubits whose index has bit b set (4 checks
of weight 8, the parity checks of the [15,11] Hamming code).  Z stabilizers:
the same 4 weight-8 rows and, for each pair of bits, the product of Z over the
indices with both bits set (6 checks of weight 4).  Logical X = X^15 and
Z = Z^15.  On this code the transversal T^15 acts as the logical T^dagger,
so R_Z(pi/4)^15 acts as the logical R_Zbar(-pi/4).

Circuit:
1. |+>^15, then the 10 Z checks measured (random outcomes) and each outcome
   1 undone by an X-type Pauli that anticommutes with that check only, which
   leaves the logical |+>;
2. noise, R_Z(pi/4) on every qubit (the 15 noisy T gates), noise;
3. R_Zbar(+pi/4) undoes the logical rotation, so that without noise the
   state is the logical |+> again;
4. the 4 X checks and the 10 Z checks measured, one detector each
   (deterministically 0 without noise), then the logical X measured as
   observable 0 (expected 0).
Noise: DEPOLARIZE1(p) before and after the T layer, or, with `z_only`, a
Z-only Pauli channel of probability p after it.  Postselecting every detector
keeps the shots a 15-to-1 protocol keeps; a kept shot with observable 1 is a
logical error.
"""
from __future__ import annotations

from typing import List

from .circuit import Circuit

N = 15


def x_checks() -> List[List[int]]:
    return [[q for q in range(N) if ((q + 1) >> b) & 1] for b in range(4)]


def z_checks() -> List[List[int]]:
    rows = [[q for q in range(N) if ((q + 1) >> b) & 1] for b in range(4)]
    for b in range(4):
        for c in range(b + 1, 4):
            rows.append([q for q in range(N) if ((q + 1) >> b) & 1 and ((q + 1) >> c) & 1])
    return rows


def _destabilizers(rows: List[List[int]]) -> List[List[int]]:
    """For each Z check j an X-type support v_j with |v_j & row_k| odd iff
    k == j (plain GF(2) elimination on the 10 x 15 check matrix)."""
    m = len(rows)
    A = [[1 if q in r else 0 for q in range(N)] + [1 if j == i else 0 for j in range(m)] for i, r in enumerate(rows)]
    piv = []
    r = 0
    for col in range(N):
        p = next((i for i in range(r, m) if A[i][col]), None)
        if p is None:
            continue
        A[r], A[p] = A[p], A[r]
        for i in range(m):
            if i != r and A[i][col]:
                A[i] = [a ^ b for a, b in zip(A[i], A[r])]
        piv.append(col)
        r += 1
    assert r == m, "Z checks are not independent"
    # reduced row i = sum_j M_ij row_j (M the right block) has a 1 at column
    # piv_i and 0 at the other pivots, so v_j = sum_i M_ij e_(piv_i) meets
    # row k in sum_i (M^-1)_ki M_ij = [j == k]
    out = []
    for j in range(m):
        v = [0] * N
        for i in range(m):
            if A[i][N + j]:
                v[piv[i]] = 1
        out.append([q for q in range(N) if v[q]])
    for j, v in enumerate(out):
        for k, row in enumerate(rows):
            assert (len(set(v) & set(row)) % 2) == (1 if j == k else 0)
    return out


def distill_15to1(p: float, z_only: bool = False) -> Circuit:
    c = Circuit(N)
    allq = list(range(N))
    c.append("H", allq)
    zc, xc = z_checks(), x_checks()
    first = [c.mpp([(q, "Z") for q in row]) for row in zc]
    for rec, v in zip(first, _destabilizers(zc)):
        c.feedback([(q, "X") for q in v], [rec])
    if not z_only:
        c.append("DEPOLARIZE1", allq, arg=p)
    for q in allq:
        c.rot([(q, "Z")], 0.7853981633974483)
    if z_only:
        for q in allq:
            c.append("PAULI_CHANNEL", [q], branches=((p, "Z"),))
    else:
        c.append("DEPOLARIZE1", allq, arg=p)
    c.rot([(q, "Z") for q in allq], 0.7853981633974483)
    for row in xc:
        c.detector([c.mpp([(q, "X") for q in row])])
    for row in zc:
        c.detector([c.mpp([(q, "Z") for q in row])])
    c.observable(0, [c.mpp([(q, "X") for q in allq])])
    return c
