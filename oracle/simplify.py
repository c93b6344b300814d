"""Rotation fusion and cancellation before planning (paper Sec. 6,
commutation-aware simplification), as the oracle states it.

TEST INFRASTRUCTURE ONLY, written apart from the GPU library's pass: the
oracle runs on the simplified circuit, because the rewrite can change how a
later operation is classified (a cancelled pair never promotes a coordinate).

The conservative rule: a rotation R_P(b) is merged into an earlier R_P(a) of
the same Pauli body (the same set of (qubit, letter) pairs; a negated Pauli
turns the angle's sign, R_-P(t) = R_P(-t)) when every operation between them
acts only on qubits outside P's support and no detector annotation lies
between them.  Operations on other qubits commute with P, so the later
rotation can move next to the earlier one, and R_P(a) R_P(b) = R_P(a + b).
The merged rotation stays at the earlier place; the later operation becomes a
TICK (nothing), so operation indices are kept.  A merged angle that is a
multiple of 2 pi leaves -I or I, a global phase, and the earlier rotation
goes too.  A rotation that reaches, under the same condition, a measurement of
+-P (an MPP of the same body, or M / MR / R of qubit q when P = Z_q) only
multiplies each outcome's branch by a phase, since the measurement's
projectors are eigenspaces of P, so it is removed.
"""
from __future__ import annotations

import math
from dataclasses import replace
from typing import Tuple

from workloads.circuit import Circuit, Op


def _signed(o: Op) -> float:
    return -o.arg if o.negate else o.arg


def _valid_body(o: Op) -> bool:
    qs = [q for q, _ in o.pauli]
    return len(qs) > 0 and len(set(qs)) == len(qs) and all(s in "XYZ" for _, s in o.pauli)


def simplify(circ: Circuit) -> Tuple[Circuit, int]:
    ops = list(circ.ops)
    removed = 0
    for i in range(len(ops)):
        o = ops[i]
        if o.name != "ROT" or not _valid_body(o):
            continue
        body = frozenset(o.pauli)
        support = {q for q, _ in o.pauli}
        theta = _signed(o)
        merged = absorbed = False
        for j in range(i + 1, len(ops)):
            x = ops[j]
            if x.name == "DETECTOR":
                break
            if x.name == "ROT" and len(x.pauli) == len(o.pauli) and frozenset(x.pauli) == body:
                theta += _signed(x)
                ops[j] = Op("TICK")
                removed += 1
                merged = True
                continue
            if support & (set(x.targets) | {q for q, _ in x.pauli}):
                if x.name == "MPP":
                    absorbed = len(x.pauli) == len(o.pauli) and frozenset(x.pauli) == body
                elif x.name in ("M", "MR", "R"):
                    absorbed = len(o.pauli) == 1 and o.pauli[0][1] == "Z"
                break
        if absorbed:
            ops[i] = Op("TICK")
            removed += 1
            continue
        if not merged:
            continue
        if abs(math.remainder(theta, 2 * math.pi)) < 1e-12:
            ops[i] = Op("TICK")
            removed += 1
        else:
            ops[i] = replace(o, arg=theta, negate=False)
    out = Circuit(circ.n_qubits)
    out.ops = ops
    return out, removed
