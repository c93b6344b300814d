"""Rotated surface-code Z-memory circuits (textbook construction).

Layout: d x d data qubits at (row, col); a measure qubit at every plaquette
centre (row + 1/2, col + 1/2).  Interior plaquettes form an X/Z
checkerboard; weight-2 X plaquettes sit on the top and bottom edges and
weight-2 Z plaquettes on the left and right edges, d^2 - 1 in total, so
n = 2 d^2 - 1 qubits.  Each round runs the four-layer CNOT schedule whose
corner order differs between X-type (NW, NE, SW, SE) and Z-type
(NW, SW, NE, SE) checks, so that the two kinds of check interleave
correctly and hook errors lie across the logical operator.

Noise (parameter p, all channels): X_ERROR after every reset and before every
measurement, DEPOLARIZE1 after single-qubit gates and on idle qubits of every
layer, DEPOLARIZE2 after every CNOT, DEPOLARIZE1 on the data during ancilla
measurement.  `p_meas` > 0 adds a readout flip of that probability to every
recorded measurement (the ancilla MR and the final data M).  Detectors: Z checks in round 1, every check against its
previous round from round 2 on, and each Z check's final data parity
against its last round.  Observable 0: the final Z measurements of data row 0.
Counts: M = r(d^2-1) + d^2 records, D = r(d^2-1) detectors, 1 observable.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

from .circuit import Circuit


def layout(d: int):
    data = {(r, c): r * d + c for r in range(d) for c in range(d)}
    checks: List[Tuple[str, Tuple[int, int]]] = []
    for r in range(-1, d):
        for c in range(-1, d):
            kind = "X" if (r + c) % 2 == 0 else "Z"
            interior = 0 <= r <= d - 2 and 0 <= c <= d - 2
            top_bottom = (r in (-1, d - 1)) and 0 <= c <= d - 2 and kind == "X"
            left_right = (c in (-1, d - 1)) and 0 <= r <= d - 2 and kind == "Z"
            if interior or top_bottom or left_right:
                checks.append((kind, (r, c)))
    anc: Dict[Tuple[int, int], int] = {}
    for i, (_, pos) in enumerate(checks):
        anc[pos] = d * d + i
    return data, checks, anc


def _corners(kind: str, r: int, c: int):
    nw, ne, sw, se = (r, c), (r, c + 1), (r + 1, c), (r + 1, c + 1)
    return (nw, ne, sw, se) if kind == "X" else (nw, sw, ne, se)


def rotated_memory_z(d: int, rounds: int, p: float, coherent: float = 0.0, p_meas: float = 0.0) -> Circuit:
    """`coherent` != 0 adds a coherent error exp(-i coherent Z / 2) on every data qubit at the start of every
    round (the coherent-noise surface-code family), which makes the circuit near-Clifford."""
    data, checks, anc = layout(d)
    n = 2 * d * d - 1
    circ = Circuit(n)
    dq = list(range(d * d))
    xa = [anc[pos] for kind, pos in checks if kind == "X"]
    za = [anc[pos] for kind, pos in checks if kind == "Z"]
    aq = [anc[pos] for _, pos in checks]
    all_q = list(range(n))

    # CNOT layers: list of (control, target) per layer
    layers: List[List[Tuple[int, int]]] = [[], [], [], []]
    for kind, (r, c) in checks:
        a = anc[(r, c)]
        for li, pos in enumerate(_corners(kind, r, c)):
            if pos not in data:
                continue
            q = data[pos]
            layers[li].append((a, q) if kind == "X" else (q, a))
    for lay in layers:
        used = [q for pair in lay for q in pair]
        assert len(used) == len(set(used)), "CNOT schedule collides"

    def idle(active):
        s = set(active)
        return [q for q in all_q if q not in s]

    circ.append("R", all_q)
    circ.append("X_ERROR", all_q, arg=p)
    rec_of: Dict[int, List[int]] = {a: [] for a in aq}
    for rnd in range(rounds):
        if coherent:
            for q in dq:
                circ.rot([(q, "Z")], coherent)
        circ.append("H", xa)
        circ.append("DEPOLARIZE1", xa, arg=p)
        circ.append("DEPOLARIZE1", idle(xa), arg=p)
        for lay in layers:
            flat = [q for pair in lay for q in pair]
            circ.append("CX", flat)
            circ.append("DEPOLARIZE2", flat, arg=p)
            circ.append("DEPOLARIZE1", idle(flat), arg=p)
        circ.append("H", xa)
        circ.append("DEPOLARIZE1", xa, arg=p)
        circ.append("DEPOLARIZE1", idle(xa), arg=p)
        circ.append("X_ERROR", aq, arg=p)
        base = circ.num_records
        circ.append("MR", aq, arg=p_meas)
        for i, a in enumerate(aq):
            rec_of[a].append(base + i)
        circ.append("X_ERROR", aq, arg=p)
        circ.append("DEPOLARIZE1", dq, arg=p)
        for kind, pos in checks:
            a = anc[pos]
            if rnd == 0:
                if kind == "Z":
                    circ.detector([rec_of[a][0]])
            else:
                circ.detector([rec_of[a][-1], rec_of[a][-2]])
    circ.append("X_ERROR", dq, arg=p)
    base = circ.num_records
    circ.append("M", dq, arg=p_meas)
    drec = {q: base + i for i, q in enumerate(dq)}
    for kind, (r, c) in checks:
        if kind != "Z":
            continue
        recs = [drec[data[pos]] for pos in _corners(kind, r, c) if pos in data]
        recs.append(rec_of[anc[(r, c)]][-1])
        circ.detector(recs)
    circ.observable(0, [drec[data[(0, c)]] for c in range(d)])
    return circ
