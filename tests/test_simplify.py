"""Commutation-aware rotation simplification (paper Sec. 6), compiled with
symft_compile_opts.simplify, on the CPU.

* The rewrite keeps the circuit's record distribution: exact distributions
  (dense density matrices and outcome tree) of the original and of the
  oracle's rewrite agree.
* The compiler's rewrite equals the oracle's: the same number of removed
  rotations, and the planner's width trajectory and instruction kinds equal
  the oracle's on the rewritten circuit.
* The compiled program replayed with the oracle's draws on the rewritten
  circuit gives the oracle's records bit for bit.
* Closed cases: a cancelled pair across a gate on another qubit leaves a
  pure-frame program; a gate on a shared qubit or a detector between the two
  stops the fusion; a negated Pauli turns the angle; a rotation followed by a
  measurement of the same body (or of its qubit, for Z) is removed, one of
  another body is not.
"""
import numpy as np
import pytest

import paper_2607_28600_amd as S
from oracle import OracleCircuit, dense
from oracle.simplify import simplify
from tests.program_replay import replay_shot, rows_from_measurements
from tests.randcirc import random_circuit
from workloads.circuit import Circuit, Op


def fusable_circuit(rng, n, length, p_noise=0.2):
    """A random circuit in which many rotations are followed, after zero or
    one gate on other qubits, by a rotation of the same body: its inverse
    (cancellation) or another angle (fusion), sometimes with the Pauli negated."""
    c = random_circuit(rng, n, length, p_noise=p_noise)
    ops = []
    for o in c.ops:
        ops.append(o)
        if o.name != "ROT" or rng.random() < 0.3:
            continue
        support = {q for q, _ in o.pauli}
        others = [q for q in range(n) if q not in support]
        if others and rng.random() < 0.6:
            ops.append(Op(str(rng.choice(["H", "S", "X"])), (int(rng.choice(others)),)))
        neg = bool(rng.random() < 0.5)
        want = -(-o.arg if o.negate else o.arg) if rng.random() < 0.5 else float(rng.uniform(-3, 3))
        pauli = tuple(o.pauli[::-1])
        ops.append(Op("ROT", pauli=pauli, negate=neg, arg=-want if neg else want))
        if rng.random() < 0.25:  # a measurement of the same body, which absorbs the rotation
            ops.append(Op("MPP", pauli=pauli, negate=bool(rng.random() < 0.5)))
    c.ops = ops
    return c


def _plan(c, simplify_=True):
    p = S.Program(c, simplify=simplify_)
    return p, p.plan(), p.info()["rotations_removed"]


def test_cancelled_pair_leaves_a_frame_program():
    c = Circuit(2)
    c.append("H", [0, 1])
    c.rot([(0, "Z")], 0.3)
    c.append("H", [1])
    c.rot([(0, "Z")], -0.3)
    c.append("M", [0, 1])
    p, _, removed = _plan(c)
    assert removed == 2 and p.k_max == 0
    assert S.Program(c).k_max == 1
    sc, r = simplify(c)
    assert r == 2 and all(o.name != "ROT" for o in sc.ops)


def test_fusion_stops_at_shared_qubits_and_detectors():
    c = Circuit(2)
    c.append("H", [0])
    c.rot([(0, "Z")], 0.3)
    c.append("H", [0])           # touches the rotation's qubit
    c.rot([(0, "Z")], -0.3)
    c.mpp([(0, "X")])            # another body: absorbs nothing
    assert _plan(c)[2] == 0
    c = Circuit(2)
    c.append("H", [0])
    c.append("M", [1])
    c.rot([(0, "Z")], 0.3)
    c.detector([0])              # a detector boundary
    c.rot([(0, "Z")], -0.3)
    assert _plan(c)[2] == 0
    c = Circuit(2)
    c.append("H", [0])
    c.rot([(0, "Z")], 0.3)
    c.rot([(0, "Z")], 0.3, negate=True)  # R_-Z(0.3) = R_Z(-0.3): cancels
    c.append("M", [0])
    assert _plan(c)[2] == 2


def test_rotation_before_a_measurement_of_its_body_is_removed():
    c = Circuit(3)
    c.append("H", [0, 1, 2])
    c.rot([(0, "X"), (1, "Y")], 0.7)
    c.append("H", [2])
    c.mpp([(1, "Y"), (0, "X")], negate=True)   # -P: still the same body
    c.rot([(2, "Z")], 0.4)
    c.append("MR", [2])
    c.rot([(0, "X")], 0.4)
    c.append("M", [0])                           # a Z measurement: another body, kept
    p, _, removed = _plan(c)
    assert removed == 2
    assert simplify(c)[1] == 2
    assert [o.name for o in simplify(c)[0].ops].count("ROT") == 1


@pytest.mark.parametrize("seed", range(3))
def test_rewrite_keeps_the_record_distribution(seed):
    rng = np.random.default_rng(6100 + seed)
    done = 0
    while done < 4:
        c = fusable_circuit(rng, int(rng.integers(2, 4)), int(rng.integers(6, 14)), p_noise=0.15)
        sc, removed = simplify(c)
        if removed == 0 or not 1 <= c.num_records <= 5:
            continue
        a = dense.exact_record_distribution(c)
        b = dense.exact_record_distribution(sc)
        for k in set(a) | set(b):
            assert abs(a.get(k, 0.0) - b.get(k, 0.0)) < 1e-9
        done += 1


@pytest.mark.parametrize("seed", range(3))
def test_compiler_rewrite_equals_oracle_rewrite(seed):
    rng = np.random.default_rng(6200 + seed)
    total = 0
    for trial in range(40):
        c = fusable_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(5, 40)))
        sc, removed = simplify(c)
        p, plan, got = _plan(c)
        assert got == removed
        total += removed
        tr = OracleCircuit(sc).trace(0, 0)
        assert np.array_equal(plan["k"], tr["k"])
        assert np.array_equal(plan["rot_kind"], tr["rot_kind"])
        assert np.array_equal(plan["meas_kind"], tr["meas_kind"])
    assert total > 20


@pytest.mark.parametrize("seed", range(2))
def test_simplified_program_replay_matches_oracle(seed):
    rng = np.random.default_rng(6300 + seed)
    for trial in range(30):
        c = fusable_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(5, 40)))
        sc, _ = simplify(c)
        exp = S.Program(c, simplify=True).export()
        oc = OracleCircuit(sc)
        s = 7000 + trial
        out = oc.sample(s, 128)
        for shot in (4, 99):
            tr = oc.trace(s, shot)
            mv, p0 = replay_shot(exp, sc, s, shot, tr["fired"])
            want = ((out[:, shot // 64] >> np.uint64(shot % 64)) & np.uint64(1)).astype(np.uint8)
            assert np.array_equal(rows_from_measurements(sc, mv), want)
