"""Pins of the CPU oracle against things other than itself.

* Philox4x32-10 known-answer vectors (Random123 publication; rocRAND).
* Clifford conjugation rules, exhaustively on 1-2 qubits, against explicit matrices.
* Every Pr(m=0) of the tableau oracle against dense projection (paper eq. for the
  factorized branch probability: the probability is the norm of the projected state).
* Closed forms for each instruction kind (paper Sec. 4.1 / 4.2).
* Exact record distributions (density matrices + outcome tree) vs oracle histograms.
* Noiseless detector determinism; surface-code counts vs the paper's d=7/9 figures.
* The whole final state (signed tableau + active vector) against the dense replay.
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import OracleCircuit, dense
from tests.randcirc import random_circuit
from workloads.circuit import Circuit
from workloads.surface import rotated_memory_z

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = oracle.philox(r[0:4], r[4:6])
        assert [int(v) for v in out] == r[6:10]


def _pauli_mat(n, x, z, e):
    letters = []
    for q in range(n):
        bx, bz = (x >> q) & 1, (z >> q) & 1
        if bx:
            letters.append((q, "X"))
    M = dense.pauli_matrix(n, letters)
    letters_z = [(q, "Z") for q in range(n) if (z >> q) & 1]
    Mz = dense.pauli_matrix(n, letters_z)
    return (1j ** e) * (M @ Mz)


def _gate_unitary(name, n, qa, qb):
    M = np.eye(2 ** n, dtype=complex)
    cols = []
    for j in range(2 ** n):
        if name in dense.GATE_1Q:
            cols.append(dense.apply_1q(M[:, j], n, dense.GATE_1Q[name], qa))
        else:
            cols.append(dense.apply_2q(M[:, j], n, dense.GATE_2Q[name], qa, qb))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("gate", ["H", "S", "S_DAG", "X", "Y", "Z", "CX", "CZ", "SWAP"])
def test_conjugation_exhaustive(gate):
    n = 2
    targets = [(0, 1), (1, 0)] if gate in dense.GATE_2Q else [(0, -1), (1, -1)]
    for qa, qb in targets:
        U = _gate_unitary(gate, n, qa, qb)
        for x in range(4):
            for z in range(4):
                for e in range(4):
                    P = _pauli_mat(n, x, z, e)
                    want = U @ P @ U.conj().T
                    x2, z2, e2 = oracle.conjugate(gate, qa, qb, x, z, e)
                    got = _pauli_mat(n, x2, z2, e2)
                    assert np.allclose(got, want), (gate, qa, qb, x, z, e)


@pytest.mark.parametrize("seed", range(6))
def test_tableau_matches_dense_projection(seed):
    rng = np.random.default_rng(100 + seed)
    kinds = np.zeros(4, int)
    for trial in range(40):
        n = int(rng.integers(2, 7))
        c = random_circuit(rng, n, int(rng.integers(5, 40)))
        oc = OracleCircuit(c)
        for shot in (0, 63, 64 + 5):
            tr = oc.trace(777 + trial, shot)
            rep = dense.replay(c, tr["fired"], tr["m"])  # raises if an outcome had zero probability
            assert np.allclose(rep["p0"], tr["p0"], atol=1e-12, rtol=0)
            kinds += np.bincount(tr["meas_kind"], minlength=4)
            # the records the tableau wrote are those it traced
            recs = oc.sample(777 + trial, 64 * 2)
            w, lane = shot // 64, shot % 64
            got = (recs[:, w] >> np.uint64(lane)) & np.uint64(1)
            want = dense.records_to_rows(c, rep["records"])
            assert np.array_equal(got.astype(np.uint8), want)
    assert kinds.min() > 0  # random, deterministic, active-diagonal and active-pair all exercised


def _p0_first_active(c, shots=(0,)):
    oc = OracleCircuit(c)
    tr = oc.trace(1, shots[0])
    return tr


def test_closed_form_promote_then_diag_measure():
    # R_X(theta)|0> then M_Z: Pr(0) = cos^2(theta/2)  (PromoteRot then ActiveDiagMeas)
    for th in (0.3, 1.1, 2.5):
        c = Circuit(1)
        c.rot([(0, "X")], th)
        c.append("M", [0])
        tr = _p0_first_active(c)
        assert tr["rot_kind"][0] == 1 and tr["meas_kind"][0] == 2
        assert abs(tr["p0"][0] - np.cos(th / 2) ** 2) < 1e-14


def test_closed_form_t_gate():
    # H R_Z(pi/4) H then M_Z: Pr(0) = cos^2(pi/8)
    c = Circuit(1)
    c.append("H", [0])
    c.rot([(0, "Z")], np.pi / 4)
    c.append("H", [0])
    c.append("M", [0])
    tr = _p0_first_active(c)
    assert abs(tr["p0"][0] - np.cos(np.pi / 8) ** 2) < 1e-14
    assert abs(tr["p0"][0] - 0.8535533905932737) < 1e-15


def test_closed_form_zz_rotation_then_x_measurement():
    # R_ZZ(theta)|++> then M_X1: Pr(0) = cos^2(theta/2); X1 lies in the stabilizer
    # coordinates' Z group after the promotion, so this is an active-diagonal measurement
    for th in (0.4, 1.3):
        c = Circuit(2)
        c.append("H", [0, 1])
        c.rot([(0, "Z"), (1, "Z")], th)
        c.mpp([(0, "X")])
        tr = _p0_first_active(c)
        assert tr["rot_kind"][1] == 1
        assert tr["meas_kind"][0] == 2
        assert abs(tr["p0"][0] - np.cos(th / 2) ** 2) < 1e-14


def test_closed_form_pair_measurement():
    # R_X(theta)|0> has Bloch vector (0, -sin theta, cos theta); M_Y: Pr(0) = (1 - sin theta)/2.
    # Y anticommutes with both coordinate generators: active-pair measurement with mu = +-i.
    for th in (0.4, 1.3, 2.9):
        c = Circuit(1)
        c.rot([(0, "X")], th)
        c.mpp([(0, "Y")])
        tr = _p0_first_active(c)
        assert tr["meas_kind"][0] == 3
        assert abs(tr["p0"][0] - (1 - np.sin(th)) / 2) < 1e-14


def test_closed_form_pair_rotation():
    # R_X(t1)|0> then R_Y(t2) (a rotation inside the active space) then M_Z:
    # Pr(0) = (1 + cos t1 cos t2)/2
    for t1, t2 in ((0.5, 0.8), (1.9, -0.6)):
        c = Circuit(1)
        c.rot([(0, "X")], t1)
        c.rot([(0, "Y")], t2)
        c.append("M", [0])
        tr = _p0_first_active(c)
        assert tr["rot_kind"][1] == 3
        assert abs(tr["p0"][0] - (1 + np.cos(t1) * np.cos(t2)) / 2) < 1e-14


def test_closed_form_pair_rotation_inverse():
    # R_P(theta) R_P(-theta) restores the state: Pr(M_Z = 0) = 1 after promoting with R_X
    c = Circuit(2)
    c.rot([(0, "X")], 0.7)
    c.rot([(0, "X"), (1, "Z")], 0.9)   # acts inside the active space
    c.rot([(0, "X"), (1, "Z")], -0.9)
    c.rot([(0, "X")], -0.7)
    c.append("M", [0])
    tr = _p0_first_active(c)
    assert abs(tr["p0"][0] - 1.0) < 1e-14


def test_random_and_deterministic_measurements():
    c = Circuit(1)
    c.mpp([(0, "X")])      # |0> measured in X: exactly 1/2, RandomMeas
    c.append("X", [0])
    c.append("H", [0])     # now the state is an X eigenstate again
    c.append("M", [0])
    oc = OracleCircuit(c)
    tr = oc.trace(3, 0)
    assert tr["meas_kind"][0] == 0 and tr["p0"][0] == 0.5
    # X then M_Z gives 1 deterministically (DetMeas with eta = 1)
    c2 = Circuit(1)
    c2.append("X", [0])
    c2.append("M", [0])
    out = OracleCircuit(c2).sample(5, 256)
    assert np.all(out[0] == np.uint64(0xFFFFFFFFFFFFFFFF))
    assert OracleCircuit(c2).trace(5, 0)["meas_kind"][0] == 1


def test_feedback_enters_sign():
    # M_X, Z^m feedback, M_X again: always 0
    c = Circuit(1)
    r = c.mpp([(0, "X")])
    c.feedback([(0, "Z")], [r])
    c.mpp([(0, "X")])
    out = OracleCircuit(c).sample(11, 64 * 16)
    assert np.count_nonzero(out[0]) > 0           # first outcome is random
    assert not np.any(out[1])                      # second is always 0


def _histogram(oc, seed, shots):
    out = oc.sample(seed, shots, threads=4)
    n_rec = oc.n_rec
    lanes = np.arange(64, dtype=np.uint64)
    bits = ((out[:n_rec, :, None] >> lanes[None, None, :]) & np.uint64(1)).reshape(n_rec, -1)[:, :shots]
    keys = {}
    for s in range(shots):
        k = tuple(int(v) for v in bits[:, s])
        keys[k] = keys.get(k, 0) + 1
    return keys


@pytest.mark.parametrize("seed", range(4))
def test_record_distribution_chi_square(seed):
    rng = np.random.default_rng(900 + seed)
    for _ in range(20):
        c = random_circuit(rng, int(rng.integers(2, 4)), int(rng.integers(6, 16)), p_noise=0.2)
        if 1 <= c.num_records <= 5:
            break
    exact = dense.exact_record_distribution(c)
    assert abs(sum(exact.values()) - 1) < 1e-9
    oc = OracleCircuit(c)
    shots = 64 * 160
    hist = _histogram(oc, 4242 + seed, shots)
    keys = sorted(set(exact) | set(hist))
    obs = np.array([hist.get(k, 0) for k in keys], dtype=float)
    exp = np.array([exact.get(k, 0.0) * shots for k in keys])
    assert obs[exp == 0].sum() == 0, "oracle produced a record tuple of probability zero"
    m = exp > 0
    # merge tiny bins
    small = exp[m] < 5
    o = np.append(obs[m][~small], obs[m][small].sum())
    e = np.append(exp[m][~small], exp[m][small].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    if len(e) > 1:
        chi2 = ((o - e) ** 2 / e).sum()
        pval = stats.chi2.sf(chi2, len(e) - 1)
        assert pval > 1e-4, (chi2, len(e), pval)


@pytest.mark.parametrize("d,r", [(3, 3), (5, 3)])
def test_noiseless_surface_detectors_zero(d, r):
    c = rotated_memory_z(d, r, 0.0)
    out = OracleCircuit(c).sample(99, 64 * 4)
    assert not np.any(out[c.num_records:])


def test_surface_counts_match_paper():
    # paper Sec. 7.2: d=7,r=7 has 97 qubits / 336 detectors, d=9,r=9 has 161 / 720
    for d, n, D in ((7, 97, 336), (9, 161, 720)):
        c = rotated_memory_z(d, d, 1e-3)
        assert c.n_qubits == n and c.num_detectors == D


def test_k_trajectory_is_shot_independent():
    from workloads import configs
    c = configs.c3(shots=64).circuit
    oc = OracleCircuit(c)
    a = oc.trace(1, 0)
    b = oc.trace(2, 12345)
    assert np.array_equal(a["k"], b["k"])
    assert np.array_equal(a["meas_kind"], b["meas_kind"])
    assert int(a["k"].max()) == 8


@pytest.mark.parametrize("seed", range(3))
def test_final_state_matches_dense_replay(seed):
    """The oracle's whole final state, psi = sum_x alpha_x Xbar^x |0bar> rebuilt
    from its signed tableau and active vector, against the dense replay of the
    same shot (noise branches and outcomes from the oracle's trace), up to a
    global phase."""
    rng = np.random.default_rng(7300 + seed)
    checked = 0
    for trial in range(25):
        n = int(rng.integers(2, 6))
        c = random_circuit(rng, n, int(rng.integers(5, 40)), p_flip=0.2 if trial % 2 else 0.0)
        oc = OracleCircuit(c)
        s = 500 + trial
        for shot in (3, 64 + 17):
            tr = oc.trace(s, shot)
            psi_d = dense.replay(c, tr["fired"], tr["m"])["state"]
            fs = oc.final_state(s, shot)
            zbar = [_pauli_mat(n, fs["x"][j], fs["z"][j], int(fs["e"][j])) for j in range(n)]
            xbar = [_pauli_mat(n, fs["x"][n + j], fs["z"][n + j], int(fs["e"][n + j])) for j in range(n)]
            v = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
            for Z in zbar:
                v = (v + Z @ v) / 2
            v /= np.linalg.norm(v)
            psi_o = np.zeros(2 ** n, dtype=complex)
            for x, a in enumerate(fs["alpha"]):
                w = v
                for j in range(fs["k"]):
                    if (x >> j) & 1:
                        w = xbar[j] @ w
                psi_o += a * w
            assert abs(np.linalg.norm(psi_o) - 1) < 1e-12
            assert abs(abs(np.vdot(psi_o, psi_d)) - 1) < 1e-10
            checked += fs["k"] > 0
    assert checked > 0


def test_oracle_rejects_registers_past_its_limit():
    # the oracle's per-shot Pauli scratch holds 64 words, so at most 4096 qubits
    c = Circuit(4097)
    c.append("H", [4096])
    with pytest.raises(ValueError):
        OracleCircuit(c)
    ok = Circuit(4096)
    ok.append("M", [4095])
    assert OracleCircuit(ok).sample(1, 64).shape[0] == 1
