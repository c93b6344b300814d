"""Readout flips (paper Sec. 6: readout flips are exogenous symbols, sampled like
Pauli noise choices) on the CPU.

A recorded measurement with flip probability p reports the complement of its
outcome with probability p and leaves the state of the true outcome.

* Closed forms at p = 1 (the flip always fires): the reported bit is the
  complement and the state is untouched, or reset on the true outcome.
* Flip frequency at p = 1/4 on a deterministic outcome, against a binomial bound.
* Every Pr(m = 0) and record of the oracle against the dense brute force, which
  applies the plain definition (projection on the true outcome, then the
  complement recorded).
* Exact record distributions (outcome tree with the flip branch) vs oracle
  histograms.
* The compiled program (sign expressions with the flip symbols), replayed on
  the CPU with the oracle's draws, against the oracle's records.
* Argument checks of the compiler.
"""
import numpy as np
import pytest
from scipy import stats

import paper_2607_28600_amd as S
from oracle import OracleCircuit, dense
from tests.program_replay import replay_shot, rows_from_measurements
from tests.randcirc import random_circuit
from tests.test_oracle_pins import _histogram
from workloads.circuit import Circuit
from workloads.surface import rotated_memory_z

ALL = np.uint64(0xFFFFFFFFFFFFFFFF)


def test_flip_at_one_complements_and_leaves_the_state():
    c = Circuit(1)
    c.append("M", [0], arg=1.0)   # |0>: reports 1
    c.append("M", [0])            # the state is still |0>
    out = OracleCircuit(c).sample(11, 256)
    assert np.all(out[0] == ALL) and not np.any(out[1])


def test_flipped_reset_acts_on_the_true_outcome():
    c = Circuit(1)
    c.append("X", [0])
    c.append("MR", [0], arg=1.0)  # true 1, reports 0, resets to |0>
    c.append("M", [0])
    out = OracleCircuit(c).sample(12, 256)
    assert not np.any(out[0]) and not np.any(out[1])


def test_flipped_pauli_product_measurement():
    c = Circuit(2)
    c.append("H", [0])
    c.append("CX", [0, 1])        # Bell state: XX = +1
    c.mpp([(0, "X"), (1, "X")], p_flip=1.0)
    c.mpp([(0, "X"), (1, "X")])
    c.mpp([(0, "Z"), (1, "Z")], p_flip=1.0)
    out = OracleCircuit(c).sample(13, 256)
    assert np.all(out[0] == ALL) and not np.any(out[1]) and np.all(out[2] == ALL)


def test_flip_frequency():
    c = Circuit(1)
    c.append("M", [0], arg=0.25)
    shots = 64 * 512
    out = OracleCircuit(c).sample(14, shots)
    k = int(sum(bin(int(v)).count("1") for v in out[0]))
    # two-sided binomial test; the flip fires with probability floor(2^32 p) / 2^32 = 1/4 exactly
    assert stats.binomtest(k, shots, 0.25).pvalue > 1e-4


@pytest.mark.parametrize("seed", range(4))
def test_oracle_matches_dense_projection_with_flips(seed):
    rng = np.random.default_rng(5100 + seed)
    flips = 0
    for trial in range(30):
        n = int(rng.integers(2, 7))
        c = random_circuit(rng, n, int(rng.integers(5, 40)), p_flip=0.35)
        oc = OracleCircuit(c)
        s = 900 + trial
        recs = oc.sample(s, 64 * 2)
        for shot in (0, 63, 64 + 5):
            tr = oc.trace(s, shot)
            rep = dense.replay(c, tr["fired"], tr["m"])
            assert np.allclose(rep["p0"], tr["p0"], atol=1e-12, rtol=0)
            got = (recs[:, shot // 64] >> np.uint64(shot % 64)) & np.uint64(1)
            assert np.array_equal(got.astype(np.uint8), dense.records_to_rows(c, rep["records"]))
            flips += int(np.sum(tr["fired"] >= 0))
    assert flips > 0


@pytest.mark.parametrize("seed", range(3))
def test_record_distribution_with_flips(seed):
    rng = np.random.default_rng(5200 + seed)
    for _ in range(40):
        c = random_circuit(rng, int(rng.integers(2, 4)), int(rng.integers(6, 16)), p_noise=0.15, p_flip=0.2)
        if 1 <= c.num_records <= 5:
            break
    exact = dense.exact_record_distribution(c)
    assert abs(sum(exact.values()) - 1) < 1e-9
    shots = 64 * 160
    hist = _histogram(OracleCircuit(c), 5300 + seed, shots)
    keys = sorted(set(exact) | set(hist))
    obs = np.array([hist.get(k, 0) for k in keys], dtype=float)
    exp = np.array([exact.get(k, 0.0) * shots for k in keys])
    assert obs[exp == 0].sum() == 0
    m = exp > 0
    small = exp[m] < 5
    o = np.append(obs[m][~small], obs[m][small].sum())
    e = np.append(exp[m][~small], exp[m][small].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    if len(e) > 1:
        chi2 = ((o - e) ** 2 / e).sum()
        assert stats.chi2.sf(chi2, len(e) - 1) > 1e-4


@pytest.mark.parametrize("seed", range(3))
def test_compiled_program_replay_with_flips(seed):
    rng = np.random.default_rng(5400 + seed)
    for trial in range(30):
        c = random_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(5, 45)), p_flip=0.3)
        exp = S.Program(c).export()
        oc = OracleCircuit(c)
        s = 6000 + trial
        out = oc.sample(s, 128)
        for shot in (2, 70, 127):
            tr = oc.trace(s, shot)
            mv, p0 = replay_shot(exp, c, s, shot, tr["fired"])
            want = ((out[:, shot // 64] >> np.uint64(shot % 64)) & np.uint64(1)).astype(np.uint8)
            assert np.array_equal(rows_from_measurements(c, mv), want)
            act = tr["meas_kind"] >= 2
            assert np.allclose(p0[act], tr["p0"][act], atol=1e-12, rtol=0)


def test_surface_flips_leave_noiseless_detectors_at_the_flip_rate():
    # only readout flips: a detector of round 1 (one Z check) fires iff that record flipped
    c = rotated_memory_z(3, 2, 0.0, p_meas=0.5)
    base = S.Program(rotated_memory_z(3, 2, 0.0)).info()["n_channels"]
    assert S.Program(c).info()["n_channels"] == base + c.num_records
    oc = OracleCircuit(c)
    out = oc.sample(21, 64 * 64)
    n_rec = c.num_records
    frac = np.mean([bin(int(v)).count("1") / 64 for v in out[n_rec]])
    assert abs(frac - 0.5) < 0.05


def _code(c):
    with pytest.raises(S.SymftError) as ei:
        S.Program(c)
    return ei.value.code


def test_flip_argument_checks():
    c = Circuit(1)
    c.append("M", [0], arg=1.5)
    assert _code(c) == -4
    c = Circuit(1)
    c.append("MR", [0], arg=-0.1)
    assert _code(c) == -4
    c = Circuit(1)
    c.mpp([(0, "X")], p_flip=2.0)
    assert _code(c) == -4
    c = Circuit(1)
    c.append("R", [0], arg=0.1)
    assert _code(c) == -1
    # p = 0 adds no channel; p > 0 one per record
    c = Circuit(2)
    c.append("M", [0, 1])
    assert S.Program(c).info()["n_channels"] == 0
    c = Circuit(2)
    c.append("M", [0, 1], arg=0.1)
    c.mpp([(0, "X")], p_flip=0.1)
    assert S.Program(c).info()["n_channels"] == 3
