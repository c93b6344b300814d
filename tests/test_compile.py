"""Host-side checks of the GPU library (no GPU needed).

* the library loads and exports every function declared in include/symft.h;
* the compiled plan (instruction kinds, active-width trajectory) equals the
  oracle's classification, which is basis-independent (paper Sec. 4);
* an FP64 replay of the exported instruction stream, fed with the oracle's
  draws, reproduces the oracle's records and branch probabilities: this pins
  the host compiler's pulled-back Paulis, pivots, mu, eta and sign expressions;
* error paths: malformed ops, acausal records, bad probabilities, bad options.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2607_28600_amd as S
from oracle import OracleCircuit
from tests.program_replay import replay_shot, rows_from_measurements
from tests.randcirc import random_circuit
from workloads import configs
from workloads.circuit import Circuit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "symft.h")).read()
    declared = set(re.findall(r"\b(symft_[a-z_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    lib = C.CDLL(S.LIB)
    for name in sorted(declared):
        assert hasattr(lib, name), f"{name} declared in symft.h but not exported"
    assert set(S.EXPORTED) == declared


@pytest.mark.parametrize("seed", range(4))
def test_plan_matches_oracle_random(seed):
    rng = np.random.default_rng(50 + seed)
    for _ in range(40):
        c = random_circuit(rng, int(rng.integers(2, 8)), int(rng.integers(5, 50)))
        pl = S.Program(c).plan()
        tr = OracleCircuit(c).trace(0, 0)
        assert np.array_equal(pl["k"], tr["k"])
        assert np.array_equal(pl["meas_kind"], tr["meas_kind"])
        assert np.array_equal(pl["rot_kind"], tr["rot_kind"])


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5_14", "c5_16"])
def test_plan_matches_oracle_configs(name):
    w = {"c1": configs.c1, "c2": lambda: configs.c2(64), "c3": lambda: configs.c3(64),
         "c5_14": lambda: configs.c5(14, 64), "c5_16": lambda: configs.c5(16, 64)}[name]()
    p = S.Program(w.circuit)
    pl = p.plan()
    tr = OracleCircuit(w.circuit).trace(0, 0)
    assert np.array_equal(pl["k"], tr["k"])
    assert np.array_equal(pl["meas_kind"], tr["meas_kind"])
    want_k = {"c1": 0, "c2": 0, "c3": 8, "c5_14": 14, "c5_16": 16}[name]
    assert p.k_max == want_k


def test_c4_peak_widths():
    ks = []
    for i, w in enumerate(configs.c4()[:24]):
        ks.append(S.Program(w.circuit).k_max)
    assert ks[:12] == list(range(1, 13)) and ks[12:24] == list(range(1, 13))


@pytest.mark.parametrize("seed", range(3))
def test_replay_of_compiled_program_matches_oracle(seed):
    rng = np.random.default_rng(700 + seed)
    for trial in range(40):
        c = random_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(5, 45)))
        exp = S.Program(c).export()
        oc = OracleCircuit(c)
        s = 4000 + trial
        out = oc.sample(s, 128)
        for shot in (1, 66, 127):
            tr = oc.trace(s, shot)
            mv, p0 = replay_shot(exp, c, s, shot, tr["fired"])
            want = ((out[:, shot // 64] >> np.uint64(shot % 64)) & np.uint64(1)).astype(np.uint8)
            assert np.array_equal(rows_from_measurements(c, mv), want)
            act = tr["meas_kind"] >= 2
            assert np.allclose(p0[act], tr["p0"][act], atol=1e-12, rtol=0)


def test_replay_near_clifford_config():
    w = configs.c3(shots=64)
    exp = S.Program(w.circuit).export()
    oc = OracleCircuit(w.circuit)
    out = oc.sample(w.seed, 64)
    for shot in (0, 9, 41):
        tr = oc.trace(w.seed, shot)
        mv, p0 = replay_shot(exp, w.circuit, w.seed, shot, tr["fired"])
        want = ((out[:, 0] >> np.uint64(shot)) & np.uint64(1)).astype(np.uint8)
        assert np.array_equal(rows_from_measurements(w.circuit, mv), want)


def _err(c):
    with pytest.raises(S.SymftError) as ei:
        S.Program(c)
    return ei.value.code


def test_error_paths():
    c = Circuit(2)
    c.append("H", [5])
    assert _err(c) == -1  # qubit out of range
    c = Circuit(2)
    c.append("CX", [0, 0])
    assert _err(c) == -1
    c = Circuit(2)
    c.append("DEPOLARIZE1", [0], arg=1.5)
    assert _err(c) == -4
    c = Circuit(2)
    c.append("M", [0])
    c.ops.append(c.ops[0].__class__("DETECTOR", recs=(3,)))
    assert _err(c) == -3  # record not yet measured
    c = Circuit(2)
    c.rot([(0, "X"), (0, "Z")], 0.3)
    assert _err(c) == -1  # repeated qubit in a Pauli
    from workloads.circuit import Op
    c = Circuit(2)
    c.ops.append(Op("PAULI_CHANNEL", (0, 1), branches=((0.7, "XX"), (0.6, "ZI"))))
    assert _err(c) == -4


def test_sample_rejects_bad_offset_before_touching_the_gpu():
    p = S.Program(configs.c1().circuit)
    o = S.symft_sample_opts(shot_offset=10)
    rc = S._lib.symft_sample_ex(p.handle, C.byref(o), 64, 1, C.c_void_p(8), None)
    assert rc == -1
    o = S.symft_sample_opts(precision=3)
    assert S._lib.symft_sample_ex(p.handle, C.byref(o), 64, 1, C.c_void_p(8), None) == -1
    o = S.symft_sample_opts()
    assert S._lib.symft_sample_ex(p.handle, C.byref(o), 64, 1, None, None) == -1
    assert S._lib.symft_sample_ex(p.handle, C.byref(o), 0, 1, None, None) == 0  # no-op


def _fold_chain_circuit(n=6, p=0.1):
    """A GHZ-style chain: Z_0 is random, every later Z_i is determined by the one just before it, and the
    detectors compare neighbours.  No noise sits between the measurements."""
    c = Circuit(n)
    c.append("H", [0])
    c.append("CX", [q for i in range(n - 1) for q in (i, i + 1)])
    c.append("X_ERROR", list(range(n)), arg=p)
    c.append("M", list(range(n)))
    for i in range(n - 1):
        c.detector([i, i + 1])
    c.observable(0, [n - 1])
    return c


def test_frame_schedule_folds_same_level_dependencies():
    """The chain's records and detectors each depend on nodes of their own level; folding those
    dependencies (one RandomMeas word per node at most) puts all of them in one EMIT step after the
    NOISE step, instead of a step per link."""
    info = S.Program(_fold_chain_circuit()).info()
    assert info["k_max"] == 0
    assert info["frame_noise_steps"] == 1
    assert info["frame_steps"] == 2


def test_small_frame_calls_report_the_wave_owned_kernel():
    """The automatic pure-frame choice: small calls (up to 4,096 words) of schedules of at most 512 rows take
    the wave-owned kernel; larger schedules and active programs report no such range."""
    from workloads.surface import rotated_memory_z
    for c, small in ((configs.c1().circuit, 4096), (rotated_memory_z(5, 5, 1e-3), 4096),
                     (rotated_memory_z(7, 7, 1e-3), 0), (configs.c2().circuit, 0), (configs.c3().circuit, 0)):
        i = S.Program(c).info()
        assert i["frame_small_words"] == small, (i["n_rows"], i["frame_small_words"])
        if small:
            assert i["n_rows"] <= 512 and i["frame_kernel"] == 2


def test_frame_relation_accepts_frame_maps_and_rejects_other_states():
    from tests.parity_util import frame_relation
    rng = np.random.default_rng(3)
    b = rng.normal(size=16) + 1j * rng.normal(size=16)
    b /= np.linalg.norm(b)
    y, s, ph = 0b0110, 0b1010, np.exp(0.7j)
    chi = np.array([(-1) ** (bin(s & x).count("1") & 1) for x in range(16)])
    a = ph * chi * b[np.arange(16) ^ y]
    assert frame_relation(a, b, 1e-12) is not None
    bad = a.copy()
    bad[3] *= -1                                   # one sign off the character
    assert frame_relation(bad, b, 1e-9) is None
    bad = a.copy()
    bad[[1, 2]] = bad[[2, 1]]                      # two amplitudes exchanged
    assert frame_relation(bad, b, 1e-9) is None
    assert frame_relation(a * np.exp(1j * 0.3 * (np.arange(16) == 5)), b, 1e-9) is None  # a relative phase


@pytest.mark.parametrize("seed", range(2))
def test_replay_final_vector_matches_oracle_up_to_frame(seed):
    """The planner-basis active vector at the end of a shot (the vector the
    kernels hold) against the oracle's, which carries concrete signs instead of
    a symbolic frame: equal up to the frame's index shift, sign character and
    global phase."""
    from tests.parity_util import frame_relation
    rng = np.random.default_rng(7700 + seed)
    nonzero = 0
    for trial in range(40):
        c = random_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(5, 45)))
        exp = S.Program(c).export()
        oc = OracleCircuit(c)
        s = 800 + trial
        for shot in (5, 70):
            tr = oc.trace(s, shot)
            _, _, a = replay_shot(exp, c, s, shot, tr["fired"], return_state=True)
            fs = oc.final_state(s, shot)
            assert frame_relation(a, fs["alpha"], 1e-9) is not None
            nonzero += fs["k"] > 0
    assert nonzero > 20
