"""GPU parity of the aggregate-count mode (paper Sec. 6: detector postselection,
per-shot discarded / logical-error flags summed into counters).

The expected flags come from the oracle's complete records (oracle.counts).
Pure-Clifford programs must match bit for bit.  On programs with a dense
active vector a shot's flags may differ from the oracle's only where its
records do, and those shots must be ones whose active-measurement draw lies
within the precision's tolerance of the threshold (the same rule as the
record parity tests).  Independently of the oracle, the flags must equal the
ones derived from the same kernels' full records: early termination of a
rejected shot may not change any kept shot.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_28600_amd as S  # noqa: E402
from oracle import OracleCircuit  # noqa: E402
from oracle.counts import count_flags  # noqa: E402
from tests.parity_util import compare_records  # noqa: E402
from workloads import configs  # noqa: E402
from workloads.surface import rotated_memory_z  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}


def _popcount(a):
    return int(sum(bin(int(x)).count("1") for x in np.asarray(a, dtype=np.uint64).reshape(-1)))


def _check(circ, prog, oc, shots, seed, post, exp=None, prec="fp64", shot_offset=0, mode=0):
    print(f"counts: k_max={prog.k_max} shots={shots} offset={shot_offset} prec={prec} post={len(post)} mode={mode}",
          flush=True)
    flags_t, counts_t = prog.sample_counts(shots, seed, post=post, obs_expected=exp, shot_offset=shot_offset,
                                           precision=prec, mode=mode)
    flags = S.bits_to_numpy(flags_t)
    counts = counts_t.cpu().numpy()
    nr, nd, no = circ.num_records, circ.num_detectors, circ.num_observables
    want_rows = oc.sample(seed, shots, shot_begin=shot_offset)
    want_f, want_c = count_flags(want_rows, nr, nd, no, shots, post, exp)
    # same kernels, full records
    rec = S.bits_to_numpy(prog.sample(shots, seed, shot_offset=shot_offset, precision=prec))
    own_f, _ = count_flags(rec, nr, nd, no, shots, post, exp)
    assert np.array_equal(flags, own_f)
    assert list(counts) == [_popcount(flags[0]), _popcount(flags[1])]
    if prog.k_max == 0:
        assert np.array_equal(flags, want_f)
        assert list(counts) == list(want_c)
        return flags, counts
    compare_records(rec, want_rows, circ, oc, seed, shot_offset, TOL[prec])
    rdiff = np.bitwise_or.reduce(rec ^ want_rows, axis=0)
    fdiff = np.bitwise_or.reduce(flags ^ want_f, axis=0)
    assert not np.any(fdiff & ~rdiff), "flags differ from the oracle in a shot whose records agree"
    return flags, counts


@pytest.fixture(scope="module")
def c1():
    w = configs.c1()
    return w, S.Program(w.circuit), OracleCircuit(w.circuit)


def test_counts_frame_c1_all_detectors(c1):
    w, p, oc = c1
    post = list(range(w.circuit.num_detectors))
    flags, counts = _check(w.circuit, p, oc, w.shots, w.seed, post)
    assert 0 < counts[0] < w.shots  # p = 1e-3 on 24 detectors discards some shots, not all


def test_counts_frame_c1_subset_expected_and_ragged(c1):
    w, p, oc = c1
    _check(w.circuit, p, oc, w.shots, w.seed, [0, 5, 17, 5], exp=[1])
    _check(w.circuit, p, oc, 1000, w.seed, [3, 4], shot_offset=64 * 37)
    _check(w.circuit, p, oc, 70, w.seed, [])


def test_counts_frame_c2_small():
    w = configs.c2()
    p = S.Program(w.circuit)
    oc = OracleCircuit(w.circuit)
    _check(w.circuit, p, oc, 64 * 20, w.seed, list(range(w.circuit.num_detectors)))


def test_counts_accumulate_over_shot_ranges(c1):
    w, p, _ = c1
    post = list(range(w.circuit.num_detectors))
    flags, counts = p.sample_counts(64 * 10, w.seed, post=post)
    acc = torch.zeros(2, dtype=torch.int64, device="cuda")
    f1 = torch.zeros((2, 4), dtype=torch.int64, device="cuda")
    f2 = torch.zeros((2, 6), dtype=torch.int64, device="cuda")
    p.sample_counts_into(f1, acc, 64 * 4, w.seed, post=post)
    p.sample_counts_into(f2, acc, 64 * 6, w.seed, post=post, shot_offset=64 * 4)
    assert torch.equal(torch.cat([f1, f2], dim=1), flags)
    assert torch.equal(acc, counts)
    before = acc.clone()
    p.sample_counts_into(None, acc, 0, w.seed, post=post)
    torch.cuda.synchronize()
    assert torch.equal(acc, before)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_counts_active_coherent_surface_d3(prec):
    """Coherent Z errors on the data of a d = 3 code (peak width 4); every detector postselected."""
    c = rotated_memory_z(3, 3, 1e-3, coherent=0.3)
    p = S.Program(c)
    assert p.k_max > 0
    oc = OracleCircuit(c)
    flags, counts = _check(c, p, oc, 64 * 32, 0x5EED0C03, list(range(c.num_detectors)), prec=prec)
    assert 0 < counts[0] < 64 * 32


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_counts_active_coherent_surface_d5(prec):
    """Peak width 12 (LDS vectors, many shot groups discarded at different instructions)."""
    c = rotated_memory_z(5, 3, 1e-3, coherent=0.1)
    p = S.Program(c)
    assert p.k_max == 12
    oc = OracleCircuit(c)
    _check(c, p, oc, 64 * 3 + 17, 0x5EED0C05, list(range(c.num_detectors)), exp=[1], prec=prec)


def test_counts_active_large_width_one_group_per_workgroup():
    """Peak width 14: one shot per workgroup, which leaves the stream at its rejection."""
    import copy
    w = configs.c5(14)
    c = copy.deepcopy(w.circuit)
    nr = c.num_records
    for r in (5, 40, 120):
        c.detector([r, r + 1])
    c.observable(0, [nr - 1])
    p = S.Program(c)
    assert p.k_max == 14
    oc = OracleCircuit(c)
    flags, counts = _check(c, p, oc, 64 * 2, w.seed, [0, 1, 2], prec="fp32")
    assert counts[0] > 0


def test_counts_random_small_circuits():
    from tests.randcirc import random_circuit
    rng = np.random.default_rng(77)
    done = 0
    for trial in range(40):
        c = random_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(20, 60)))
        if c.num_detectors == 0:
            continue
        p = S.Program(c)
        oc = OracleCircuit(c)
        for prec in ("fp64", "fp32"):
            _check(c, p, oc, 64 * 3, 4242 + trial, [0], exp=[int(rng.integers(2))], prec=prec)
        done += 1
    assert done >= 10


def test_counts_do_not_depend_on_threads_per_shot_and_autotune():
    c = rotated_memory_z(5, 3, 1e-3, coherent=0.1)
    p = S.Program(c)
    post = list(range(c.num_detectors))
    ref_f, ref_c = p.sample_counts(64 * 5 + 9, 0x5EED0C06, post=post, precision="fp32")
    for tps in (4, 16, 64, 128, 256):
        f, n = p.sample_counts(64 * 5 + 9, 0x5EED0C06, post=post, precision="fp32", threads_per_shot=tps)
        assert torch.equal(f, ref_f), tps
        assert torch.equal(n, ref_c), tps
    tps = p.autotune_counts(post, precision="fp32")
    assert tps in (1, 4, 8, 16, 32, 64, 128, 256)  # 1: the lane kernel
    f, n = p.sample_counts(64 * 5 + 9, 0x5EED0C06, post=post, precision="fp32")
    assert torch.equal(f, ref_f) and torch.equal(n, ref_c)


def test_counts_with_32_word_tiles_match_forced_16_word_records(c1):
    """2^20 shots of C1: the count launch takes 32-word tiles (at least two per CU), and its flags must
    equal those derived from records written with 16-word tiles (which the record tests pin to the
    oracle)."""
    w, p, oc = c1
    shots = 1 << 20
    post = list(range(0, w.circuit.num_detectors, 3))
    print("counts C1 2^20 shots, 32-word tiles", flush=True)
    flags_t, counts_t = p.sample_counts(shots, w.seed, post=post)
    rec = S.bits_to_numpy(p.sample(shots, w.seed, frame_tile_words=16))
    c = w.circuit
    want_f, want_c = count_flags(rec, c.num_records, c.num_detectors, c.num_observables, shots, post, None)
    assert np.array_equal(S.bits_to_numpy(flags_t), want_f)
    assert list(counts_t.cpu().numpy()) == list(want_c)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_counts_via_records_path(prec):
    """Count path 2 (rows written by the record kernel, then reduced) against the oracle, on a coherent-noise
    surface code and random circuits, with a ragged range at an offset; and the autotuner's choice keeps the
    flags."""
    from tests.randcirc import random_circuit
    c = rotated_memory_z(3, 3, 2e-3, coherent=0.15)
    p = S.Program(c)
    oc = OracleCircuit(c)
    post = list(range(c.num_detectors))
    _check(c, p, oc, 64 * 9 + 5, 31, post, prec=prec, shot_offset=64 * 3, mode=2)
    exp = [1] * c.num_observables
    _check(c, p, oc, 64 * 5, 32, post[::2], exp=exp, prec=prec, mode=2)
    rng = np.random.default_rng(77)
    for trial in range(6):
        rc = random_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(15, 50)))
        if rc.num_detectors == 0:
            continue
        rp = S.Program(rc)
        _check(rc, rp, OracleCircuit(rc), 64 * 3, 40 + trial, list(range(rc.num_detectors)), prec=prec, mode=2)
    p.autotune_counts(post, precision=prec)
    a, _ = p.sample_counts(64 * 7, 33, post=post, precision=prec)
    b, _ = p.sample_counts(64 * 7, 33, post=post, precision=prec, mode=1)
    assert np.array_equal(S.bits_to_numpy(a), S.bits_to_numpy(b))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_count_paths_agree_over_several_chunks(prec):
    """Count path 2 runs its range in chunks of 4096 words (bounded scratch for the detector and observable
    rows only): over three and a half chunks at an offset, paths 1 and 2 and the automatic choice give the
    same flags and counts, equal to those derived from the same kernels' full records."""
    from workloads.distill import distill_15to1
    c = distill_15to1(1e-2)
    p = S.Program(c)
    post = list(range(c.num_detectors))
    shots, off, seed = 3 * 4096 * 64 + 64 * 2048 + 37, 64 * 5, 4099
    print(f"count paths over {shots} shots, {prec}", flush=True)
    f1, c1 = p.sample_counts(shots, seed, post=post, shot_offset=off, precision=prec, mode=1)
    f2, c2 = p.sample_counts(shots, seed, post=post, shot_offset=off, precision=prec, mode=2)
    p.autotune_counts(post, precision=prec)
    f0, c0 = p.sample_counts(shots, seed, post=post, shot_offset=off, precision=prec, mode=0)
    a1, a2, a0 = S.bits_to_numpy(f1), S.bits_to_numpy(f2), S.bits_to_numpy(f0)
    assert np.array_equal(a1, a2) and np.array_equal(a1, a0)
    assert list(c1.cpu().numpy()) == list(c2.cpu().numpy()) == list(c0.cpu().numpy())
    rec = S.bits_to_numpy(p.sample(shots, seed, shot_offset=off, precision=prec))
    own, own_c = count_flags(rec, c.num_records, c.num_detectors, c.num_observables, shots, post, None)
    assert np.array_equal(a1, own)
    assert list(c1.cpu().numpy()) == list(own_c)


@pytest.mark.parametrize("prec,tps", [("fp32", 64), ("fp32", 256), ("fp64", 64), ("fp64", 256)])
def test_counts_sub_word_units(prec, tps):
    """One shot group per workgroup: the count launch splits each word into units of 4 shots (LDS vectors:
    one workgroup per unit; HBM vectors, as FP64 at width 12: resident workgroups take units from a
    counter).  On a flag buffer that starts as all ones, every unit must write exactly its shots' bits:
    the flags equal those derived from the same kernels' full records, padding bits included, over a
    ragged range at an offset."""
    w = configs.postselect()
    c = w.circuit
    p = S.Program(c)
    assert p.k_max == 12
    post = list(range(c.num_detectors))
    shots, off = 64 * 37 + 13, 64 * 11
    words = (shots + 63) // 64
    print(f"sub-word units: {prec} tps={tps}", flush=True)
    flags = torch.full((2, words), -1, dtype=torch.int64, device="cuda")
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    p.sample_counts_into(flags, counts, shots, w.seed, post=post, shot_offset=off, precision=prec, threads_per_shot=tps)
    rec = S.bits_to_numpy(p.sample(shots, w.seed, shot_offset=off, precision=prec))
    own_f, _ = count_flags(rec, c.num_records, c.num_detectors, c.num_observables, shots, post, None)
    got = S.bits_to_numpy(flags)
    assert np.array_equal(got, own_f)
    assert list(counts.cpu().numpy()) == [_popcount(own_f[0]), _popcount(own_f[1])]
    assert 0 < _popcount(own_f[0]) < shots
