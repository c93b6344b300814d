"""GPU parity: records from the HIP kernels (through the C ABI) vs the CPU oracle.

Pure-Clifford circuits must match bit for bit.  Near-Clifford circuits must
match except shots with an active-measurement draw within 1e-5 (FP32) or
1e-9 (FP64) of its branch threshold; branch probabilities from the kernels
must agree with the oracle within 1e-5 (FP32) / 1e-12 (FP64).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
import paper_2607_28600_amd as S  # noqa: E402
from oracle import OracleCircuit  # noqa: E402
from tests.parity_util import compare_records, frame_relation  # noqa: E402
from tests.randcirc import random_circuit, wide_circuit  # noqa: E402
from workloads import configs  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}
P0_TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _gpu(prog, shots, seed, **kw):
    return S.bits_to_numpy(prog.sample(shots, seed, **kw))


@pytest.fixture(scope="module")
def c1():
    w = configs.c1()
    return w, S.Program(w.circuit), OracleCircuit(w.circuit)


@pytest.fixture(scope="module")
def c2():
    w = configs.c2()
    return w, S.Program(w.circuit), OracleCircuit(w.circuit)


@pytest.fixture(scope="module", params=["auto", "off"])
def c3(request):
    """C3 with the automatic representation (product components: its active state is nearly separable) and
    with the dense vector."""
    w = configs.c3()
    return w, S.Program(w.circuit, components=request.param), OracleCircuit(w.circuit)


def test_c1_full_bit_exact(c1):
    w, p, oc = c1
    got = _gpu(p, w.shots, w.seed)
    want = oc.sample(w.seed, w.shots)
    assert np.array_equal(got, want)


def test_c2_small_bit_exact(c2):
    w, p, oc = c2
    got = _gpu(p, 64 * 20, w.seed)          # two tiles, the second partial
    want = oc.sample(w.seed, 64 * 20, threads=0)
    assert np.array_equal(got, want)


def test_c2_ragged_offset_and_split(c2):
    w, p, oc = c2
    shots, off = 1000, 64 * 37
    got = _gpu(p, shots, w.seed, shot_offset=off)
    want = oc.sample(w.seed, shots, shot_begin=off)
    assert np.array_equal(got, want)
    # padding bits of the last word are zero
    assert not np.any(got[:, -1] >> np.uint64(shots % 64))
    full = _gpu(p, 64 * 8, w.seed)
    a = _gpu(p, 64 * 3, w.seed)
    b = _gpu(p, 64 * 5, w.seed, shot_offset=64 * 3)
    assert np.array_equal(full, np.concatenate([a, b], axis=1))


def test_c2_full_size_sampled_words(c2):
    """2^24 shots in the benchmark's launch configuration; words spread over the range."""
    w, p, oc = c2
    out = p.sample(w.shots, w.seed)
    words = [0, 1, 4095, 65536, 131071, 200003, 262143]
    got = S.bits_to_numpy(out[:, words])
    del out
    want = oc.sample_words(w.seed, words)
    assert np.array_equal(got, want)


def test_frame_deterministic(c1):
    w, p, _ = c1
    a = _gpu(p, 64 * 64, w.seed)
    b = _gpu(p, 64 * 64, w.seed)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_records(c3, prec):
    w, p, oc = c3
    n = 64 * 48
    got = _gpu(p, n, w.seed, precision=prec)
    want = oc.sample(w.seed, n)
    excluded = compare_records(got, want, w.circuit, oc, w.seed, 0, TOL[prec])
    assert excluded <= max(3, n // 200)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_branch_probabilities(c3, prec):
    w, p, oc = c3
    shots = list(range(64 * 7, 64 * 7 + 24))
    p0 = p.probe(shots[0], len(shots), w.seed, precision=prec)
    worst = 0.0
    for i, s in enumerate(shots):
        tr = oc.trace(w.seed, s)
        act = tr["meas_kind"] >= 2
        # compare only up to the first draw that could flip between the two precisions
        ts = np.flatnonzero(act)
        for t in ts:
            worst = max(worst, abs(p0[i, t] - tr["p0"][t]))
            if abs(O.active_u(w.seed, int(t), s) - tr["p0"][t]) < TOL[prec]:
                break
    assert worst < P0_TOL[prec], worst


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_full_size_sampled_words(c3, prec):
    w, p, oc = c3
    out = p.sample(w.shots, w.seed, precision=prec)
    words = [0, 777, 8191, 16383]
    got = S.bits_to_numpy(out[:, words])
    del out
    want = oc.sample_words(w.seed, words)
    for j, wd in enumerate(words):
        compare_records(got[:, j:j + 1], want[:, j:j + 1], w.circuit, oc, w.seed, 64 * wd, TOL[prec])


@pytest.mark.parametrize("comp", ["auto", "off"])
@pytest.mark.parametrize("i", [0, 3, 7, 10, 11, 23, 59, 127])
def test_c4_programs(i, comp):
    w = configs.c4()[i]
    p = S.Program(w.circuit, components=comp)
    oc = OracleCircuit(w.circuit)
    n = 64 * 8
    for prec in ("fp64", "fp32"):
        got = _gpu(p, n, w.seed, precision=prec)
        want = oc.sample(w.seed, n)
        compare_records(got, want, w.circuit, oc, w.seed, 0, TOL[prec])


@pytest.mark.parametrize("comp", ["auto", "off"])
@pytest.mark.parametrize("k,prec", [(14, "fp32"), (14, "fp64"), (16, "fp32"), (16, "fp64")])
def test_c5_large_active_state(k, prec, comp):
    w = configs.c5(k)
    p = S.Program(w.circuit, components=comp)
    assert p.k_max == k
    oc = OracleCircuit(w.circuit)
    n = 64 * 2
    got = _gpu(p, n, w.seed, precision=prec)
    want = oc.sample(w.seed, n)
    compare_records(got, want, w.circuit, oc, w.seed, 0, TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_widest_state_records(prec):
    """Maximum size: a peak active width of 20 (2^20 amplitudes per shot, HBM-resident, 1024 threads per
    shot; the dense vector), 64 shots against the oracle."""
    c = wide_circuit(18, 7)
    p = S.Program(c, components="off")
    assert p.k_max == 20
    oc = OracleCircuit(c)
    seed = 4242
    print(f"widest state k_max={p.k_max} {prec}", flush=True)
    got = _gpu(p, 64, seed, precision=prec)
    compare_records(got, oc.sample(seed, 64), c, oc, seed, 0, TOL[prec])


def test_random_small_circuits():
    rng = np.random.default_rng(2024)
    for trial in range(25):
        c = random_circuit(rng, int(rng.integers(2, 8)), int(rng.integers(10, 60)))
        oc = OracleCircuit(c)
        seed = 31337 + trial
        want = oc.sample(seed, 64 * 3)
        for comp in ("auto", "off"):
            p = S.Program(c, components=comp)
            for prec in ("fp64", "fp32"):
                got = _gpu(p, 64 * 3, seed, precision=prec)
                compare_records(got, want, c, oc, seed, 0, TOL[prec])


def test_zero_shots_is_noop(c1):
    w, p, _ = c1
    out = torch.full((p.n_rows, 4), 7, dtype=torch.int64, device="cuda")
    p.sample_into(out, 0, w.seed)
    torch.cuda.synchronize()
    assert int((out != 7).sum()) == 0


def test_sections_only_detectors(c1):
    w, p, oc = c1
    out = torch.zeros((p.n_rows, 16), dtype=torch.int64, device="cuda")
    p.sample_into(out, 1024, w.seed, sections=2)
    got = S.bits_to_numpy(out)
    want = oc.sample(w.seed, 1024)
    n_rec = w.circuit.num_records
    n_det = w.circuit.num_detectors
    assert not np.any(got[:n_rec]) and not np.any(got[n_rec + n_det:])
    assert np.array_equal(got[n_rec:n_rec + n_det], want[n_rec:n_rec + n_det])


def test_batch_graph_replays_match_single_launches_and_oracle():
    ws = configs.c4()[:24]
    progs = [S.Program(w.circuit) for w in ws]
    shots = [64 * (3 + i % 5) + (i * 7) % 64 for i in range(len(ws))]  # ragged last words
    seeds = [w.seed for w in ws]
    outs = [torch.zeros((p.n_rows, (s + 63) // 64), dtype=torch.int64, device="cuda") for p, s in zip(progs, shots)]
    first = None
    for rep in range(3):
        for o in outs:
            o.fill_(-1)                      # eager work between replays
        torch.cuda.synchronize()
        S.sample_batch(progs, shots, seeds, outs, precision="fp32", graph=True)
        torch.cuda.synchronize()
        got = [S.bits_to_numpy(o) for o in outs]
        if first is None:
            first = got
        for a, b in zip(first, got):
            assert np.array_equal(a, b), "graph replay differs"
    for i, (p, s, sd) in enumerate(zip(progs, shots, seeds)):
        single = _gpu(p, s, sd, precision="fp32")
        assert np.array_equal(single, first[i]), f"program {i}: batch differs from its own launch"
        if i % 4 == 0:
            oc = OracleCircuit(ws[i].circuit)
            compare_records(first[i], oc.sample(sd, s), ws[i].circuit, oc, sd, 0, TOL["fp32"])


def test_batch_without_graph_and_fp64():
    ws = configs.c4()[24:40]
    progs = [S.Program(w.circuit) for w in ws]
    shots = [256 + 64 * (i % 3) for i in range(len(ws))]
    seeds = [w.seed for w in ws]
    outs = [torch.zeros((p.n_rows, (s + 63) // 64), dtype=torch.int64, device="cuda") for p, s in zip(progs, shots)]
    S.sample_batch(progs, shots, seeds, outs, precision="fp64", graph=False)
    torch.cuda.synchronize()
    for i in (0, 5, 11):
        oc = OracleCircuit(ws[i].circuit)
        compare_records(S.bits_to_numpy(outs[i]), oc.sample(seeds[i], shots[i]), ws[i].circuit, oc, seeds[i], 0,
                        TOL["fp64"])


def test_autotune_choice_keeps_records():
    w = configs.c3(shots=64 * 16)
    p = S.Program(w.circuit)
    oc = OracleCircuit(w.circuit)
    tps = p.autotune("fp32")
    assert tps in (1, 4, 8, 16, 32, 64, 128, 256)  # 1: the lane kernel
    got = _gpu(p, w.shots, w.seed, precision="fp32")
    compare_records(got, oc.sample(w.seed, w.shots), w.circuit, oc, w.seed, 0, TOL["fp32"])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_autotuned_width_12_records(prec):
    """A width-12 program after the autotuner, which at widths 9..12 also times narrow groups with vectors
    in HBM scratch: records equal the oracle's outside the threshold exclusion, whichever it keeps."""
    w = configs.postselect()
    p = S.Program(w.circuit)
    assert p.k_max == 12
    tps = p.autotune(prec)
    print(f"width-12 autotune {prec}: {tps} threads per shot", flush=True)
    assert tps in (4, 8, 16, 32, 64, 128, 256)
    oc = OracleCircuit(w.circuit)
    n, off = 64 * 3 + 11, 64 * 40
    got = _gpu(p, n, w.seed, shot_offset=off, precision=prec)
    compare_records(got, oc.sample(w.seed, n, shot_begin=off), w.circuit, oc, w.seed, off, TOL[prec])


def _multiclass_surface(d, rounds, k):
    """Surface-code memory whose channels carry k different probabilities (k classes, interleaved
    along the circuit), and one non-uniform general channel."""
    import dataclasses
    from workloads.surface import rotated_memory_z
    c = rotated_memory_z(d, rounds, 1e-3)
    ops, swapped = [], False
    for op in c.ops:
        if op.name in ("X_ERROR", "DEPOLARIZE1", "DEPOLARIZE2"):
            if op.name == "DEPOLARIZE1" and not swapped:
                for q in op.targets:
                    ops.append(dataclasses.replace(op, name="PAULI_CHANNEL", targets=(q,), arg=0.0,
                                                   branches=((0.002, "X"), (0.0005, "Y"), (0.001, "Z"))))
                swapped = True
                continue
            width = 2 if op.name == "DEPOLARIZE2" else 1
            for i in range(0, len(op.targets), width):
                t = op.targets[i:i + width]
                ops.append(dataclasses.replace(op, targets=t, arg=op.arg * (1.0 + (t[0] % k) / 10.0)))
        else:
            ops.append(op)
    c.ops = ops
    return c


@pytest.mark.parametrize("tw", [0, 32])
@pytest.mark.parametrize("k", [3, 12])
@pytest.mark.parametrize("cap", [0, 8])
def test_frame_multiclass_bit_exact(k, cap, tw):
    """cap = 8 flip entries per (word, class) sends nearly every word down the fallback that
    draws its events again at every NOISE step."""
    c = _multiclass_surface(5, 4, k)
    p = S.Program(c)
    info = p.info()
    assert info["k_max"] == 0 and info["n_classes"] >= k
    oc = OracleCircuit(c)
    seed = 0xC1A55 + k
    n = 64 * 40 + 17
    assert np.array_equal(_gpu(p, n, seed, frame_entry_cap=cap, frame_tile_words=tw), oc.sample(seed, n))
    off = 64 * 21
    assert np.array_equal(_gpu(p, 700, seed, shot_offset=off, frame_entry_cap=cap, frame_tile_words=tw),
                          oc.sample(seed, 700, shot_begin=off))


@pytest.mark.parametrize("tw", [16, 32])
def test_frame_tile_widths_bit_exact(c1, c2, tw):
    """Both tile widths forced: C1 in full (256 words) and ragged at an offset, C2 over 40 words (a
    32-word tile and a partial one)."""
    w, p, oc = c1
    print(f"C1 tile width {tw}", flush=True)
    assert np.array_equal(_gpu(p, w.shots, w.seed, frame_tile_words=tw), oc.sample(w.seed, w.shots))
    assert np.array_equal(_gpu(p, 1000, w.seed, shot_offset=64 * 37, frame_tile_words=tw),
                          oc.sample(w.seed, 1000, shot_begin=64 * 37))
    w, p, oc = c2
    print(f"C2 tile width {tw}", flush=True)
    assert np.array_equal(_gpu(p, 64 * 40, w.seed, frame_tile_words=tw), oc.sample(w.seed, 64 * 40))


def test_frame_tile_width_falls_back_to_16_words():
    """A schedule whose slots fit LDS at 16 words per tile but not at 32: the automatic choice takes 16,
    and forcing 32 is a capacity error, raised before any launch."""
    from workloads.surface import rotated_memory_z
    c = rotated_memory_z(13, 3, 1e-3)
    p = S.Program(c)
    oc = OracleCircuit(c)
    print("d13 r3: automatic tile width", flush=True)
    assert np.array_equal(_gpu(p, 64 * 600, 5), _gpu(p, 64 * 600, 5, frame_tile_words=16))
    assert np.array_equal(_gpu(p, 64 * 4, 5), oc.sample(5, 64 * 4))
    with pytest.raises(S.SymftError) as ei:
        _gpu(p, 64 * 600, 5, frame_tile_words=32)
    assert ei.value.code == -5
    with pytest.raises(S.SymftError):
        _gpu(p, 64, 5, frame_tile_words=24)


def test_c2_entry_fallback_bit_exact(c2):
    w, p, oc = c2
    want = oc.sample(w.seed, 64 * 24, threads=0)
    for cap in (64, 1100, 1180):  # every word, most words, some words fall back (mean about 1140)
        assert np.array_equal(_gpu(p, 64 * 24, w.seed, frame_entry_cap=cap), want), cap


def test_frame_folded_chain_bit_exact():
    """Records and detectors of a chain folded into one EMIT level (each determined by the record just
    before it, starting from a random outcome) equal the oracle's bit for bit."""
    from tests.test_compile import _fold_chain_circuit
    c = _fold_chain_circuit()
    p = S.Program(c)
    assert p.info()["frame_steps"] == 2
    oc = OracleCircuit(c)
    for n, off in ((64 * 9 + 5, 0), (64 * 40, 64 * 13)):
        assert np.array_equal(_gpu(p, n, 0xF01D, shot_offset=off), oc.sample(0xF01D, n, shot_begin=off))


@pytest.mark.parametrize("p32", [1, 4295, 429497, 4294967, 85899346, 1288490189, 2147483648, 4294967295, 4294967296])
def test_gap_decision_at_table_boundaries(p32):
    Q = O.gap_table(p32).astype(np.int64)
    rng = np.random.default_rng(p32 % 1000003)
    q = Q[1:]
    cand = np.concatenate([q - 2, q - 1, q, q + 1, rng.integers(0, 1 << 32, 1 << 20), [0, (1 << 32) - 1]])
    cand = cand[(cand >= 0) & (cand < (1 << 32))]
    want = np.searchsorted(-Q, -cand, side="left") - 1  # G = #{g : v < Q[g]} - 1 (Q non-increasing)
    v = torch.from_numpy(cand.astype(np.uint32).view(np.int32)).cuda()
    got = S.gap_check(p32, v).cpu().numpy()
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, (p32, cand[bad[:5]], got[bad[:5]], want[bad[:5]])


@pytest.mark.parametrize("name", ["c3", "c4_11"])
def test_final_amplitudes_fp32_vs_fp64(name):
    """The amplitude probe: unit-norm final active vectors, FP32 within 1e-5 of FP64 on shots whose
    records agree in both precisions, and a width equal to the plan's last width."""
    w = configs.c3() if name == "c3" else configs.c4()[11]
    p = S.Program(w.circuit)
    n = 64
    a64 = p.probe_amplitudes(0, n, w.seed, precision="fp64")
    a32 = p.probe_amplitudes(0, n, w.seed, precision="fp32")
    k_end = int(p.plan()["k"][-1])
    assert a64.shape == (n, 1 << k_end) and k_end > 0
    assert np.allclose(np.sum(np.abs(a64) ** 2, axis=1), 1.0, atol=1e-12)
    assert np.allclose(np.sum(np.abs(a32) ** 2, axis=1), 1.0, atol=1e-5)
    r64 = _gpu(p, n, w.seed, precision="fp64")
    r32 = _gpu(p, n, w.seed, precision="fp32")
    same = [s for s in range(n)
            if np.array_equal((r32[:, s // 64] >> np.uint64(s % 64)) & np.uint64(1),
                              (r64[:, s // 64] >> np.uint64(s % 64)) & np.uint64(1))]
    assert len(same) >= n - 2
    assert np.max(np.abs(a32[same] - a64[same])) < 1e-5


@pytest.mark.parametrize("name,prec", [("c3", "fp64"), ("c3", "fp32"), ("c4_11", "fp64"), ("random", "fp64")])
def test_final_amplitudes_match_oracle(name, prec):
    """The amplitude probe against the oracle's own final active vector (which
    carries concrete signs where the kernels keep a symbolic Pauli frame): per
    shot, equal up to the frame's index shift x -> x XOR y, sign character
    (-1)^(s.x) and global phase, within 1e-9 (FP64) or 1e-5 (FP32), on every
    shot whose records agree with the oracle's."""
    if name == "random":
        rng = np.random.default_rng(99)
        cases = []
        while len(cases) < 6:
            c = random_circuit(rng, int(rng.integers(3, 8)), int(rng.integers(20, 60)))
            if int(S.Program(c).plan()["k"][-1]) > 0:
                cases.append((c, 777 + len(cases)))
    else:
        w = configs.c3() if name == "c3" else configs.c4()[11]
        cases = [(w.circuit, w.seed)]
    tol = 1e-9 if prec == "fp64" else 1e-5
    n = 64
    for circ, seed in cases:
        p = S.Program(circ)
        oc = OracleCircuit(circ)
        print(f"probe vs oracle: {name} k_max={p.k_max} {prec}", flush=True)
        amp = p.probe_amplitudes(0, n, seed, precision=prec)
        rec = _gpu(p, n, seed, precision=prec)
        want = oc.sample(seed, n)
        checked = 0
        for shot in range(n):
            bit = np.uint64(shot % 64)
            if not np.array_equal((rec[:, shot // 64] >> bit) & np.uint64(1), (want[:, shot // 64] >> bit) & np.uint64(1)):
                continue
            fs = oc.final_state(seed, shot)
            assert amp.shape[1] == 1 << fs["k"]
            assert frame_relation(amp[shot], fs["alpha"], tol) is not None, (name, shot)
            checked += 1
        assert checked >= n - 2
