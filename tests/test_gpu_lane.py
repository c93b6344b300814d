"""GPU parity of the lane kernel (symft_sample_opts.active_kernel = 2; paper Sec. 5, the per-shot active
instructions): one wave per 64-shot word, one lane per shot, every shot's vector buffer in LDS
amplitude-major.  Records must equal the oracle's outside the threshold exclusion, on product-component and
dense programs whose per-wave state fits, in both precisions, with ragged shot counts, offsets, sections and
row strides.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_28600_amd as S  # noqa: E402
from oracle import OracleCircuit  # noqa: E402
from tests.parity_util import compare_records  # noqa: E402
from tests.randcirc import random_circuit  # noqa: E402
from workloads import configs  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}


def _lane(prog, shots, seed, **kw):
    return S.bits_to_numpy(prog.sample(shots, seed, active_kernel=2, **kw))


def _fits(prog, prec):
    """The lane kernel's per-wave state (exogenous words, outcome bits, 64 vector buffers) within 64 KB."""
    i = prog.info()
    amps = i["product_vector_amplitudes"] if i["product_selected"] else 1 << i["k_max"]
    n_instr = sum(i["n_instr"].values())
    head = (8 * n_instr + 256 * ((i["n_measurements"] + 31) // 32) + 15) // 16 * 16
    return head + 64 * amps * (16 if prec == "fp64" else 8) <= 65536


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_records(prec):
    w = configs.c3()
    p = S.Program(w.circuit)
    assert p.info()["product_selected"] == 1
    oc = OracleCircuit(w.circuit)
    n, off = 64 * 40 + 21, 64 * 9
    print(f"lane kernel c3 {prec}", flush=True)
    got = _lane(p, n, w.seed, shot_offset=off, precision=prec)
    excluded = compare_records(got, oc.sample(w.seed, n, shot_begin=off), w.circuit, oc, w.seed, off, TOL[prec])
    assert excluded <= max(3, n // 200)
    assert not np.any(got[:, -1] >> np.uint64(n % 64))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_full_size_sampled_words(prec):
    w = configs.c3()
    p = S.Program(w.circuit)
    oc = OracleCircuit(w.circuit)
    out = p.sample(w.shots, w.seed, precision=prec, active_kernel=2)
    words = [0, 4097, 12000, 16383]
    got = S.bits_to_numpy(out[:, words])
    del out
    want = oc.sample_words(w.seed, words)
    for j, wd in enumerate(words):
        compare_records(got[:, j:j + 1], want[:, j:j + 1], w.circuit, oc, w.seed, 64 * wd, TOL[prec])


@pytest.mark.parametrize("comp", ["auto", "off"])
def test_c4_members(comp):
    """Members of every width whose per-wave state fits: on components (auto) and dense (off, widths up to
    about 5 in FP32)."""
    done = 0
    for i, w in enumerate(configs.c4()[:24]):
        p = S.Program(w.circuit, components=comp)
        oc = OracleCircuit(w.circuit)
        n, off = 64 * 4 + 7, 64 * 2
        want = oc.sample(w.seed, n, shot_begin=off)
        for prec in ("fp64", "fp32"):
            if not _fits(p, prec):
                with pytest.raises(S.SymftError):
                    _lane(p, n, w.seed, shot_offset=off, precision=prec)
                continue
            got = _lane(p, n, w.seed, shot_offset=off, precision=prec)
            compare_records(got, want, w.circuit, oc, w.seed, off, TOL[prec])
            done += 1
    assert done >= 20


def test_random_circuits():
    rng = np.random.default_rng(909)
    done = 0
    while done < 25:
        c = random_circuit(rng, int(rng.integers(2, 9)), int(rng.integers(10, 80)))
        p = S.Program(c)
        if p.k_max == 0:
            continue
        oc = OracleCircuit(c)
        seed = 5200 + done
        want = oc.sample(seed, 64 * 3 + 1)
        for prec in ("fp64", "fp32"):
            if not _fits(p, prec):
                continue
            got = _lane(p, 64 * 3 + 1, seed, precision=prec)
            compare_records(got, want, c, oc, seed, 0, TOL[prec])
        done += 1


def test_same_records_as_the_shot_group_kernel():
    w = configs.c3()
    p = S.Program(w.circuit)
    n = 64 * 128
    a = S.bits_to_numpy(p.sample(n, w.seed, precision="fp64", active_kernel=2))
    b = S.bits_to_numpy(p.sample(n, w.seed, precision="fp64", active_kernel=1))
    assert np.array_equal(a, b)


def test_sections_stride_and_noalloc():
    from workloads.surface import rotated_memory_z
    c = rotated_memory_z(3, 3, 1e-3, coherent=0.3)
    p = S.Program(c)
    seed, n = 616, 64 * 6 + 3
    words = (n + 63) // 64
    full = _lane(p, n, seed, precision="fp64")
    oc = OracleCircuit(c)
    compare_records(full, oc.sample(seed, n), c, oc, seed, 0, TOL["fp64"])
    stride = words + 3
    out = torch.full((p.n_rows, stride), -1, dtype=torch.int64, device="cuda")
    p.sample_into(out, n, seed, precision="fp64", sections=6, row_stride_words=stride, active_kernel=2)
    got = S.bits_to_numpy(out)
    nr = p.n_rec
    assert np.array_equal(got[nr:, :words], full[nr:])
    assert np.all(got[:nr] == np.uint64(2 ** 64 - 1))
    assert np.all(got[:, words:] == np.uint64(2 ** 64 - 1))
    nb = torch.zeros((p.n_rows, words), dtype=torch.int64, device="cuda")
    p.sample_noalloc_into(nb, n, seed, precision="fp64", active_kernel=2)
    torch.cuda.synchronize()
    assert np.array_equal(S.bits_to_numpy(nb), full)


def test_too_large_is_refused():
    w = configs.c3()
    p = S.Program(w.circuit, components="off")  # 256 amplitudes x 64 shots: past 64 KB
    with pytest.raises(S.SymftError):
        p.sample(64, w.seed, active_kernel=2)


def test_probes_after_the_autotuner_picks_it():
    """Once the autotuner has chosen the lane kernel (reported as 1 thread per shot), the probes run on it:
    branch probabilities against the oracle (C3 on components, FP64 1e-12) and the final vector of a dense
    width-4 program against the oracle's up to the Pauli frame."""
    import oracle as O
    from tests.parity_util import frame_relation
    w = configs.c3()
    p = S.Program(w.circuit)
    tps = p.autotune("fp64")
    print(f"c3 fp64 autotune: {tps}", flush=True)
    if tps != 1:
        pytest.skip("the autotuner kept the shot-group kernel on this box")
    oc = OracleCircuit(w.circuit)
    shots = list(range(64 * 3, 64 * 3 + 20))
    p0 = p.probe(shots[0], len(shots), w.seed, precision="fp64")
    worst = 0.0
    for i, s in enumerate(shots):
        tr = oc.trace(w.seed, s)
        for t in np.flatnonzero(tr["meas_kind"] >= 2):
            worst = max(worst, abs(p0[i, t] - tr["p0"][t]))
            if abs(O.active_u(w.seed, int(t), s) - tr["p0"][t]) < TOL["fp64"]:
                break
    assert worst < 1e-12, worst
    x = [x for x in configs.c4() if S.Program(x.circuit, components="off").k_max == 4][0]
    q = S.Program(x.circuit, components="off")
    if q.autotune("fp64") != 1:
        pytest.skip("the autotuner kept the shot-group kernel for the width-4 program")
    n = 32
    amp = q.probe_amplitudes(0, n, x.seed, precision="fp64")
    rec = S.bits_to_numpy(q.sample(n, x.seed, precision="fp64"))
    ox = OracleCircuit(x.circuit)
    want = ox.sample(x.seed, n)
    checked = 0
    for shot in range(n):
        bit = np.uint64(shot % 64)
        if not np.array_equal((rec[:, shot // 64] >> bit) & np.uint64(1), (want[:, shot // 64] >> bit) & np.uint64(1)):
            continue
        fs = ox.final_state(x.seed, shot)
        assert amp.shape[1] == 1 << fs["k"]
        assert frame_relation(amp[shot], fs["alpha"], 1e-9) is not None, shot
        checked += 1
    assert checked >= n - 2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_count_mode(prec):
    """Count mode on the lane kernel (threads_per_shot = 1): flags equal those derived from the same kernel's
    full records (a discarded shot's early exit changes no kept shot), counters their popcounts, on a coherent
    distance-3 code with every detector postselected (most shots discarded) and on C3 with a random subset of
    observables' expected values; offsets and a ragged last word."""
    from oracle.counts import count_flags
    from workloads.surface import rotated_memory_z

    def popcount(a):
        return int(sum(bin(int(x)).count("1") for x in np.asarray(a, dtype=np.uint64).reshape(-1)))

    cases = [(rotated_memory_z(3, 3, 1e-3, coherent=0.3), 77), (rotated_memory_z(3, 2, 2e-2, coherent=0.2), 78)]
    for c, seed in cases:
        p = S.Program(c)
        assert _fits(p, prec)
        n, off = 64 * 11 + 37, 64 * 5
        post = list(range(c.num_detectors))
        exp = [1] * c.num_observables
        f, cnt = p.sample_counts(n, seed, post=post, obs_expected=exp, shot_offset=off, precision=prec,
                                 threads_per_shot=1)
        flags = S.bits_to_numpy(f)
        rec = _lane(p, n, seed, shot_offset=off, precision=prec)
        own, own_c = count_flags(rec, c.num_records, c.num_detectors, c.num_observables, n, post, exp)
        assert np.array_equal(flags, own)
        assert list(cnt.cpu().numpy()) == [popcount(flags[0]), popcount(flags[1])] == list(own_c)
        assert popcount(flags[0]) > n // 4  # many discarded: early exits happen
        oc = OracleCircuit(c)
        compare_records(rec, oc.sample(seed, n, shot_begin=off), c, oc, seed, off, TOL[prec])


def test_count_batch_lane_queue():
    """Count mode inside the batched queue: lane-eligible members run the lane queue in count mode; flags equal
    the ones from the same batch's records."""
    from oracle.counts import count_flags
    from workloads.surface import rotated_memory_z
    circs = [rotated_memory_z(3, 3, 1e-3, coherent=0.3), configs.c3(shots=64 * 4).circuit,
             configs.c4()[4].circuit, configs.c4()[17].circuit]
    progs = [S.Program(c) for c in circs]
    shots = [64 * 3 + 11, 64 * 4, 64 * 2 + 1, 64 * 5]
    seeds = [101, 102, 103, 104]
    posts = [list(range(c.num_detectors)) for c in circs]
    flags = [torch.full((2, (s + 63) // 64), -1, dtype=torch.int64, device="cuda") for s in shots]
    counts = torch.zeros(2 * len(progs), dtype=torch.int64, device="cuda")
    S.sample_counts_batch(progs, shots, seeds, posts, flags, counts, precision="fp64")
    outs = [torch.zeros((p.n_rows, (s + 63) // 64), dtype=torch.int64, device="cuda") for p, s in zip(progs, shots)]
    S.sample_batch(progs, shots, seeds, outs, precision="fp64", graph=False)
    torch.cuda.synchronize()
    cnt = counts.cpu().numpy()
    for i, c in enumerate(circs):
        got = S.bits_to_numpy(flags[i])
        own, own_c = count_flags(S.bits_to_numpy(outs[i]), c.num_records, c.num_detectors, c.num_observables,
                                 shots[i], posts[i], None)
        assert np.array_equal(got, own), i
        assert list(cnt[2 * i:2 * i + 2]) == list(own_c), i
