"""GPU parity of the two pure-frame kernels and the choice between them.

The wave-owned kernel (each wave of a 16-wave workgroup owns one 64-shot word
for the whole schedule) and the step-synchronous kernel must both give the
oracle's records bit for bit; schedules too large for the first run on the
second, and schedules too large for both run on the active kernel, with the
same records.
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
from workloads import configs  # noqa: E402
from workloads.surface import rotated_memory_z  # noqa: E402


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


def test_automatic_choice_is_the_step_kernel(c1, c2):
    assert c1[1].info()["frame_kernel"] == 2
    assert c2[1].info()["frame_kernel"] == 2


@pytest.mark.parametrize("fk", [1, 2])
def test_c1_both_kernels_bit_exact(c1, fk):
    w, p, oc = c1
    print(f"C1 frame kernel {fk}", flush=True)
    assert np.array_equal(_gpu(p, w.shots, w.seed, frame_kernel=fk), oc.sample(w.seed, w.shots))
    # ragged at an offset: a partial last tile and a partial last word
    assert np.array_equal(_gpu(p, 1000, w.seed, shot_offset=64 * 37, frame_kernel=fk),
                          oc.sample(w.seed, 1000, shot_begin=64 * 37))
    # one word, then one shot
    assert np.array_equal(_gpu(p, 64, w.seed, shot_offset=64 * 5, frame_kernel=fk),
                          oc.sample(w.seed, 64, shot_begin=64 * 5))
    assert np.array_equal(_gpu(p, 1, w.seed, frame_kernel=fk), oc.sample(w.seed, 1))


def test_c2_wave_kernel_bit_exact(c2):
    """Two 16-word tiles and a partial third, a ragged range at an offset, and the step kernel's records."""
    w, p, oc = c2
    print("C2 wave kernel", flush=True)
    n = 64 * 40 + 29
    want = oc.sample(w.seed, n, threads=0)
    got = _gpu(p, n, w.seed, frame_kernel=1)
    assert np.array_equal(got, want)
    assert np.array_equal(got, _gpu(p, n, w.seed, frame_kernel=2))
    off = 64 * 1000
    assert np.array_equal(_gpu(p, 64 * 3 + 7, w.seed, shot_offset=off, frame_kernel=1),
                          oc.sample(w.seed, 64 * 3 + 7, shot_begin=off))


def test_c2_wave_kernel_full_size_sampled_words(c2):
    """The benchmark's launch (2^24 shots, about 64 tiles per workgroup): words spread over the range."""
    w, p, oc = c2
    print("C2 full size, wave kernel", flush=True)
    out = p.sample(w.shots, w.seed, frame_kernel=1)
    words = [0, 15, 16, 4095, 131071, 262143]
    got = S.bits_to_numpy(out[:, words])
    del out
    assert np.array_equal(got, oc.sample_words(w.seed, words))


@pytest.mark.parametrize("cap", [0, 8, 1100, 1400])
def test_wave_kernel_overflow_fallback(c2, cap):
    """cap slot flips kept per (word, class): 8 sends every word down the fallback that draws its events
    again at every NOISE step; 1100 and 1400, near the mean, send some words and keep others."""
    w, p, oc = c2
    print(f"C2 wave kernel, cap {cap}", flush=True)
    n = 64 * 20
    assert np.array_equal(_gpu(p, n, w.seed, frame_entry_cap=cap, frame_kernel=1), oc.sample(w.seed, n, threads=0))


@pytest.mark.parametrize("k", [3, 12])
@pytest.mark.parametrize("cap", [0, 8])
def test_wave_kernel_multiclass(k, cap):
    from tests.test_gpu_parity import _multiclass_surface
    c = _multiclass_surface(5, 4, k)
    p = S.Program(c)
    assert p.info()["frame_kernel"] == 2
    oc = OracleCircuit(c)
    seed = 0xC1A55 + k
    n = 64 * 40 + 17
    assert np.array_equal(_gpu(p, n, seed, frame_entry_cap=cap, frame_kernel=1), oc.sample(seed, n))


def test_wave_kernel_sections_and_stride(c1):
    w, p, oc = c1
    want = oc.sample(w.seed, 1024)
    n_rec, n_det = w.circuit.num_records, w.circuit.num_detectors
    for sec, rows in ((1, slice(0, n_rec)), (2, slice(n_rec, n_rec + n_det)), (4, slice(n_rec + n_det, None))):
        out = torch.zeros((p.n_rows, 20), dtype=torch.int64, device="cuda")
        p.sample_into(out, 1024, w.seed, sections=sec, row_stride_words=20, frame_kernel=1)
        got = S.bits_to_numpy(out)
        assert np.array_equal(got[rows, :16], want[rows])
        mask = np.ones(p.n_rows, dtype=bool)
        mask[rows] = False
        assert not np.any(got[mask]) and not np.any(got[:, 16:])


@pytest.mark.parametrize("fk", [1, 2])
def test_wave_kernel_counts(c1, c2, fk):
    """Aggregate counts from both frame kernels equal those of the oracle's records."""
    for w, p, oc, n in ((c1[0], c1[1], c1[2], 64 * 37 + 3), (c2[0], c2[1], c2[2], 64 * 20 + 5)):
        c = w.circuit
        post = list(range(0, c.num_detectors, 2))
        flags, counts = p.sample_counts(n, w.seed, post=post, shot_offset=64 * 3, frame_kernel=fk)
        want = oc.sample(w.seed, n, shot_begin=64 * 3)
        wf, wc = count_flags(want, c.num_records, c.num_detectors, c.num_observables, n, post, None)
        assert np.array_equal(S.bits_to_numpy(flags), wf)
        assert list(counts.cpu().numpy()) == list(wc)


def test_schedule_past_the_wave_kernel_runs_on_the_step_kernel():
    c = rotated_memory_z(17, 3, 1e-3)
    p = S.Program(c)
    assert p.info()["frame_kernel"] == 2
    with pytest.raises(S.SymftError) as ei:
        _gpu(p, 64, 5, frame_kernel=1)
    assert ei.value.code == -5
    oc = OracleCircuit(c)
    print("d17 r3: step kernel", flush=True)
    assert np.array_equal(_gpu(p, 64 * 2, 5), oc.sample(5, 64 * 2))


def test_schedule_past_both_frame_kernels_runs_on_the_active_kernel():
    """A pure-Clifford schedule whose slots fit neither frame kernel's LDS (d = 19, 3 rounds: 1,301 slots)
    runs on the active kernel, bit for bit."""
    c = rotated_memory_z(19, 3, 1e-3)
    p = S.Program(c)
    info = p.info()
    assert info["k_max"] == 0 and info["frame_kernel"] == 0
    oc = OracleCircuit(c)
    print("d19 r3: active kernel", flush=True)
    assert np.array_equal(_gpu(p, 64 * 2 - 9, 11, shot_offset=64 * 7), oc.sample(11, 64 * 2 - 9, shot_begin=64 * 7))


def _fanout_circuit(n=24, p=0.05):
    """An error on the control of a CX fan-out flips every later record: an event of up to n + 1 slot flips
    (seven packed entries: the record's two, two from the extension, three more from its list)."""
    from workloads.circuit import Circuit
    c = Circuit(n)
    c.append("X_ERROR", [0], arg=p)
    c.append("DEPOLARIZE1", [0], arg=p)
    c.append("CX", [q for t in range(1, n) for q in (0, t)])
    c.append("M", list(range(n)))
    for i in range(n - 1):
        c.detector([i, i + 1])
    c.observable(0, [n - 1])
    return c


@pytest.mark.parametrize("fk", [1, 2])
@pytest.mark.parametrize("cap", [0, 8])
def test_events_with_many_flips_bit_exact(fk, cap):
    c = _fanout_circuit()
    p = S.Program(c)
    info = p.info()
    assert info["k_max"] == 0 and info["frame_slots"] > 16
    oc = OracleCircuit(c)
    seed = 0xFA9 + fk
    n = 64 * 40 + 11
    print(f"fan-out, frame kernel {fk}, cap {cap}", flush=True)
    assert np.array_equal(_gpu(p, n, seed, frame_entry_cap=cap, frame_kernel=fk), oc.sample(seed, n))
    off = 64 * 9
    assert np.array_equal(_gpu(p, 64 * 3, seed, shot_offset=off, frame_entry_cap=cap, frame_kernel=fk),
                          oc.sample(seed, 64 * 3, shot_begin=off))
