"""GPU parity of the product-component representation (paper Sec. 6): per-component vectors with exact
Kronecker merges, through the C ABI, against the dense FP64 oracle.

Records must equal the oracle's outside the threshold exclusion, and branch probabilities must agree with
the oracle's to 1e-12 (FP64) / 1e-5 (FP32), on separable states, on states whose components merge, on the
near-Clifford workloads at every width, with ragged shot counts and offsets, in single launches, batches and
count mode.
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
from oracle.counts import count_flags  # noqa: E402
from tests.parity_util import compare_records  # noqa: E402
from tests.randcirc import random_circuit  # noqa: E402
from workloads import configs  # noqa: E402
from workloads.circuit import Circuit  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}
P0_TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _gpu(prog, shots, seed, **kw):
    return S.bits_to_numpy(prog.sample(shots, seed, **kw))


def _p0_vs_oracle(p, oc, seed, shots, prec):
    """Branch probabilities of the GPU probe against the oracle's, up to the first draw that could flip."""
    p0 = p.probe(shots[0], len(shots), seed, precision=prec)
    worst = 0.0
    for i, s in enumerate(shots):
        tr = oc.trace(seed, s)
        for t in np.flatnonzero(tr["meas_kind"] >= 2):
            worst = max(worst, abs(p0[i, t] - tr["p0"][t]))
            if abs(O.active_u(seed, int(t), s) - tr["p0"][t]) < TOL[prec]:
                break
    return worst


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_independent_rotations(prec):
    """Twelve independent rotated qubits: a dense width of 12 against twelve components of two amplitudes;
    every branch probability is cos^2(theta/2)."""
    thetas = np.linspace(0.15, 2.9, 12)
    c = Circuit(12)
    for q, t in enumerate(thetas):
        c.rot([(q, "X")], float(t))
    for q in range(12):
        c.append("M", [q])
    p = S.Program(c, components="on")
    assert p.info()["product_selected"] == 1 and p.k_max == 12
    oc = OracleCircuit(c)
    n, seed = 64 * 9 + 5, 99
    print(f"independent rotations {prec}", flush=True)
    compare_records(_gpu(p, n, seed, precision=prec), oc.sample(seed, n), c, oc, seed, 0, TOL[prec])
    p0 = p.probe(64, 16, seed, precision=prec)
    assert np.max(np.abs(p0 - np.cos(thetas / 2) ** 2)) < P0_TOL[prec]


def _coupled(seed):
    """Promotions in four groups; rotations inside a group, then across groups (merges of two and of three
    components), with measurements and Cliffords in between."""
    rng = np.random.default_rng(seed)
    c = Circuit(10)
    for q in range(10):
        c.rot([(q, "X")], float(rng.uniform(0.2, 2.8)))
    groups = [[0, 1, 2], [3, 4], [5, 6, 7], [8, 9]]
    for g in groups:
        c.rot([(q, "Z") for q in g], float(rng.uniform(-2, 2)))
    c.mpp([(1, "Z")])
    c.append("CX", [3, 5])
    c.rot([(0, "Z"), (4, "Y")], 0.7)
    c.rot([(2, "X"), (6, "Z"), (9, "Z")], -1.1)
    c.append("H", [7])
    c.mpp([(0, "X"), (8, "Z")])
    for q in range(10):
        c.append("M", [q])
    c.detector([0, 1])
    c.observable(0, [c.num_records - 1])
    return c


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coupled_components_merge(prec):
    for seed in (1, 2, 3):
        c = _coupled(seed)
        p = S.Program(c, components="on")
        i = p.info()
        assert i["product_merges"] >= 3, i["product_merges"]
        oc = OracleCircuit(c)
        n, off = 64 * 5 + 33, 64 * 3
        print(f"coupled seed {seed} {prec}: {i['product_components']} components, {i['product_merges']} merges",
              flush=True)
        compare_records(_gpu(p, n, seed, shot_offset=off, precision=prec), oc.sample(seed, n, shot_begin=off), c,
                        oc, seed, off, TOL[prec])
        assert _p0_vs_oracle(p, oc, seed, list(range(off, off + 12)), prec) < P0_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_branch_probabilities(prec):
    w = configs.c3()
    p = S.Program(w.circuit, components="on")
    oc = OracleCircuit(w.circuit)
    assert _p0_vs_oracle(p, oc, w.seed, list(range(64 * 7, 64 * 7 + 24)), prec) < P0_TOL[prec]


@pytest.mark.parametrize("k", [3, 6, 9, 12])
def test_c4_member_branch_probabilities(k):
    i = [j for j, x in enumerate(configs.c4()) if S.Program(x.circuit).k_max == k][0]
    w = configs.c4()[i]
    p = S.Program(w.circuit, components="on")
    oc = OracleCircuit(w.circuit)
    for prec in ("fp64", "fp32"):
        assert _p0_vs_oracle(p, oc, w.seed, list(range(64, 64 + 16)), prec) < P0_TOL[prec]


def test_random_circuits_forced_on():
    """Every random circuit with an active state, with components forced on (the automatic choice would keep
    some dense)."""
    rng = np.random.default_rng(777)
    done = 0
    while done < 25:
        c = random_circuit(rng, int(rng.integers(3, 9)), int(rng.integers(20, 90)))
        p = S.Program(c, components="on")
        if not p.info()["product_selected"]:
            continue
        oc = OracleCircuit(c)
        seed = 4100 + done
        want = oc.sample(seed, 64 * 3 + 7)
        for prec in ("fp64", "fp32"):
            compare_records(_gpu(p, 64 * 3 + 7, seed, precision=prec), want, c, oc, seed, 0, TOL[prec])
        done += 1


def test_postselect_forced_on_records_and_counts():
    """The coherent-noise d=5 code forced onto components (44 merges, a 12,288-amplitude buffer in HBM
    scratch): records against the oracle, and count-mode flags against its own records."""
    w = configs.postselect()
    p = S.Program(w.circuit, components="on")
    i = p.info()
    assert i["product_selected"] == 1 and i["product_merges"] > 10
    oc = OracleCircuit(w.circuit)
    n, off = 64 * 2 + 9, 64 * 5
    print("postselect forced on", flush=True)
    rec = _gpu(p, n, w.seed, shot_offset=off, precision="fp64")
    compare_records(rec, oc.sample(w.seed, n, shot_begin=off), w.circuit, oc, w.seed, off, TOL["fp64"])
    post = list(range(p.n_det))
    f, cnt = p.sample_counts(n, w.seed, post=post, shot_offset=off, precision="fp64")
    own, own_c = count_flags(rec, p.n_rec, p.n_det, p.n_obs, n, post, None)
    assert np.array_equal(S.bits_to_numpy(f), own)
    assert list(cnt.cpu().numpy()) == list(own_c)


def test_batch_mixes_product_and_dense_members():
    """A batch of members on components and members on the dense vector (the same circuits compiled both
    ways), graph-replayed: every member equals its single launch and the oracle."""
    ws = [configs.c4()[j] for j in (2, 7, 11, 30, 55)] + [configs.c3(shots=64 * 4)]
    circs = [x.circuit for x in ws]
    progs = [S.Program(c, components=m) for c in circs for m in ("on", "off")]
    shots = [64 * 3 + 17 * (j % 3) for j in range(len(progs))]
    seeds = [ws[j // 2].seed for j in range(len(progs))]
    outs = [torch.zeros((p.n_rows, (s + 63) // 64), dtype=torch.int64, device="cuda") for p, s in zip(progs, shots)]
    for _ in range(2):
        S.sample_batch(progs, shots, seeds, outs, precision="fp64", graph=True)
        torch.cuda.synchronize()
    for j, p in enumerate(progs):
        c = circs[j // 2]
        oc = OracleCircuit(c)
        got = S.bits_to_numpy(outs[j])
        compare_records(got, oc.sample(seeds[j], shots[j]), c, oc, seeds[j], 0, TOL["fp64"])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_c4_full_batch_sampled_words(prec):
    """The 128-program batch at its full size (the benchmark's launch: most members on components), on
    words spread over its largest members."""
    ws = configs.c4()
    progs = [S.Program(x.circuit) for x in ws]
    outs = [torch.zeros((p.n_rows, (x.shots + 63) // 64), dtype=torch.int64, device="cuda") for p, x in zip(progs, ws)]
    S.sample_batch(progs, [x.shots for x in ws], [x.seed for x in ws], outs, precision=prec, graph=True)
    torch.cuda.synchronize()
    for j in (11, 23, 70, 127):
        x = ws[j]
        oc = OracleCircuit(x.circuit)
        nw = (x.shots + 63) // 64
        words = [0, nw // 3, nw - 1]
        got = S.bits_to_numpy(outs[j][:, words])
        want = oc.sample_words(x.seed, words)
        for q, wd in enumerate(words):
            compare_records(got[:, q:q + 1], want[:, q:q + 1], x.circuit, oc, x.seed, 64 * wd, TOL[prec])
