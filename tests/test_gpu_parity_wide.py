"""GPU parity on the configurations and launch shapes the benchmark runs:
branch probabilities against the oracle on every active workload, full-size
launches of the HBM-resident widths and of the
batched queue (sampled words), and batch plans across freed programs.

Tolerances: records bit-exact outside
the threshold exclusion (1e-9 FP64, 1e-5 FP32), Pr(m = 0) within 1e-12 (FP64)
or 1e-5 (FP32) of the oracle's.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_28600_amd as S  # noqa: E402
from oracle import OracleCircuit  # noqa: E402
from tests.parity_util import compare_records, p0_error  # noqa: E402
from workloads import configs  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}
P0_TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _workload(name):
    if name.startswith("c4_"):
        return configs.c4()[int(name[3:])]
    if name == "c5_k14":
        return configs.c5(14)
    if name == "c5_k16":
        return configs.c5(16)
    if name == "post":
        return configs.postselect()
    if name == "distill":
        return configs.distill()
    raise KeyError(name)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["c4_3", "c4_11", "c4_59", "c4_127", "c5_k14", "c5_k16", "post", "distill"])
def test_branch_probabilities_match_oracle(name, prec):
    """Pr(recorded bit = 0) of every active measurement, from the kernels' probe, against the oracle's,
    on shots spread over the first words (both precisions)."""
    w = _workload(name)
    p = S.Program(w.circuit)
    oc = OracleCircuit(w.circuit)
    n = 12 if p.k_max >= 14 else 24
    s0 = 64 * 3 + 5
    print(f"P0 vs oracle: {name} k_max={p.k_max} {prec}", flush=True)
    p0 = p.probe(s0, n, w.seed, precision=prec)
    worst, cnt = p0_error(p0, oc, w.seed, list(range(s0, s0 + n)), TOL[prec])
    print(f"  {cnt} probabilities, worst {worst:.3e}", flush=True)
    assert cnt > 0
    assert worst < P0_TOL[prec], worst


@pytest.mark.parametrize("k,prec", [(14, "fp32"), (14, "fp64"), (16, "fp32"), (16, "fp64")])
def test_c5_full_launch_sampled_words(k, prec):
    """The benchmark's launch: all 2^16 shots in one call (up to about a thousand shot groups, each with
    its vector slice in HBM scratch, and a grid-stride loop over words where the grid is smaller than
    the 1024 words); words spread over the range, the first and last of a grid-stride pass included,
    against the oracle."""
    w = configs.c5(k)
    p = S.Program(w.circuit)
    p.autotune(prec)
    oc = OracleCircuit(w.circuit)
    print(f"C5 k={k} {prec}: full launch", flush=True)
    out = p.sample(w.shots, w.seed, precision=prec)
    words = [0, 255, 511, 512, 777, 1023]
    got = S.bits_to_numpy(out[:, words])
    del out
    want = oc.sample_words(w.seed, words)
    for j, wd in enumerate(words):
        compare_records(got[:, j:j + 1], want[:, j:j + 1], w.circuit, oc, w.seed, 64 * wd, TOL[prec])


def test_c4_full_batch_sampled_words():
    """The benchmark's batch: all 128 programs at their full shot counts in one graph-replayed launch;
    the first, a middle and the last word of the four programs with the most dense work, against the
    oracle."""
    ws = configs.c4()
    progs = [S.Program(w.circuit) for w in ws]
    outs = [torch.zeros((p.n_rows, (w.shots + 63) // 64), dtype=torch.int64, device="cuda") for p, w in zip(progs, ws)]
    print("C4 full batch", flush=True)
    for _ in range(2):
        S.sample_batch(progs, [w.shots for w in ws], [w.seed for w in ws], outs, precision="fp32", graph=True)
    torch.cuda.synchronize()
    heavy = sorted(range(len(ws)), key=lambda i: -(progs[i].info()["dense_flops_per_shot"] + 1) * ws[i].shots)[:4]
    for i in heavy:
        nw = outs[i].shape[1]
        words = sorted({0, nw // 2, nw - 1})
        got = S.bits_to_numpy(outs[i][:, words])
        oc = OracleCircuit(ws[i].circuit)
        want = oc.sample_words(ws[i].seed, words)
        print(f"  program {i}: k_max={progs[i].k_max} shots={ws[i].shots} words {words}", flush=True)
        for j, wd in enumerate(words):
            g, x = got[:, j:j + 1], want[:, j:j + 1]
            if wd == nw - 1 and ws[i].shots % 64:
                mask = np.uint64((1 << (ws[i].shots % 64)) - 1)
                x = x & mask
            compare_records(g, x, ws[i].circuit, oc, ws[i].seed, 64 * wd, TOL["fp32"])


def test_batch_plan_survives_program_free():
    """Freeing the programs of a cached batch plan releases it: a later batch over new programs with the
    same shots, seeds and output buffers (so a stale plan keyed on reused addresses would match) samples
    the new programs."""
    import gc
    ws_a = configs.c4()[40:48]
    ws_b = configs.c4()[60:68]
    shots = [64 * 4 + 9 * i for i in range(8)]
    seeds = [1000 + i for i in range(8)]
    rows = max(max(S.Program(w.circuit).n_rows for w in ws_a), max(S.Program(w.circuit).n_rows for w in ws_b))
    outs = [torch.zeros((rows, (s + 63) // 64), dtype=torch.int64, device="cuda") for s in shots]
    for rep in range(2):
        ws = ws_a if rep == 0 else ws_b
        progs = [S.Program(w.circuit) for w in ws]
        views = [o[: p.n_rows] for o, p in zip(outs, progs)]
        for v in views:
            v.fill_(-1)
        S.sample_batch(progs, shots, seeds, views, precision="fp32", graph=True)
        torch.cuda.synchronize()
        for i in (0, 3, 7):
            oc = OracleCircuit(ws[i].circuit)
            compare_records(S.bits_to_numpy(views[i]), oc.sample(seeds[i], shots[i]), ws[i].circuit, oc, seeds[i], 0,
                            TOL["fp32"])
        del progs, views
        gc.collect()
