"""The allocation-free entry point captured in a HIP graph (paper Sec. 6, batch sampler on the device; the
launch-latency-bound small-circuit case): replays with eager work between them give the eager call's records
every time, on the frame kernel (C1) and on the active kernels (C3 on its tuned kernel, a dense width-4
program on the shot-group kernel)."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_28600_amd as S  # noqa: E402
from workloads import configs  # noqa: E402


def _cases():
    w1 = configs.c1()
    w3 = configs.c3(shots=64 * 40)
    w4 = [x for x in configs.c4() if S.Program(x.circuit, components="off").k_max == 4][0]
    return [("c1", S.Program(w1.circuit), w1.shots, w1.seed, "fp64", 0),
            ("c3", S.Program(w3.circuit), w3.shots, w3.seed, "fp32", 0),
            ("c4_k4_dense", S.Program(w4.circuit, components="off"), 64 * 9 + 5, w4.seed, "fp64", 1)]


@pytest.mark.parametrize("case", [0, 1, 2])
def test_noalloc_graph_replays(case):
    name, p, shots, seed, prec, ak = _cases()[case]
    words = (shots + 63) // 64
    want = p.sample(shots, seed, precision=prec, active_kernel=ak)   # also makes the program resident
    torch.cuda.synchronize()
    out = torch.zeros((p.n_rows, words), dtype=torch.int64, device="cuda")
    # one eager call first: it looks up the fixed scratch's device address outside the capture
    p.sample_noalloc_into(out, shots, seed, precision=prec, active_kernel=ak)
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    print(f"graph capture {name}", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        p.sample_noalloc_into(out, shots, seed, precision=prec, active_kernel=ak)
    for rep in range(3):
        out.fill_(-1)                   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), (name, rep)
