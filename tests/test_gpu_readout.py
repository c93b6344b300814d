"""GPU parity of readout flips (paper Sec. 6: readout flips are exogenous
symbols): records and aggregate counts from the HIP kernels vs the CPU oracle,
with every recorded measurement carrying a flip probability.

Pure-Clifford programs must match bit for bit; near-Clifford ones under the
same rule as the other record parity tests (a shot may differ only where an
active-measurement draw lies within the precision's tolerance of its branch
threshold).
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
from tests.test_gpu_counts import _check  # noqa: E402
from workloads.surface import rotated_memory_z  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}


def _gpu(prog, shots, seed, **kw):
    return S.bits_to_numpy(prog.sample(shots, seed, **kw))


@pytest.fixture(scope="module")
def surface():
    c = rotated_memory_z(5, 5, 2e-3, p_meas=1e-2)
    return c, S.Program(c), OracleCircuit(c)


def test_surface_with_flips_bit_exact(surface):
    c, p, oc = surface
    assert p.k_max == 0
    seed = 97
    print("surface d5 r5 readout flips: 1280 shots", flush=True)
    assert np.array_equal(_gpu(p, 64 * 20, seed), oc.sample(seed, 64 * 20))
    print("surface d5 r5 readout flips: 1000 shots at word 37", flush=True)
    got = _gpu(p, 1000, seed, shot_offset=64 * 37)
    assert np.array_equal(got, oc.sample(seed, 1000, shot_begin=64 * 37))


def test_surface_with_flips_counts(surface):
    c, p, oc = surface
    nd = c.num_detectors
    _check(c, p, oc, 64 * 12 + 5, 98, list(range(0, nd, 2)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coherent_surface_with_flips(prec):
    c = rotated_memory_z(3, 3, 2e-3, coherent=0.15, p_meas=2e-2)
    p = S.Program(c)
    assert p.k_max > 0
    oc = OracleCircuit(c)
    seed = 99
    print(f"coherent surface d3 r3 readout flips k_max={p.k_max} {prec}", flush=True)
    got = _gpu(p, 64 * 4, seed, precision=prec)
    compare_records(got, oc.sample(seed, 64 * 4), c, oc, seed, 0, TOL[prec])


def test_random_circuits_with_flips():
    rng = np.random.default_rng(4711)
    for trial in range(20):
        c = random_circuit(rng, int(rng.integers(2, 8)), int(rng.integers(10, 60)), p_flip=0.3)
        p = S.Program(c)
        oc = OracleCircuit(c)
        seed = 5000 + trial
        for prec in ("fp64", "fp32"):
            print(f"random circuit {trial} with flips k_max={p.k_max} {prec}", flush=True)
            got = _gpu(p, 64 * 3, seed, precision=prec)
            compare_records(got, oc.sample(seed, 64 * 3), c, oc, seed, 0, TOL[prec])
