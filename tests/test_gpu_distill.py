"""GPU parity on the 15-to-1 distillation workload (peak width 5, every
detector postselected): records in both precisions and aggregate counts,
through the C ABI, against the CPU oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_28600_amd as S  # noqa: E402
from oracle import OracleCircuit  # noqa: E402
from tests.parity_util import compare_records  # noqa: E402
from tests.test_gpu_counts import _check  # noqa: E402
from workloads.distill import distill_15to1  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}


@pytest.fixture(scope="module")
def distill():
    c = distill_15to1(1e-2)
    return c, S.Program(c), OracleCircuit(c)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_distillation_records(distill, prec):
    c, p, oc = distill
    assert p.k_max == 5
    seed = 1515
    print(f"distillation records {prec}", flush=True)
    got = S.bits_to_numpy(p.sample(64 * 8 + 5, seed, precision=prec))
    compare_records(got, oc.sample(seed, 64 * 8 + 5), c, oc, seed, 0, TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_distillation_counts(distill, prec):
    c, p, oc = distill
    print(f"distillation counts {prec}", flush=True)
    _check(c, p, oc, 64 * 16 + 3, 1516, list(range(c.num_detectors)), prec=prec)
