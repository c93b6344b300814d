"""GPU parity of programs compiled with rotation simplification
(symft_compile_opts.simplify; paper Sec. 6): records from the HIP kernels vs
the CPU oracle run on the oracle's own rewrite of the same circuit, in both
precisions, and a cancelled pair that turns a near-Clifford circuit into a
pure-frame program sampled bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_28600_amd as S  # noqa: E402
from oracle import OracleCircuit  # noqa: E402
from oracle.simplify import simplify  # noqa: E402
from tests.parity_util import compare_records  # noqa: E402
from tests.test_simplify import fusable_circuit  # noqa: E402
from workloads.surface import rotated_memory_z  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_simplified_random_circuits(prec):
    rng = np.random.default_rng(8080)
    for trial in range(15):
        c = fusable_circuit(rng, int(rng.integers(2, 8)), int(rng.integers(10, 50)))
        sc, removed = simplify(c)
        p = S.Program(c, simplify=True)
        assert p.info()["rotations_removed"] == removed
        oc = OracleCircuit(sc)
        seed = 4100 + trial
        print(f"simplified circuit {trial}: removed {removed}, k_max {p.k_max}, {prec}", flush=True)
        got = S.bits_to_numpy(p.sample(64 * 3, seed, precision=prec))
        compare_records(got, oc.sample(seed, 64 * 3), sc, oc, seed, 0, TOL[prec])


def test_cancelled_coherent_errors_leave_the_frame_path():
    # a coherent error and its inverse on every data qubit at the start of each round
    c = rotated_memory_z(3, 3, 1e-2, coherent=0.2)
    ops = []
    for o in c.ops:
        ops.append(o)
        if o.name == "ROT":
            ops.append(o.__class__("ROT", pauli=o.pauli, arg=-o.arg))
    c.ops = ops
    p = S.Program(c, simplify=True)
    assert p.k_max == 0 and S.Program(c).k_max > 0
    sc, _ = simplify(c)
    print("surface d3 r3 with cancelled coherent errors", flush=True)
    got = S.bits_to_numpy(p.sample(64 * 10 + 9, 77))
    assert np.array_equal(got, OracleCircuit(sc).sample(77, 64 * 10 + 9))
