"""GPU parity on degenerate inputs, through the C ABI, against the CPU oracle.

* No noise at all (no probability class): the frame kernel's walks have no stream.
* Certain events (p = 1): every position of every stream fires, and every
  branch draw picks among all branches.
* Heavy noise (p = 0.3) on a surface code.
* A single shot, on the frame and the active path.
* Rotations by 0 and by pi (R_P(pi) = -iP, a Pauli), which promote a
  coordinate whose new half (angle 0) or old half (pi) carries no amplitude.
* Programs with no rows, on both paths: sampling writes nothing and succeeds.
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
from workloads.circuit import Circuit  # noqa: E402
from workloads.surface import rotated_memory_z  # noqa: E402

TOL = {"fp64": 1e-9, "fp32": 1e-5}
ALL = np.uint64(0xFFFFFFFFFFFFFFFF)


def _gpu(prog, shots, seed, **kw):
    return S.bits_to_numpy(prog.sample(shots, seed, **kw))


def test_noiseless_frame_program():
    c = rotated_memory_z(3, 3, 0.0)
    p = S.Program(c)
    assert p.k_max == 0 and p.info()["n_classes"] == 0
    print("noiseless surface d3 r3", flush=True)
    got = _gpu(p, 64 * 20, 3)
    assert np.array_equal(got, OracleCircuit(c).sample(3, 64 * 20))
    nr, nd = c.num_records, c.num_detectors
    assert not np.any(got[nr:nr + nd])


def test_certain_events():
    c = Circuit(6)
    c.append("X_ERROR", [0, 1, 2], arg=1.0)
    c.append("M", [0, 1, 2])                      # always 1
    c.append("DEPOLARIZE1", [3], arg=1.0)
    c.append("DEPOLARIZE2", [4, 5], arg=1.0)
    c.append("M", [3, 4, 5])
    c.append("MR", [0, 1, 2], arg=1.0)            # true 1, reported 0
    c.detector([0, 6])
    p = S.Program(c)
    assert p.k_max == 0
    print("certain events", flush=True)
    got = _gpu(p, 64 * 33 + 7, 4)
    assert np.array_equal(got, OracleCircuit(c).sample(4, 64 * 33 + 7))
    last = np.uint64((1 << 7) - 1)
    for r in range(3):
        assert np.all(got[r, :-1] == ALL) and got[r, -1] == last
        assert not np.any(got[6 + r])


def test_heavy_noise_surface():
    c = rotated_memory_z(3, 2, 0.3)
    p = S.Program(c)
    print("surface d3 r2 p=0.3", flush=True)
    assert np.array_equal(_gpu(p, 64 * 40, 5), OracleCircuit(c).sample(5, 64 * 40))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_single_shot(prec):
    rng = np.random.default_rng(17)
    surf = rotated_memory_z(3, 3, 1e-2)
    for c in [surf] + [random_circuit(rng, 5, 40) for _ in range(4)]:
        p = S.Program(c)
        oc = OracleCircuit(c)
        print(f"single shot k_max={p.k_max} {prec}", flush=True)
        got = _gpu(p, 1, 8, precision=prec, shot_offset=64 * 5)
        assert got.shape == (c.num_rows, 1)
        assert not np.any(got[:, 0] >> np.uint64(1))
        compare_records(got, oc.sample(8, 1, shot_begin=64 * 5), c, oc, 8, 64 * 5, TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rotations_by_zero_and_pi(prec):
    rng = np.random.default_rng(23)
    for trial in range(8):
        c = random_circuit(rng, int(rng.integers(3, 7)), int(rng.integers(15, 50)))
        # every rotation of the circuit by 0 or by pi
        from workloads.circuit import Op
        c.ops = [Op(o.name, o.targets, o.pauli, o.negate, float(np.pi) if (i % 2) else 0.0, o.recs, o.obs, o.branches)
                 if o.name == "ROT" else o for i, o in enumerate(c.ops)]
        p = S.Program(c)
        oc = OracleCircuit(c)
        seed = 900 + trial
        print(f"rotations by 0 / pi: trial {trial} k_max={p.k_max} {prec}", flush=True)
        compare_records(_gpu(p, 64 * 2, seed, precision=prec), oc.sample(seed, 64 * 2), c, oc, seed, 0, TOL[prec])


def test_programs_without_rows():
    c = Circuit(4)
    c.append("H", [0, 1])
    c.append("CX", [0, 2])
    c.append("X_ERROR", [1, 3], arg=0.1)
    c.append("R", [2])
    c.rot([(0, "X"), (3, "Z")], 0.4)              # X0 anticommutes with Z0 after the reset: a promotion
    frame = Circuit(4)
    frame.append("H", [0])
    frame.append("DEPOLARIZE1", [0, 1], arg=0.2)
    frame.append("R", [0])
    for circ, active in ((c, True), (frame, False)):
        p = S.Program(circ)
        assert p.n_rows == 0 and (p.k_max > 0) == active
        print(f"no rows, active={active}", flush=True)
        out = p.sample(1000, 9)
        torch.cuda.synchronize()
        assert tuple(out.shape) == (0, 16)
        rc = S._lib.symft_sample(p.handle, 1000, 9, None, None)
        assert rc == 0
