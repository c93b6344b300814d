"""The allocation-free entry point (symft_sample_noalloc) against symft_sample_ex.

Every kernel's scratch comes from the library's fixed device array, so a
launch may run fewer workgroups than symft_sample_ex would; records never
depend on the grid, so the two entry points must agree bit for bit.  Each
case makes two calls in a row through the C ABI, the second with a smaller
input, on: the wave-owned frame kernel (surface codes d = 3 and d = 11), the
step-synchronous frame kernel, the active kernel with vectors in LDS (FP32
and FP64), and the active kernel with vectors in HBM scratch at widths 14 and
16 (grids capped by the fixed scratch).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_28600_amd as S  # noqa: E402
from workloads import configs  # noqa: E402
from workloads.surface import rotated_memory_z  # noqa: E402


def _ex(p, n, seed, off, prec, fk=0):
    out = torch.full((max(p.n_rows, 1), (n + 63) // 64), -1, dtype=torch.int64, device="cuda")
    out.zero_()
    p.sample_into(out, n, seed, shot_offset=off, precision=prec, frame_kernel=fk)
    return out


def _noalloc(p, n, seed, off, prec, fk=0):
    out = torch.full((max(p.n_rows, 1), (n + 63) // 64), -1, dtype=torch.int64, device="cuda")
    out.zero_()
    p.sample_noalloc_into(out, n, seed, shot_offset=off, precision=prec, frame_kernel=fk)
    return out


CASES = [
    ("surface_d3", lambda: configs.c1().circuit, "fp64", 0, (64 * 300 + 17, 64 * 20 + 3)),
    ("surface_d11_wave", lambda: configs.c2(64).circuit, "fp64", 1, (64 * 2000 + 5, 64 * 33)),
    ("surface_d11_step", lambda: configs.c2(64).circuit, "fp64", 2, (64 * 1200, 64 * 40 + 9)),
    ("near_clifford_k8_fp32", lambda: configs.c3(64).circuit, "fp32", 0, (64 * 900 + 1, 64 * 10)),
    ("near_clifford_k8_fp64", lambda: configs.c3(64).circuit, "fp64", 0, (64 * 600, 64 * 7 + 63)),
    ("near_clifford_k14_fp32", lambda: configs.c5(14).circuit, "fp32", 0, (64 * 300, 64 * 20 + 1)),
    ("near_clifford_k16_fp32", lambda: configs.c5(16).circuit, "fp32", 0, (64 * 70, 64 * 3)),
]


@pytest.mark.parametrize("name,make,prec,fk,sizes", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_sample_ex(name, make, prec, fk, sizes):
    p = S.Program(make())
    seed = 0xA110C + len(name)
    # the program becomes resident on the device through the ordinary entry point
    _ex(p, 64, seed, 0, prec, fk)
    for n, off in ((sizes[0], 64 * 3), (sizes[1], 0)):
        print(f"no-alloc {name}: {n} shots at offset {off}", flush=True)
        want = S.bits_to_numpy(_ex(p, n, seed, off, prec, fk))
        got = S.bits_to_numpy(_noalloc(p, n, seed, off, prec, fk))
        assert np.array_equal(got, want), name


def test_noalloc_rejects_a_program_not_resident_here():
    p = S.Program(configs.c1().circuit)
    out = torch.zeros((p.n_rows, 4), dtype=torch.int64, device="cuda")
    with pytest.raises(S.SymftError) as ei:
        p.sample_noalloc_into(out, 256, 1)
    assert ei.value.code == -1
    assert int((out != 0).sum()) == 0


def test_noalloc_rejects_a_workgroup_past_the_fixed_scratch():
    """A width-23 state in FP64 (the dense vector) needs 128 MiB of vector scratch for its one shot group:
    ECAPACITY, raised before any launch."""
    from tests.randcirc import wide_circuit
    c = wide_circuit(19, 7)
    p = S.Program(c, components="off")
    assert p.k_max == 23
    # the autotuner uploads the program (and times nothing at widths past 14)
    p.autotune("fp64")
    out = torch.zeros((p.n_rows, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(S.SymftError) as ei:
        p.sample_noalloc_into(out, 64, 3, precision="fp64")
    assert ei.value.code == -5
