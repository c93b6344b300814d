"""The product-component representation (paper Sec. 6): pins of the oracle on
separable circuits, and the host lowering's plan against closed forms.

The oracle keeps one dense active vector; these tests pin it where the state
is a product, so that the GPU's per-component path has a reference whose
behaviour on separable states is fixed by something other than itself:

* independent X rotations measured in Z: every Pr(m=0) is cos^2(theta/2);
* a circuit on two disjoint qubit sets: adding the second set's operations
  changes nothing in the first set's records (outcome draws are keyed by
  measurement index, which the construction keeps equal).

The plan (symft_program_info's product fields) is pinned by closed forms:
one component per promoted coordinate, one merge per coupling of two
components, and regions placed without overlap.
"""
import numpy as np
import pytest

import paper_2607_28600_amd as S
from oracle import OracleCircuit, active_u
from tests.randcirc import random_circuit
from workloads.circuit import Circuit


def _rotations(thetas):
    c = Circuit(len(thetas))
    for q, t in enumerate(thetas):
        c.rot([(q, "X")], float(t))
    for q in range(len(thetas)):
        c.append("M", [q])
    return c


def test_oracle_independent_rotations_closed_form():
    thetas = np.array([0.3, 1.1, -2.0, 2.9, 0.77, -0.5])
    oc = OracleCircuit(_rotations(thetas))
    want = np.cos(thetas / 2) ** 2
    for shot in range(12):
        tr = oc.trace(7, shot)
        assert np.all(tr["meas_kind"] >= 2)  # active measurements, on a state of width up to 6
        assert np.max(np.abs(tr["p0"] - want)) < 1e-12


def _disjoint(seed, with_b):
    """Random rotations, Cliffords and measurements on qubits 0..3 (set A) interleaved with the same on
    qubits 4..7 (set B, only when with_b); every B measurement comes after every A measurement."""
    rng = np.random.default_rng(seed)
    c = Circuit(8)
    a_ops, b_ops = [], []
    for ops, base in ((a_ops, 0), (b_ops, 4)):
        for _ in range(14):
            r = rng.random()
            qs = [base + int(q) for q in rng.choice(4, int(rng.integers(1, 4)), replace=False)]
            if r < 0.35:
                ops.append(("rot", [(q, str(rng.choice(list("XYZ")))) for q in qs], float(rng.uniform(-3, 3))))
            elif r < 0.6:
                ops.append(("gate", str(rng.choice(["H", "S", "CX"])), qs[:2] if len(qs) >= 2 else qs[:1]))
            else:
                ops.append(("mpp", [(q, str(rng.choice(list("XYZ")))) for q in qs]))
    a_meas = [o for o in a_ops if o[0] == "mpp"]
    a_rest = [o for o in a_ops if o[0] != "mpp"]
    b_meas = [o for o in b_ops if o[0] == "mpp"]
    b_rest = [o for o in b_ops if o[0] != "mpp"]

    def put(o):
        if o[0] == "rot":
            c.rot(o[1], o[2])
        elif o[0] == "gate":
            name, qs = o[1], o[2]
            if name == "CX" and len(qs) < 2:
                name = "H"
            c.append(name, qs if name == "CX" else qs[:1])
        else:
            c.mpp(o[1])

    # A's unitaries and B's unitaries interleaved, then A's measurements, then B's
    for i in range(max(len(a_rest), len(b_rest))):
        if i < len(a_rest):
            put(a_rest[i])
        if with_b and i < len(b_rest):
            put(b_rest[i])
    for o in a_meas:
        put(o)
    if with_b:
        for o in b_meas:
            put(o)
    return c, len(a_meas)


@pytest.mark.parametrize("seed", [3, 8, 21])
def test_oracle_disjoint_sets_do_not_interact(seed):
    ca, na = _disjoint(seed, False)
    cab, na2 = _disjoint(seed, True)
    assert na == na2 and na > 0
    n = 256
    ra = OracleCircuit(ca).sample(11, n)
    rab = OracleCircuit(cab).sample(11, n)[:na]
    oab = OracleCircuit(cab)
    diff = np.flatnonzero(np.any(ra[:na] != rab, axis=0))
    for col in diff:
        x = ra[:na, col] ^ rab[:, col]
        for lane in range(64):
            if not np.any((x >> np.uint64(lane)) & np.uint64(1)):
                continue
            # only a draw within rounding of its threshold may differ (the two vectors differ in size)
            tr = oab.trace(11, 64 * int(col) + lane)
            assert any(abs(active_u(11, int(t), 64 * int(col) + lane) - tr["p0"][t]) < 1e-9
                       for t in np.flatnonzero(tr["meas_kind"] >= 2)), (seed, col, lane)


def test_plan_independent_rotations():
    n = 7
    p = S.Program(_rotations(np.linspace(0.2, 2.5, n)), components="on")
    i = p.info()
    assert i["k_max"] == n
    assert i["product_selected"] == 1
    assert i["product_components"] == n and i["product_merges"] == 0
    # all n components are alive at once, 2 amplitudes each, placed side by side
    assert i["product_vector_amplitudes"] == 2 * n
    # per qubit: a promotion from the amplitude 1 (4 flops) and a measurement at width 1
    kinds = i["n_instr"]
    per_meas = 5.0 if kinds["ActiveDiagMeas"] == n else 11.0
    assert i["product_flops_per_shot"] == pytest.approx(n * (4.0 + 2 * per_meas))
    # the dense plan reaches 2^n amplitudes: the automatic choice takes the components
    assert S.Program(_rotations(np.linspace(0.2, 2.5, n))).info()["product_selected"] == 1
    assert S.Program(_rotations(np.linspace(0.2, 2.5, n)), components="off").info()["product_selected"] == 0


def test_plan_merges_on_coupling():
    """n promoted coordinates, then one rotation whose Z mask spans all of them: n - 1 pairwise merges
    (components n + n - 1), the last one of width n."""
    n = 5
    c = Circuit(n)
    for q in range(n):
        c.rot([(q, "X")], 0.4 + 0.1 * q)
    c.rot([(q, "Z") for q in range(n)], 0.9)
    for q in range(n):
        c.append("M", [q])
    p = S.Program(c, components="on")
    i = p.info()
    assert i["k_max"] == n
    assert i["product_components"] == 2 * n - 1 and i["product_merges"] == n - 1
    # the merged component (2^n) and, while it is built, the parts it is built from
    assert (1 << n) <= i["product_vector_amplitudes"] <= 4 << n
    # merging everything does not pay: the automatic choice stays dense
    assert S.Program(c).info()["product_selected"] == 0


def test_plan_automatic_choice_rule():
    rng = np.random.default_rng(5)
    seen = 0
    for _ in range(40):
        c = random_circuit(rng, int(rng.integers(3, 9)), int(rng.integers(20, 80)))
        p = S.Program(c)
        i = p.info()
        if i["k_max"] == 0:
            assert i["product_selected"] == 0
            continue
        seen += 1
        clear = (i["product_flops_per_shot"] + 64 * i["product_merges"] <= 0.5 * i["dense_flops_per_shot"]
                 and i["product_vector_amplitudes"] <= 1 << i["k_max"])
        assert i["product_selected"] == int(clear)
        # a component per promotion and per merge
        assert i["product_components"] == i["n_instr"]["PromoteRot"] + i["product_merges"]
    assert seen > 10


def test_forced_plan_valid_everywhere():
    """With components forced on, every program with an active state gets a product plan: the lowering
    keeps each component's coordinates in dense order, so every pivot stays the highest set bit of its
    local mask (the lowering falls back to dense otherwise, which this would catch)."""
    from workloads import configs
    circs = [configs.c3().circuit, configs.postselect().circuit, configs.distill().circuit,
             configs.c5(14).circuit, configs.c5(16).circuit] + [w.circuit for w in configs.c4()[::7]]
    rng = np.random.default_rng(17)
    circs += [random_circuit(rng, int(rng.integers(3, 10)), int(rng.integers(30, 120))) for _ in range(60)]
    for c in circs:
        i = S.Program(c, components="on").info()
        if i["k_max"] == 0:
            continue
        assert i["product_selected"] == 1, (i["k_max"], i["product_merges"], i["product_vector_amplitudes"])


def test_compile_option_is_checked():
    c = _rotations([0.5])
    opts = S.symft_compile_opts(components=3)
    import ctypes as C
    arr, keep = S._marshal(c)
    h = C.c_void_p()
    rc = S._lib.symft_compile(c.n_qubits, arr, len(c.ops), C.cast(C.pointer(opts), C.c_void_p), C.byref(h))
    assert rc == -1  # SYMFT_EINVAL
