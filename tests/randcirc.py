"""Seeded random small circuits for the tests (no method arithmetic)."""
import numpy as np

from workloads.circuit import Circuit


def random_circuit(rng, n, length, p_noise=0.3, allow_reset=True, p_flip=0.0):
    # p_flip > 0: every M / MR / MPP gets a readout flip of probability p_flip
    # (no extra draws otherwise, so the circuits of a seed stay as they were)
    c = Circuit(n)
    for _ in range(length):
        r = rng.random()
        if r < 0.25:
            c.append(str(rng.choice(["H", "S", "S_DAG", "X", "Y", "Z"])), [int(rng.integers(n))])
        elif r < 0.4 and n >= 2:
            a, b = rng.choice(n, 2, replace=False)
            c.append(str(rng.choice(["CX", "CZ", "SWAP"])), [int(a), int(b)])
        elif r < 0.55:
            w = int(rng.integers(1, min(n, 4) + 1))
            qs = rng.choice(n, w, replace=False)
            c.rot([(int(q), str(rng.choice(list("XYZ")))) for q in qs], float(rng.uniform(-np.pi, np.pi)),
                  negate=bool(rng.random() < 0.3))
        elif r < 0.72:
            w = int(rng.integers(1, min(n, 4) + 1))
            qs = rng.choice(n, w, replace=False)
            c.mpp([(int(q), str(rng.choice(list("XYZ")))) for q in qs], negate=bool(rng.random() < 0.3),
                  p_flip=p_flip)
            if rng.random() < 0.5:
                qs2 = rng.choice(n, int(rng.integers(1, min(n, 2) + 1)), replace=False)
                nr = c.num_records
                recs = sorted(set(int(x) for x in rng.choice(nr, int(rng.integers(1, min(nr, 2) + 1)), replace=False)))
                c.feedback([(int(q), str(rng.choice(list("XYZ")))) for q in qs2], recs)
        elif r < 0.8:
            names = ["M", "MR", "R"] if allow_reset else ["M"]
            nm = str(rng.choice(names))
            c.append(nm, [int(rng.integers(n))], arg=p_flip if nm != "R" else 0.0)
        elif r < 0.9:
            c.append("DEPOLARIZE1", [int(rng.integers(n))], arg=p_noise)
        elif r < 0.95 and n >= 2:
            a, b = rng.choice(n, 2, replace=False)
            c.append("DEPOLARIZE2", [int(a), int(b)], arg=p_noise)
        else:
            c.append("X_ERROR", [int(rng.integers(n))], arg=p_noise)
    if c.num_records >= 2 and rng.random() < 0.7:
        c.detector([0, c.num_records - 1])
    if c.num_records >= 1:
        c.observable(0, [c.num_records - 1])
    return c


def wide_circuit(k, seed, p_noise=2e-2, p_flip=1e-2):
    """A state of peak active width k + 2 on k + 4 qubits: |+>^n, a Z rotation
    on each of the first k qubits (one promotion each), then twelve rounds of a
    CNOT, depolarizing noise and a weight-3 rotation anywhere (two more
    promotions, pair and diagonal rotations), then an X measurement of every
    qubit with readout flips (active-diagonal measurements down to width 0)."""
    rng = np.random.default_rng(seed)
    n = k + 4
    c = Circuit(n)
    c.append("H", list(range(n)))
    for q in range(k):
        c.rot([(q, "Z")], float(rng.uniform(0.2, 1.2)))
    for _ in range(12):
        a, b = (int(v) for v in rng.choice(k, 2, replace=False))
        c.append("CX", [a, b])
        c.append("DEPOLARIZE1", [a, b], arg=p_noise)
        qs = rng.choice(n, 3, replace=False)
        c.rot([(int(q), "XYZ"[int(rng.integers(3))]) for q in qs], float(rng.uniform(-1, 1)))
    for q in range(n):
        c.mpp([(q, "X")], p_flip=p_flip)
    c.detector([0, 1])
    c.observable(0, [n - 1])
    return c
