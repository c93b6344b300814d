"""Pins of the oracle's noise and measurement draws (draw contract) by statistics.

* the exact-integer geometric table, element by element against a big-integer
  recomputation, and within g + 1 of 2^32 (1-p)^g;
* per-channel firing frequency vs P32 / 2^32 (binomial z-test) and branch
  frequencies (uniform D1/D2, weighted general channels: chi-square);
* per-detector marginals of a noisy surface code vs the exact value
  (1 - prod_i (1 - 2 q_i)) / 2 for independent channels, where q_i is the
  probability that channel i flips the detector, found by brute force: every
  branch Pauli is injected alone into the noiseless circuit;
* RandomMeas bits balanced; active-measurement uniforms uniform.
"""
import numpy as np
from scipy import stats

import oracle
from oracle import OracleCircuit
from workloads.circuit import Circuit, Op
from workloads.surface import rotated_memory_z


def _exact_table(p32: int):
    """Q[0] = 2^32, Q[g+1] = floor(Q[g] (2^32 - P32) / 2^32) in Python big integers."""
    q = [1 << 32]
    for _ in range(4096):
        q.append((q[-1] * ((1 << 32) - p32)) >> 32)
    return q


# P32 values of the workloads (p = 1e-3 surface codes and distillation, 5e-4
# near-Clifford circuits, readout flips 1e-2 and 2e-2, heavy noise 0.3) and the
# edges of the range: the smallest and largest P32 below 2^32, and 2^32 itself
# (a channel that always fires).
_P32S = [int(p * 2 ** 32) for p in (1e-3, 5e-4, 1e-2, 2e-2, 0.3, 0.05, 0.15, 0.09)] + [1, 2, (1 << 32) - 1, 1 << 32]


def test_gap_table_exact_integers():
    for p32 in _P32S:
        got = [int(v) for v in oracle.gap_table(p32)]
        want = _exact_table(p32)
        assert got == want, p32


def test_gap_table_closed_form():
    # the integer table stays within one unit per step of 2^32 q^g, q = 1 - P32/2^32
    for p32 in _P32S:
        Q = oracle.gap_table(p32).astype(np.float64)
        assert Q[0] == 2 ** 32
        assert Q[1] == 2 ** 32 - p32
        assert np.all(np.diff(Q) <= 0)
        g = np.arange(0, 4097)
        want = 2.0 ** 32 * (1 - p32 / 2 ** 32) ** g
        assert np.all(np.abs(Q - want) <= g + 1)


def _noise_circuit():
    c = Circuit(4)
    c.append("X_ERROR", [0, 1], arg=0.05)
    c.append("DEPOLARIZE1", [2, 3], arg=0.09)
    c.append("DEPOLARIZE2", [0, 1, 2, 3], arg=0.15)
    c.ops.append(Op("PAULI_CHANNEL", (0, 3), branches=((0.01, "XI"), (0.05, "ZZ"), (0.04, "IY"))))
    c.append("X_ERROR", [2], arg=0.05)   # same class as the first op's channels
    return c


def test_firing_and_branch_frequencies():
    c = _noise_circuit()
    oc = OracleCircuit(c)
    cls, rank, p32 = oc.channel_info()
    words = 3000
    counts, br = oc.noise_counts(12345, 0, words)
    trials = words * 64
    for ch in range(oc.n_chan):
        p = float(p32[ch]) / 2 ** 32
        z = (counts[ch] - trials * p) / np.sqrt(trials * p * (1 - p))
        assert abs(z) < 5, (ch, counts[ch], trials * p)
    # D1 channels 2,3: three equal branches; D2 channels 4,5: fifteen
    for ch, J in ((2, 3), (3, 3), (4, 15), (5, 15)):
        obs = br[ch, :J].astype(float)
        assert stats.chisquare(obs).pvalue > 1e-4
    # general channel 6: branch weights 0.01 : 0.05 : 0.04
    obs = br[6, :3].astype(float)
    exp = np.array([0.1, 0.5, 0.4]) * obs.sum()
    assert stats.chisquare(obs, exp).pvalue > 1e-4
    # class structure: equal P32 shares a class, ranked in circuit order
    assert cls[0] == cls[1] == cls[7] and rank[7] == 2
    assert len(set(cls.tolist())) == 4


def _inject(circ, target_channel, letters):
    """The circuit with every noise op removed except one channel, replaced by a
    probability-1 Pauli on its qubits."""
    out = Circuit(circ.n_qubits)
    ch = 0
    for o in circ.ops:
        if o.name in ("X_ERROR", "DEPOLARIZE1", "DEPOLARIZE2"):
            step = 2 if o.name == "DEPOLARIZE2" else 1
            for i in range(0, len(o.targets), step):
                if ch == target_channel:
                    qs = tuple(o.targets[i:i + step])
                    out.ops.append(Op("PAULI_CHANNEL", qs, branches=((1.0, letters),)))
                ch += 1
        else:
            out.ops.append(o)
    return out


def test_detector_marginals_exact():
    p = 1e-2
    c = rotated_memory_z(3, 2, p)
    oc = OracleCircuit(c)
    n_rec, n_det = c.num_records, c.num_detectors
    # flip sets by injection
    chans = []
    for o in c.ops:
        if o.name == "X_ERROR":
            chans += [(p, ("X",))] * len(o.targets)
        elif o.name == "DEPOLARIZE1":
            chans += [(p / 3, ("X", "Y", "Z"))] * len(o.targets)
        elif o.name == "DEPOLARIZE2":
            br = tuple(a + b for a in "IXYZ" for b in "IXYZ" if a + b != "II")
            chans += [(p / 15, br)] * (len(o.targets) // 2)
    q = np.zeros((len(chans), n_det))
    for i, (pb, letters) in enumerate(chans):
        for L in letters:
            out = OracleCircuit(_inject(c, i, L)).sample(1, 64)
            flips = (out[n_rec:n_rec + n_det, 0] & np.uint64(1)).astype(bool)
            q[i] += pb * flips
    exact = (1 - np.prod(1 - 2 * q, axis=0)) / 2
    shots = 64 * 2500
    recs = oc.sample(2024, shots, threads=8)
    det = recs[n_rec:n_rec + n_det]
    ones = np.array([sum(bin(int(w)).count("1") for w in row) for row in det])
    freq = ones / shots
    z = (freq - exact) / np.sqrt(exact * (1 - exact) / shots)
    assert np.all(np.abs(z) < 5), (freq, exact)
    assert exact.min() > 0.005


def test_random_measurement_and_uniform_draws():
    bits = [oracle.rmeas_bit(77, t, s) for t in range(8) for s in range(512)]
    assert abs(np.mean(bits) - 0.5) < 5 * 0.5 / np.sqrt(len(bits))
    u = np.array([oracle.active_u(77, t, s) for t in range(4) for s in range(2000)])
    assert u.min() >= 0 and u.max() < 1
    assert stats.kstest(u, "uniform").pvalue > 1e-4
