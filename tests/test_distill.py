"""The 15-to-1 distillation workload (textbook [[15,1,3]] Reed-Muller code),
pinned on the CPU by facts of the code rather than by the oracle itself.

* The checks: X checks are the [15,11] Hamming parity checks; X and Z checks
  commute; logical X^15 and Z^15 commute with every check and anticommute
  with each other.
* Without noise every detector and the logical observable are 0 (so the
  transversal R_Z(pi/4)^15 acts as the logical R_Zbar(-pi/4)).
* With independent Z errors of probability p, an error pattern is undetected
  iff it is a Hamming codeword, and flips the logical X iff its weight is odd.
  So Pr(kept) = sum over codewords c of p^|c| (1-p)^(15-|c|), and Pr(kept and
  logical error) the same sum over odd-weight codewords; the codewords are
  enumerated by brute force over 2^15 patterns.  The oracle's rates must
  agree within 5 sigma.
* The planner's width trajectory equals the oracle's (peak width 5).
"""
import numpy as np
import pytest

import paper_2607_28600_amd as S
from oracle import OracleCircuit
from oracle.counts import count_flags
from workloads.distill import N, distill_15to1, x_checks, z_checks


def _mask(rows):
    return [sum(1 << q for q in r) for r in rows]


def test_checks_form_the_reed_muller_code():
    xs, zs = _mask(x_checks()), _mask(z_checks())
    assert len(xs) == 4 and len(zs) == 10
    for q in range(N):  # column q of the X checks is the binary form of q + 1
        assert sum(((x >> q) & 1) << b for b, x in enumerate(xs)) == q + 1
    for x in xs:
        for z in zs:
            assert bin(x & z).count("1") % 2 == 0
    full = (1 << N) - 1
    for r in xs + zs:
        assert bin(full & r).count("1") % 2 == 0
    assert bin(full & full).count("1") % 2 == 1
    # the Z checks are independent (rank 10 over GF(2))
    basis = []
    for z in zs:
        for b in basis:
            z = min(z, z ^ b)
        assert z
        basis.append(z)


def test_noiseless_detectors_and_observable_are_zero():
    for z_only in (False, True):
        c = distill_15to1(0.0, z_only=z_only)
        out = OracleCircuit(c).sample(7, 64 * 16)
        assert not np.any(out[c.num_records:])


def test_z_noise_rates_match_the_hamming_code():
    p = 0.1
    xs = _mask(x_checks())
    keep = logic = 0.0
    for e in range(1 << N):
        if all(bin(e & x).count("1") % 2 == 0 for x in xs):
            w = bin(e).count("1")
            pr = p ** w * (1 - p) ** (N - w)
            keep += pr
            if w % 2:
                logic += pr
    c = distill_15to1(p, z_only=True)
    shots = 64 * 2000
    rows = OracleCircuit(c).sample(11, shots, threads=4)
    flags, counts = count_flags(rows, c.num_records, c.num_detectors, c.num_observables, shots,
                                list(range(c.num_detectors)), None)
    kept = shots - int(counts[0])
    for got, want in ((kept, keep), (int(counts[1]), logic)):
        sd = np.sqrt(shots * want * (1 - want))
        assert abs(got - shots * want) < 5 * sd + 1, (got, shots * want)


def test_planner_width_matches_oracle():
    c = distill_15to1(1e-3)
    p = S.Program(c)
    assert p.k_max == 5
    assert np.array_equal(p.plan()["k"], OracleCircuit(c).k_trajectory())
