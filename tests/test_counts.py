"""Aggregate counts (paper Sec. 6: detector postselection and the per-shot
discarded / logical-error flags): pins of the oracle's definition, and the
C-ABI entry point's argument checks that need no GPU."""
import os

import numpy as np

from oracle import OracleCircuit
from oracle.counts import count_flags
from workloads.circuit import Circuit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    shots, rows, cases = 0, None, []
    with open(os.path.join(GOLDEN, "count_flags_example.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "shots":
                shots = int(t[1])
            elif t[0] == "rows":
                rows = np.array([[int(x, 16)] for x in t[1:]], dtype=np.uint64)
            elif t[0] == "case":
                post = [] if t[2] == "-" else [int(x) for x in t[2].split(",")]
                exp = [int(c) for c in t[3]]
                cases.append((t[1], post, exp, int(t[4], 16), int(t[5], 16), int(t[6]), int(t[7])))
    return shots, rows, cases


def test_count_flags_hand_worked_example():
    shots, rows, cases = _golden()
    assert len(cases) == 3
    for name, post, exp, d, l, nd, nl in cases:
        flags, counts = count_flags(rows, 2, 2, 2, shots, post, exp)
        assert int(flags[0, 0]) == d, name
        assert int(flags[1, 0]) == l, name
        assert list(counts) == [nd, nl], name


def test_count_flags_closed_form_rates():
    """Independent X errors: Pr(discard) = p1 and Pr(kept with a logical error) = (1 - p1) p2."""
    p1, p2, shots = 0.2, 0.1, 1 << 14
    c = Circuit(2)
    c.append("X_ERROR", [0], arg=p1)
    c.append("X_ERROR", [1], arg=p2)
    c.append("M", [0, 1])
    c.detector([0])
    c.observable(0, [1])
    rows = OracleCircuit(c).sample(0x5EED00C0, shots)
    flags, counts = count_flags(rows, 2, 1, 1, shots, [0])
    for got, want in ((counts[0] / shots, p1), (counts[1] / shots, (1 - p1) * p2)):
        sd = np.sqrt(want * (1 - want) / shots)
        assert abs(got - want) < 5 * sd, (got, want)
    # the flags of a shot are the detector / observable bits themselves here
    assert np.array_equal(flags[0], rows[2])
    assert np.array_equal(flags[1], rows[3] & ~rows[2])


def test_count_flags_masks_ragged_tail():
    rows = np.full((3, 2), np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    flags, counts = count_flags(rows, 1, 1, 1, 70, [], [0])
    assert int(flags[1, 1]) == (1 << 6) - 1
    assert list(counts) == [0, 70]


def test_sample_counts_rejects_bad_arguments_before_any_gpu_work():
    import pytest

    import paper_2607_28600_amd as S
    c = Circuit(1)
    c.append("M", [0])
    c.detector([0])
    c.observable(0, [0])
    p = S.Program(c)
    with pytest.raises(S.SymftError) as e:
        p.sample_counts_into(None, None, 64, 1, post=[1], stream=0)
    assert e.value.code == -1
    with pytest.raises(S.SymftError) as e:
        p.sample_counts_into(None, None, 64, 1, post=[0], obs_expected=[2], stream=0)
    assert e.value.code == -1
    with pytest.raises(S.SymftError) as e:
        p.sample_counts_into(None, None, 64, 1, post=[0], shot_offset=32, stream=0)
    assert e.value.code == -1
    for bad in (3, 2, 2048):
        with pytest.raises(S.SymftError) as e:
            p.sample_counts_into(None, None, 64, 1, post=[0], stream=0, threads_per_shot=bad)
        assert e.value.code == -1
