"""Helpers for GPU-vs-oracle parity (test harness only)."""
from __future__ import annotations

import numpy as np

import oracle as O


def meas_rows(circ):
    """Row of every measurement (-1 for the unrecorded ones inside resets)."""
    rows = []
    r = 0
    for o in circ.ops:
        if o.name in ("R", "M", "MR"):
            for _ in o.targets:
                if o.name == "R":
                    rows.append(-1)
                else:
                    rows.append(r)
                    r += 1
        elif o.name == "MPP":
            rows.append(r)
            r += 1
    return np.asarray(rows, dtype=np.int64)


def shot_bits(arr, col, lane):
    return ((arr[:, col] >> np.uint64(lane)) & np.uint64(1)).astype(np.uint8)


def compare_records(got, want, circ, oc, seed, shot_base, tol):
    """Bit-exact comparison of [rows, words] arrays for shots shot_base + 64*col + lane.

    A shot may differ only if one of its active-measurement draws lies within
    `tol` of the oracle's Pr(m=0); records of measurements before that draw
    must still agree.  Returns the number of such excluded shots."""
    assert got.shape == want.shape, (got.shape, want.shape)
    diff = np.flatnonzero((got != want).any(axis=0))
    if diff.size == 0:
        return 0
    rows_of = meas_rows(circ)
    excluded = 0
    for col in diff:
        x = got[:, col] ^ want[:, col]
        for lane in range(64):
            if not np.any((x >> np.uint64(lane)) & np.uint64(1)):
                continue
            shot = shot_base + 64 * int(col) + lane
            tr = oc.trace(seed, shot)
            act = np.flatnonzero(tr["meas_kind"] >= 2)
            close = [t for t in act if abs(O.active_u(seed, int(t), shot) - tr["p0"][t]) < tol]
            assert close, f"shot {shot} differs from the oracle with no draw near a threshold"
            t0 = min(close)
            g = shot_bits(got, col, lane)
            w = shot_bits(want, col, lane)
            early = [r for t, r in enumerate(rows_of) if r >= 0 and t < t0]
            assert np.array_equal(g[early], w[early]), f"shot {shot}: records before the tied draw differ"
            excluded += 1
    return excluded
