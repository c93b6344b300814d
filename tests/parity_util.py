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


def frame_relation(a, b, tol):
    """Whether a_x = e^{i phi} (-1)^{s.x} b_{x XOR y} for some phase phi and bit
    vectors s, y (returned as (y, s), else None).  Two representations of one
    state on the same active coordinates differ by exactly such a map: a Pauli
    frame F = i^e Xbar^y Zbar^s' (times dormant factors) sends
    sum_x alpha_x Xbar^x |0bar> to i^e sum_x (-1)^{s'.x} alpha_x Xbar^(x XOR y) |0bar>,
    and sign conventions of the generators add further characters."""
    m = frame_match(a, b, tol)
    return None if m is None else m[:2]


def frame_match(a, b, tol):
    """As frame_relation, returning (y, s, err) with err the largest
    abs(a_x - e^{i phi} (-1)^{s.x} b_{x XOR y}) of the match, or None."""
    a = np.asarray(a, dtype=complex)
    b = np.asarray(b, dtype=complex)
    if a.shape != b.shape:
        return None
    N = a.size
    k = N.bit_length() - 1
    idx = np.arange(N)
    mag_a = np.abs(a)
    r = int(np.argmax(mag_a))
    # entries large enough for their sign to be read at this tolerance
    sig = mag_a > 100 * tol
    for y in range(N):
        bb = b[idx ^ y]
        if np.max(np.abs(mag_a - np.abs(bb))) > tol:
            continue
        ph = a[r] / bb[r]
        ph /= abs(ph)
        # the signs must be a character of x XOR r: solve s over GF(2), then check every entry
        xs = (idx[sig] ^ r).tolist()
        bits = ((a[sig] * np.conj(ph * bb[sig])).real < 0).astype(int).tolist()
        basis = {}  # pivot bit -> (row, rhs)
        ok = True
        for x, v in zip(xs, bits):
            for p in sorted(basis, reverse=True):
                if (x >> p) & 1:
                    x ^= basis[p][0]
                    v ^= basis[p][1]
            if x == 0:
                if v:
                    ok = False
                    break
                continue
            basis[x.bit_length() - 1] = (x, v)
        if not ok:
            continue
        s = 0
        for p in sorted(basis):
            row, v = basis[p]
            lower = row & ~(1 << p)
            par = bin(lower & s).count("1") & 1
            if v ^ par:
                s |= 1 << p
        chi = np.array([(-1) ** (bin(s & (x ^ r)).count("1") & 1) for x in range(N)])
        err = float(np.max(np.abs(a - ph * chi * bb)))
        if err <= tol:
            return y, s, err
    return None


def p0_error(p0_gpu, oc, seed, shots, tol):
    """Largest abs(P0_gpu - P0_oracle) over the active measurements of `shots`.

    p0_gpu[i, t] is the kernels' Pr(recorded bit = 0) of measurement t in
    shots[i].  Each shot is compared up to and including its first active draw
    within `tol` of the oracle's threshold: past that draw the two sides may
    take different branches, and their later probabilities need not agree.
    Returns (worst error, number of probabilities compared)."""
    worst, n = 0.0, 0
    for i, s in enumerate(shots):
        tr = oc.trace(seed, s)
        for t in np.flatnonzero(tr["meas_kind"] >= 2):
            worst = max(worst, abs(float(p0_gpu[i, t]) - float(tr["p0"][t])))
            n += 1
            if abs(O.active_u(seed, int(t), s) - tr["p0"][t]) < tol:
                break
    return worst, n
