"""Aggregate counts from full records (test infrastructure only).

The paper's detector postselection and aggregate-count interface (Sec. 6,
"Detector postselection" and the aggregate-count output of the GPU backend):
a shot is discarded when any postselected detector is 1; for every other
shot one logical-error flag records whether some observable differs from
its expected value; the two flags are summed into counters.  Early
termination of rejected shots is an optimisation that leaves both flags
unchanged, so the definition here starts from the complete records the
oracle samples (rows: records, then detectors, then observables; bit s % 64
of word s // 64 is shot s).
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np


def count_flags(rows: np.ndarray, n_rec: int, n_det: int, n_obs: int, shots: int,
                post: Sequence[int] = (), obs_expected: Optional[Sequence[int]] = None
                ) -> Tuple[np.ndarray, np.ndarray]:
    """Returns (flags [2, words] uint64: discarded, kept with a logical error; counts [2] int64)."""
    rows = np.asarray(rows, dtype=np.uint64)
    words = rows.shape[1]
    assert rows.shape[0] == n_rec + n_det + n_obs
    disc = np.zeros(words, dtype=np.uint64)
    for d in set(int(x) for x in post):
        if not 0 <= d < n_det:
            raise ValueError("detector index out of range")
        disc |= rows[n_rec + d]
    logic = np.zeros(words, dtype=np.uint64)
    for b in range(n_obs):
        want = np.uint64(0xFFFFFFFFFFFFFFFF) if (obs_expected is not None and obs_expected[b]) else np.uint64(0)
        logic |= rows[n_rec + n_det + b] ^ want
    logic &= ~disc
    # bits of shots past the end are 0
    mask = np.full(words, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    if words and shots % 64:
        mask[-1] = np.uint64((1 << (shots % 64)) - 1)
    if words * 64 > shots + (64 if shots % 64 else 0):
        raise ValueError("more words than shots")
    disc &= mask
    logic &= mask
    pop = lambda a: int(sum(bin(int(x)).count("1") for x in a))  # noqa: E731
    return np.stack([disc, logic]), np.array([pop(disc), pop(logic)], dtype=np.int64)
