"""GPU parity of aggregate counts inside the batched work queue
(symft_sample_counts_batch; paper Sec. 6, detector postselection in the batch
sampler).

Every program's flags must equal the ones derived from the same batch's full
records (symft_sample_batch runs the same launch configuration, so a shot
kept in count mode has the records of the records launch), and its counts the
popcounts of its flags.  The pure-Clifford member, which runs outside the
queue, must also match the oracle bit for bit; active members' flags may
differ from the oracle's only in shots whose records do.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_28600_amd as S  # noqa: E402
from oracle import OracleCircuit  # noqa: E402
from oracle.counts import count_flags  # noqa: E402
from tests.randcirc import random_circuit  # noqa: E402
from workloads import configs  # noqa: E402
from workloads.surface import rotated_memory_z  # noqa: E402


def _popcount(a):
    return int(sum(bin(int(x)).count("1") for x in np.asarray(a, dtype=np.uint64).reshape(-1)))


def _members():
    """Active programs of several widths with detectors and observables, a member without detectors, and a
    pure-Clifford member (which runs as its own launch)."""
    circs = [rotated_memory_z(3, 3, 1e-3, coherent=0.3), rotated_memory_z(5, 3, 1e-3, coherent=0.1)]
    rng = np.random.default_rng(2024)
    while len(circs) < 6:
        c = random_circuit(rng, int(rng.integers(3, 7)), int(rng.integers(30, 60)))
        if c.num_detectors and c.num_observables:
            circs.append(c)
    circs.append(configs.c4()[7].circuit)   # no detectors: nothing discarded
    circs.append(configs.c1().circuit)      # pure Clifford
    return circs


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_counts_batch_matches_its_records_and_the_oracle(prec):
    circs = _members()
    progs = [S.Program(c) for c in circs]
    n = len(progs)
    shots = [64 * (2 + i % 4) + (13 * i) % 64 for i in range(n)]  # ragged last words
    seeds = [0xBA7C0 + 17 * i for i in range(n)]
    rng = np.random.default_rng(5)
    posts, exps = [], []
    for c in circs:
        nd, no = c.num_detectors, c.num_observables
        posts.append(sorted(set(rng.integers(0, nd, size=max(1, nd // 2)).tolist())) if nd else [])
        exps.append(rng.integers(0, 2, size=no).astype(np.uint8) if no else None)
    flags = [torch.full((2, (s + 63) // 64), -1, dtype=torch.int64, device="cuda") for s in shots]
    counts = torch.zeros(2 * n, dtype=torch.int64, device="cuda")
    print(f"counts batch: {n} programs, {prec}", flush=True)
    S.sample_counts_batch(progs, shots, seeds, posts, flags, counts, obs_expected=exps, precision=prec)
    outs = [torch.zeros((p.n_rows, (s + 63) // 64), dtype=torch.int64, device="cuda") for p, s in zip(progs, shots)]
    S.sample_batch(progs, shots, seeds, outs, precision=prec, graph=False)
    torch.cuda.synchronize()
    cnt = counts.cpu().numpy()
    for i, (c, p) in enumerate(zip(circs, progs)):
        got = S.bits_to_numpy(flags[i])
        rec = S.bits_to_numpy(outs[i])
        own, _ = count_flags(rec, c.num_records, c.num_detectors, c.num_observables, shots[i], posts[i], exps[i])
        assert np.array_equal(got, own), f"program {i}: flags differ from its batch records"
        assert list(cnt[2 * i:2 * i + 2]) == [_popcount(got[0]), _popcount(got[1])], f"program {i}: counts"
        oc = OracleCircuit(c)
        want_rows = oc.sample(seeds[i], shots[i])
        want, want_c = count_flags(want_rows, c.num_records, c.num_detectors, c.num_observables, shots[i],
                                   posts[i], exps[i])
        if p.k_max == 0:
            assert np.array_equal(got, want) and list(cnt[2 * i:2 * i + 2]) == list(want_c), f"program {i}"
        else:
            rdiff = np.bitwise_or.reduce(rec ^ want_rows, axis=0)
            fdiff = np.bitwise_or.reduce(got ^ want, axis=0)
            assert not np.any(fdiff & ~rdiff), f"program {i}: flags differ from the oracle where records agree"
    assert cnt[0] + cnt[2] > 0  # the coherent codes discard some shots


def test_counts_batch_graph_replays_add_and_offsets():
    """Graph replays give the same flags and add to the counters again; shot offsets select the same shots
    as single-program count launches at those offsets."""
    circs = _members()[:4]
    progs = [S.Program(c) for c in circs]
    n = len(progs)
    shots = [64 * 3 + 5 * i for i in range(n)]
    seeds = [0xC0DE + i for i in range(n)]
    offs = [64 * (7 * i) for i in range(n)]
    posts = [list(range(c.num_detectors)) for c in circs]
    flags = [torch.zeros((2, (s + 63) // 64), dtype=torch.int64, device="cuda") for s in shots]
    counts = torch.zeros(2 * n, dtype=torch.int64, device="cuda")
    first = None
    for rep in range(3):
        for f in flags:
            f.fill_(-1)                     # eager work between replays
        torch.cuda.synchronize()
        S.sample_counts_batch(progs, shots, seeds, posts, flags, counts, shot_offsets=offs, precision="fp64",
                              graph=True)
        torch.cuda.synchronize()
        got = [S.bits_to_numpy(f) for f in flags]
        if first is None:
            first = got
            once = counts.cpu().numpy().copy()
        for a, b in zip(first, got):
            assert np.array_equal(a, b), "graph replay differs"
    assert np.array_equal(counts.cpu().numpy(), 3 * once)
    for i, p in enumerate(progs):
        f1, c1 = p.sample_counts(shots[i], seeds[i], post=posts[i], shot_offset=offs[i], precision="fp64")
        # the single launch may choose another launch configuration: in FP64 that moves a branch probability by
        # rounding only, far below what would move a draw across its threshold
        assert np.array_equal(S.bits_to_numpy(f1), first[i]), f"program {i}: offset shots differ"
        assert list(c1.cpu().numpy()) == list(once[2 * i:2 * i + 2])
