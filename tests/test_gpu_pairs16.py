"""The packed int16 pairwise fill (two pairs per wavefront segment, values
held with a per-pair bias) and its checkpoint walk, against the oracle:

- pairs that leave the exact int16 range go to the int32 kernels and carry
  DSA_ST_INT32, the others status 0: local pairs whose best score passes the
  limit (found while filling), global and semi-global pairs whose query's sum
  of row maxima passes it (found before filling), alone or beside a pair of
  the other kind in the same segment;
- an odd number of pairs per segment width (a segment with one pair);
- pairs of very different target lengths sharing a segment;
- every result equals the int32 path's (DSA_PAIR_INT32=1);
- the value frame at its limits: a gap extension that puts the score table
  at the top of int8, one past it, and one that leaves the frame little room.
"""
import numpy as np
import pytest

import oracle
from gpu_util import log
from test_gpu_pairs import compare_pairs, gpu_pairs
from workloads import gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu


def _wavefront(monkeypatch):
    monkeypatch.setenv("DSA_PAIR_WF_ROWS", "1")
    monkeypatch.setenv("DSA_PAIR_WF_CELLS", "0")


def _mixed_range_case(seed):
    """Pairs near the top of the int16 range and ordinary ones, interleaved
    so that segments hold one of each, both or neither."""
    rng = np.random.default_rng([170101575, seed])
    W = 17  # W in the BLOSUM62 code order of the workloads (score 11 against itself)
    qs, ts = [], []
    for k in range(24):
        kind = k % 4
        if kind == 0:    # identical W runs: scores 11 per residue
            L = int(rng.integers(2900, 3400))
            a = np.full(L, W, np.uint8)
            qs.append(a)
            ts.append(a.copy())
        elif kind == 1:  # related protein pair of similar length
            q, t = gen.related_pairs(int(rng.integers(1 << 30)), 1, 800, 1400)
            qs.append(q[0])
            ts.append(t[0])
        elif kind == 2:  # W run against a shorter copy inside random residues
            L = int(rng.integers(2000, 2600))
            a = np.full(L, W, np.uint8)
            t = np.concatenate([gen.background_residues(rng, 300), a[:L - 50], gen.background_residues(rng, 200)])
            qs.append(a)
            ts.append(t.astype(np.uint8))
        else:            # random pair
            qs.append(gen.background_residues(rng, int(rng.integers(500, 1500))))
            ts.append(gen.background_residues(rng, int(rng.integers(100, 3000))))
    return SeqSet.from_list(qs), SeqSet.from_list(ts)


@pytest.mark.parametrize("mode", ["local", "global", "semiglobal"])
def test_range_reruns_and_status(mode, blosum, monkeypatch):
    _wavefront(monkeypatch)
    assert blosum[17, 17] == 11
    Q, T = _mixed_range_case(300)
    log(f"pairs16 range {mode} n={len(Q)}")
    got = gpu_pairs(Q, T, blosum, 10, 1, mode, traceback=True)
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode=mode, traceback=True)
    compare_pairs(got, exp, True, f"range {mode}")
    st = got["status"][:len(Q)]
    # identical W runs of 2,900+ residues score above 31,000: never exact in int16
    big = np.array([k % 4 == 0 for k in range(len(Q))])
    assert ((st[big] & 1) == 1).all(), st[big]
    # ordinary pairs stay in the packed fill
    small = np.array([k % 4 in (1, 3) for k in range(len(Q))])
    assert ((st[small] & 1) == 0).all(), st[small]


@pytest.mark.parametrize("mode,ends", [("local", None), ("global", None), ("semiglobal", None),
                                       ("semiglobal", 2 | 8), ("semiglobal", 1 | 2 | 4 | 8)])
@pytest.mark.parametrize("traceback", [True, False], ids=["tb", "score"])
def test_equals_int32_path(mode, ends, traceback, blosum, monkeypatch):
    """The packed fill and the int32 kernels give the same results on pairs
    of very different shapes sharing segments (odd counts per width)."""
    _wavefront(monkeypatch)
    rng = np.random.default_rng([170101575, 301])
    qs, ts = [], []
    for L in [1, 16, 17, 63, 65, 129, 300, 513, 1025, 1100, 2049]:
        for n in [0, 1, 40, 700, 2500]:
            qs.append(gen.background_residues(rng, L))
            ts.append(gen.background_residues(rng, n))
    Q, T = SeqSet.from_list(qs), SeqSet.from_list(ts)
    log(f"pairs16 vs int32 {mode}/{ends} tb={traceback} n={len(Q)}")
    a = gpu_pairs(Q, T, blosum, 11, 1, mode, ends, traceback)
    monkeypatch.setenv("DSA_PAIR_INT32", "1")
    b = gpu_pairs(Q, T, blosum, 11, 1, mode, ends, traceback)
    n = len(Q)
    for f in ("score", "q_end", "t_end") + (("q_begin", "t_begin") if traceback else ()):
        assert (a[f][:n] == b[f][:n]).all(), f
    if traceback:
        for k in range(n):
            assert (a["cigars"][k] == b["cigars"][k]).all(), k
    exp = oracle.align_pairs(Q, T, blosum, 11, 1, mode=mode, ends=ends, traceback=traceback)
    compare_pairs(a, exp, traceback, f"packed {mode}/{ends}")


@pytest.mark.parametrize("mode", ["local", "global"])
def test_dna_reads(mode, dna, monkeypatch):
    """Reads against windows (a 5-letter alphabet with N) under the default
    routing: short reads in lane groups, longer ones in the packed fill."""
    monkeypatch.setenv("DSA_PAIR_WF_ROWS", "64")
    monkeypatch.setenv("DSA_PAIR_WF_CELLS", "0")
    c = gen.cfg3(n_pairs=900)
    Q, T = c["queries"], c["targets"]
    got = gpu_pairs(Q, T, c["matrix"], c["gap_open"], c["gap_extend"], mode)
    exp = oracle.align_pairs(Q, T, c["matrix"], c["gap_open"], c["gap_extend"], mode=mode, traceback=True)
    compare_pairs(got, exp, True, f"dna {mode}")
    assert ((got["status"][:len(Q)] & 1) == 0).all()


@pytest.mark.parametrize("mode,ends", [("local", None), ("global", None), ("semiglobal", None),
                                       ("semiglobal", 2 | 8)])
@pytest.mark.parametrize("o,e", [(60, 58), (70, 59), (120, 100)], ids=["e58", "e59", "e100"])
def test_frame_limits(mode, ends, o, e, blosum, monkeypatch):
    """The fill holds values in a frame that grows by e per row and column,
    and its int8 score table carries s + 2e (local s + e).  With the largest
    BLOSUM62 score 11, e = 58 puts s + 2e exactly at 127 (the table's
    limit), e = 59 past it (global and semi-global pairs then run int32),
    and e = 100 leaves only short pairs room for the frame.  Every result
    must equal the oracle's, whichever kernel took the pair."""
    _wavefront(monkeypatch)
    rng = np.random.default_rng([170101575, 302, e])
    qs, ts = [], []
    for L, n in [(48, 60), (100, 90), (130, 200), (257, 250), (400, 380)]:
        q, t = gen.related_pairs(int(rng.integers(1 << 30)), 1, L, L)
        qs.append(q[0])
        ts.append(t[0][:n] if len(t[0]) >= n else np.concatenate([t[0], gen.background_residues(rng, n - len(t[0]))]))
        qs.append(gen.background_residues(rng, L))
        ts.append(gen.background_residues(rng, n))
    Q, T = SeqSet.from_list(qs), SeqSet.from_list([x.astype(np.uint8) for x in ts])
    log(f"pairs16 frame limits {mode}/{ends} o={o} e={e} n={len(Q)}")
    got = gpu_pairs(Q, T, blosum, o, e, mode, ends, traceback=True)
    exp = oracle.align_pairs(Q, T, blosum, o, e, mode=mode, ends=ends, traceback=True)
    compare_pairs(got, exp, True, f"frame limits {mode}/{ends} e={e}")
