"""GPU parity of pairwise alignment (query k vs target k) with and without
traceback against the CPU oracle: score, both begins, both ends and the CIGAR
must be identical.  Covers every mode, lengths around the 16-row strip
boundaries, empty sequences, code storage split into several chunks, a CIGAR
buffer that is too small, the hand-worked golden cases and reduced versions
of the read-mapping and global / semi-global workloads.  Large pairs go to
the wavefront kernel (one wave per pair); the routing thresholds are set
through DSA_PAIR_WF_ROWS / DSA_PAIR_WF_CELLS to send every pair down either
path."""
import numpy as np
import pytest

import oracle
from golden_cases import load as load_golden
from gpu_util import log
from workloads import gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu

CASES = [
    ("local", None), ("global", None), ("semiglobal", None),
    ("semiglobal", 1 | 4), ("semiglobal", 4), ("semiglobal", 8), ("semiglobal", 1 | 8),
]


def gpu_pairs(Q, T, S, o, e, mode, ends=None, traceback=True, **kw):
    import torch
    import paper_1701_01575_amd as dsa
    r = dsa.align(Q, targets=T, matrix=S, gap_open=o, gap_extend=e, mode=mode, free_ends=ends,
                  traceback=traceback, **kw)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items() if hasattr(v, "cpu") and k != "cigar_ops"}
    if traceback:
        out["cigars"] = dsa.cigars(r)
    out["capacity_ok"] = r["capacity_ok"]
    return out


def compare_pairs(got, exp, traceback=True, label=""):
    n = len(exp["score"])
    fields = ["score", "q_end", "t_end"] + (["q_begin", "t_begin"] if traceback else [])
    for f in fields:
        g = got[f][:n].astype(np.int64)
        x = np.asarray(exp[f]).astype(np.int64)
        bad = np.nonzero(g != x)[0]
        if len(bad):
            k = bad[0]
            raise AssertionError(f"{label} {f}: {len(bad)} mismatches; first pair {k}: gpu "
                                 f"{[int(got[x][k]) for x in fields]} oracle "
                                 f"{[int(exp[x][k]) for x in fields]}")
    if traceback:
        for k in range(n):
            a, b = got["cigars"][k], exp["cigars"][k]
            if len(a) != len(b) or (a != b).any():
                raise AssertionError(f"{label} cigar of pair {k}: gpu {oracle.cigar_string(a)} "
                                     f"oracle {oracle.cigar_string(b)}")


def _pairs(seed, n, lo, hi, alphabet, related=False):
    if related:
        return gen.related_pairs(seed, n, max(lo, 1), hi)
    return gen.random_pairs(seed, n, hi, alphabet, min_len=lo)


@pytest.mark.parametrize("mode,ends", CASES)
@pytest.mark.parametrize("traceback", [True, False], ids=["tb", "score"])
def test_pairs_protein(mode, ends, traceback, blosum):
    Q, T = _pairs(11, 300, 0, 90, 20)
    Q2, T2 = _pairs(12, 120, 30, 200, 20, related=True)
    Q = SeqSet.from_list([Q[k] for k in range(len(Q))] + [Q2[k] for k in range(len(Q2))])
    T = SeqSet.from_list([T[k] for k in range(len(T))] + [T2[k] for k in range(len(T2))])
    log(f"pairs protein mode={mode} ends={ends} tb={traceback} n={len(Q)}")
    got = gpu_pairs(Q, T, blosum, 10, 1, mode, ends, traceback)
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode=mode, ends=ends, traceback=traceback)
    compare_pairs(got, exp, traceback, f"protein {mode}/{ends}")


@pytest.mark.parametrize("mode,ends", CASES[:3])
def test_pairs_strip_edges(mode, ends, dna):
    lens = [0, 1, 2, 15, 16, 17, 31, 32, 33, 47, 48, 49]
    rng = np.random.default_rng([170101575, 60])
    qs, ts = [], []
    for a in lens:
        for b in lens:
            qs.append(rng.integers(0, 4, size=a).astype(np.uint8))
            ts.append(rng.integers(0, 5, size=b).astype(np.uint8))
    Q, T = SeqSet.from_list(qs), SeqSet.from_list(ts)
    got = gpu_pairs(Q, T, dna, 5, 2, mode, ends)
    exp = oracle.align_pairs(Q, T, dna, 5, 2, mode=mode, ends=ends, traceback=True)
    compare_pairs(got, exp, True, f"edges {mode}")


@pytest.mark.parametrize("mode,ends", CASES[:3] + [("semiglobal", 1 | 8)])
def test_pairs_plain(mode, ends, blosum):
    """The plain form (one launch per pair, input order) gives the batched results."""
    Q, T = _pairs(15, 90, 0, 140, 20)
    Q2, T2 = _pairs(16, 40, 30, 260, 20, related=True)
    Q = SeqSet.from_list([Q[k] for k in range(len(Q))] + [Q2[k] for k in range(len(Q2))])
    T = SeqSet.from_list([T[k] for k in range(len(T))] + [T2[k] for k in range(len(T2))])
    got = gpu_pairs(Q, T, blosum, 10, 1, mode, ends, plain=True)
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode=mode, ends=ends, traceback=True)
    compare_pairs(got, exp, True, f"plain {mode}/{ends}")
    got = gpu_pairs(Q, T, blosum, 10, 1, mode, ends, traceback=False, plain=True)
    compare_pairs(got, exp, False, f"plain score-only {mode}/{ends}")


def all_wavefront(monkeypatch):
    monkeypatch.setenv("DSA_PAIR_WF_ROWS", "1")
    monkeypatch.setenv("DSA_PAIR_WF_CELLS", "0")


def _edge_pairs(seed, alphabet, m_lens, n_lens):
    rng = np.random.default_rng([170101575, seed])
    qs, ts = [], []
    for a in m_lens:
        for b in n_lens:
            q = rng.integers(0, alphabet, size=a).astype(np.uint8)
            # half the targets share a stretch of the query so that scores are large
            t = rng.integers(0, alphabet, size=b).astype(np.uint8)
            if a and b and rng.random() < 0.5:
                k = min(a, b) // 2
                t[:k] = q[a - k:]
            qs.append(q)
            ts.append(t)
    return qs, ts


@pytest.mark.parametrize("mode,ends", CASES)
@pytest.mark.parametrize("traceback", [True, False], ids=["tb", "score"])
def test_pairs_wavefront(mode, ends, traceback, blosum, monkeypatch):
    """Every pair through the wavefront kernel: 4- to 64-lane segments
    (queries up to 64, 128, 256, 512 rows and beyond), segments of one wave with different
    target lengths, multi-pass pairs (over 1024 rows) and lengths at the
    16-row strip and segment edges."""
    all_wavefront(monkeypatch)
    Q, T = _pairs(17, 60, 0, 120, 20)
    Q2, T2 = _pairs(18, 16, 900, 2600, 20, related=True)
    eq, et = _edge_pairs(61, 20, [1, 15, 16, 17, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513,
                                  1023, 1024, 1025, 2049], [0, 1, 5, 300])
    Q = SeqSet.from_list([Q[k] for k in range(len(Q))] + [Q2[k] for k in range(len(Q2))] + eq)
    T = SeqSet.from_list([T[k] for k in range(len(T))] + [T2[k] for k in range(len(T2))] + et)
    log(f"pairs wavefront mode={mode} ends={ends} tb={traceback} n={len(Q)}")
    got = gpu_pairs(Q, T, blosum, 10, 1, mode, ends, traceback)
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode=mode, ends=ends, traceback=traceback)
    compare_pairs(got, exp, traceback, f"wavefront {mode}/{ends}")


@pytest.mark.parametrize("mode", ["local", "global", "semiglobal"])
def test_pairs_wavefront_chunked_plain(mode, blosum, monkeypatch):
    """Wavefront pairs with their codes split over many chunks, mixed with
    lane-group pairs (both kinds run concurrently), then the plain form."""
    monkeypatch.setenv("DSA_TB_BUDGET", str(1 << 20))
    monkeypatch.setenv("DSA_PAIR_WF_ROWS", "200")
    monkeypatch.setenv("DSA_PAIR_WF_CELLS", "40000")
    Q, T = _pairs(19, 120, 20, 700, 20, related=True)
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode=mode, traceback=True)
    got = gpu_pairs(Q, T, blosum, 10, 1, mode)
    compare_pairs(got, exp, True, f"wavefront chunked {mode}")
    got = gpu_pairs(Q, T, blosum, 10, 1, mode, plain=True)
    compare_pairs(got, exp, True, f"wavefront plain {mode}")


@pytest.mark.parametrize("mode", ["local", "global", "semiglobal"])
def test_pairs_longest(mode, blosum):
    """Pairs at the 65,532-residue maximum on either side: a 4,096-strip
    query (64 wavefront passes) and a 65,532-column target."""
    rng = np.random.default_rng([170101575, 62])
    a = gen.background_residues(rng, 65532)
    b = gen.background_residues(rng, 100)
    c = a[1000:1100].copy()
    Q = SeqSet.from_list([b, a, c])
    T = SeqSet.from_list([a, b, a])
    log(f"longest pairs {mode}")
    got = gpu_pairs(Q, T, blosum, 10, 1, mode)
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode=mode, traceback=True)
    compare_pairs(got, exp, True, f"longest {mode}")


@pytest.mark.parametrize("ends", [2, 2 | 8, 1 | 2, 2 | 4, 15])
@pytest.mark.parametrize("route", ["lanes", "wavefront"])
@pytest.mark.parametrize("traceback", [True, False], ids=["tb", "score"])
def test_pairs_free_query_end(ends, route, traceback, blosum, monkeypatch):
    """Semi-global with a free query end, through either pair kernel: the
    alignment may stop before the last query residue, or at row 0."""
    if route == "lanes":
        monkeypatch.setenv("DSA_PAIR_WF_ROWS", str(1 << 30))
    else:
        all_wavefront(monkeypatch)
    Q, T = _pairs(20, 80, 0, 150, 20)
    Q2, T2 = _pairs(21, 30, 50, 1200, 20, related=True)
    # queries whose tail matches nothing: the free end pays off
    rng = np.random.default_rng([170101575, 63])
    tails = [np.concatenate([T2[k][:60], np.full(40, 22, np.uint8)]) for k in range(10)]
    Q = SeqSet.from_list([Q[k] for k in range(len(Q))] + [Q2[k] for k in range(len(Q2))] + tails)
    T = SeqSet.from_list([T[k] for k in range(len(T))] + [T2[k] for k in range(len(T2))] +
                         [T2[k] for k in range(10)])
    log(f"pairs QE ends={ends} route={route} tb={traceback}")
    got = gpu_pairs(Q, T, blosum, 10, 1, "semiglobal", ends, traceback)
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode="semiglobal", ends=ends, traceback=traceback)
    compare_pairs(got, exp, traceback, f"QE {ends} {route}")
    assert (np.asarray(exp["q_end"]) < Q.lengths - 1).any()


def test_pairs_chunked_codes(blosum, monkeypatch):
    monkeypatch.setenv("DSA_TB_BUDGET", str(1 << 20))  # many chunks of direction codes
    Q, T = _pairs(13, 400, 20, 300, 20, related=True)
    got = gpu_pairs(Q, T, blosum, 10, 1, "global")
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode="global", traceback=True)
    compare_pairs(got, exp, True, "chunked")


def test_pairs_cigar_capacity_short(blosum):
    Q, T = _pairs(14, 50, 10, 60, 20, related=True)
    need = int((Q.lengths + T.lengths + 1).sum())
    got = gpu_pairs(Q, T, blosum, 10, 1, "local", cigar_capacity=need // 2)
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode="local", traceback=True)
    assert not got["capacity_ok"]
    assert (got["score"] == exp["score"]).all() and (got["q_end"] == exp["q_end"]).all()
    trunc = (got["status"] & 2) != 0
    assert trunc.any() and not trunc.all()
    for k in np.nonzero(~trunc)[0]:
        assert (got["cigars"][k] == exp["cigars"][k]).all()


def test_pairs_golden():
    cases = load_golden()
    for c in cases:
        got = gpu_pairs(SeqSet.from_list([c["query"]]), SeqSet.from_list([c["target"]]), c["S"],
                        c["o"], c["e"], c["mode"], c["ends"] or None)
        res = (int(got["score"][0]), int(got["q_begin"][0]), int(got["q_end"][0]),
               int(got["t_begin"][0]), int(got["t_end"][0]), oracle.cigar_string(got["cigars"][0]))
        assert res == (c["score"], c["q_begin"], c["q_end"], c["t_begin"], c["t_end"], c["cigar"]), c["name"]


def test_cfg3_reduced_full_parity():
    c = gen.cfg3(n_pairs=3000)
    log("cfg3 reduced: 3000 read / window pairs")
    got = gpu_pairs(c["queries"], c["targets"], c["matrix"], 5, 2, "local")
    exp = oracle.align_pairs(c["queries"], c["targets"], c["matrix"], 5, 2, mode="local", traceback=True)
    compare_pairs(got, exp, True, "cfg3")


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
def test_cfg4_reduced_full_parity(mode):
    c = gen.cfg4(n_pairs=300)
    log(f"cfg4 reduced {mode}: 300 pairs")
    got = gpu_pairs(c["queries"], c["targets"], c["matrix"], 10, 1, mode)
    exp = oracle.align_pairs(c["queries"], c["targets"], c["matrix"], 10, 1, mode=mode, traceback=True)
    compare_pairs(got, exp, True, f"cfg4 {mode}")
