"""GPU parity of per-query top-K database search (Section II.B.2) against a
full sort of the oracle's per-target results, with and without traceback of
the hits."""
import numpy as np
import pytest

import oracle
from gpu_util import log
from workloads import gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu


def run_topk(Q, T, S, o, e, K, mode="local", traceback=False, ends=None):
    import torch
    import paper_1701_01575_amd as dsa
    db = dsa.Database.from_seqset(T, S.shape[0])
    r = dsa.align(Q, db=db, matrix=S, gap_open=o, gap_extend=e, mode=mode, free_ends=ends,
                  top_k=K, traceback=traceback)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items() if hasattr(v, "cpu") and k != "cigar_ops"}
    if traceback:
        out["cigars"] = dsa.cigars(r)
    return out


def expected_topk(Q, T, S, o, e, K, mode, ends=None):
    full = oracle.search(Q, T, S, o, e, mode=mode, ends=ends)
    nq, nt = len(Q), len(T)
    sc = full["score"].reshape(nq, nt)
    hits = []
    for q in range(nq):
        idx = oracle.top_k(sc[q], K, positive_only=(mode == "local"))
        hits.append(list(idx) + [-1] * (K - len(idx)))
    return full, np.array(hits, dtype=np.int64)


@pytest.mark.parametrize("mode", ["local", "global", "semiglobal"])
@pytest.mark.parametrize("traceback", [False, True], ids=["score", "tb"])
def test_topk_parity(mode, traceback, blosum):
    c = gen.cfg2(n_targets=1500, query_lengths=(30, 144, 700))
    Q, T = c["queries"], c["targets"]
    K = 10
    log(f"top-k mode={mode} tb={traceback}")
    got = run_topk(Q, T, blosum, 11, 1, K, mode, traceback)
    full, hits = expected_topk(Q, T, blosum, 11, 1, K, mode)
    nq, nt = len(Q), len(T)
    assert (got["t_index"].reshape(nq, K) == hits).all()
    for q in range(nq):
        for k in range(K):
            t = hits[q, k]
            oi = q * K + k
            if t < 0:
                assert got["score"][oi] == 0
                continue
            fi = q * nt + t
            assert got["score"][oi] == full["score"][fi]
            assert got["q_end"][oi] == full["q_end"][fi] and got["t_end"][oi] == full["t_end"][fi]
    if traceback:
        valid = hits.reshape(-1) >= 0
        qi = np.repeat(np.arange(nq), K)[valid]
        ti = hits.reshape(-1)[valid]
        exp = oracle.align_index(qi, ti, Q, T, blosum, 11, 1, mode=mode, traceback=True)
        pos = np.nonzero(valid)[0]
        for j, oi in enumerate(pos):
            assert got["q_begin"][oi] == exp["q_begin"][j] and got["t_begin"][oi] == exp["t_begin"][j]
            assert (got["cigars"][oi] == exp["cigars"][j]).all(), (oi, oracle.cigar_string(got["cigars"][oi]),
                                                                 oracle.cigar_string(exp["cigars"][j]))


def test_topk_fewer_hits_than_k(dna):
    rng = np.random.default_rng([170101575, 70])
    T = SeqSet.from_list([np.full(20, 3, np.uint8), rng.integers(0, 4, 30).astype(np.uint8),
                          np.zeros(0, np.uint8), np.full(5, 0, np.uint8)])
    Q = SeqSet.from_list([np.full(12, 2, np.uint8), rng.integers(0, 4, 25).astype(np.uint8)])
    got = run_topk(Q, T, dna, 5, 2, 6, "local", traceback=True)
    full, hits = expected_topk(Q, T, dna, 5, 2, 6, "local")
    assert (got["t_index"].reshape(2, 6) == hits).all()
    assert (got["t_index"] == -1).any()


def test_topk_free_query_end_traceback(blosum):
    """Top-K of a semi-global search with free query and target ends, the
    hits traced: the search and the hit traceback both run int32 kernels."""
    c = gen.cfg2(n_targets=800, query_lengths=(40, 300))
    Q, T = c["queries"], c["targets"]
    K, ends = 6, 2 | 8
    got = run_topk(Q, T, blosum, 11, 1, K, "semiglobal", traceback=True, ends=ends)
    full, hits = expected_topk(Q, T, blosum, 11, 1, K, "semiglobal", ends=ends)
    nq, nt = len(Q), len(T)
    assert (got["t_index"].reshape(nq, K) == hits).all()
    qi = np.repeat(np.arange(nq), K)
    ti = hits.reshape(-1)
    exp = oracle.align_index(qi, ti, Q, T, blosum, 11, 1, mode="semiglobal", ends=ends, traceback=True)
    for f in ("score", "q_begin", "q_end", "t_begin", "t_end"):
        assert (got[f] == np.asarray(exp[f])).all(), f
    for k in range(len(qi)):
        assert (got["cigars"][k] == exp["cigars"][k]).all(), k



def test_cfg5_full_size_topk_sampled(blosum):
    """Top-10 with traceback against the full 500,000-target serving database
    (the benchmark's serving configuration), checked by properties that hold
    at any size: every hit is recomputed by the oracle (score, ends, begins,
    CIGAR), and no sampled non-hit beats the tenth hit under the (score
    descending, index ascending) order."""
    c = gen.cfg5_db()
    T = c["targets"]
    rng = np.random.default_rng([170101575, 61])
    Q = SeqSet.from_list([gen.background_residues(rng, L) for L in (60, 400, 1500)])
    K = 10
    log("cfg5 full size: 3 queries x 500,000 targets, top-10 with traceback")
    got = run_topk(Q, T, blosum, 11, 1, K, "local", traceback=True)
    nq, nt = len(Q), len(T)
    hits = got["t_index"].reshape(nq, K)
    assert (hits >= 0).all()
    qi = np.repeat(np.arange(nq), K)
    exp = oracle.align_index(qi, hits.reshape(-1), Q, T, blosum, 11, 1, mode="local", traceback=True)
    for f in ("score", "q_end", "t_end", "q_begin", "t_begin"):
        assert (got[f] == exp[f]).all(), f
    for oi in range(nq * K):
        assert (got["cigars"][oi] == exp["cigars"][oi]).all(), oi
    sc = got["score"].reshape(nq, K)
    for q in range(nq):
        assert (np.diff(sc[q]) <= 0).all()
        others = np.setdiff1d(rng.integers(0, nt, size=3000), hits[q])
        o = oracle.align_index(np.full(len(others), q), others, Q, T, blosum, 11, 1, mode="local")
        worst, worst_t = int(sc[q, -1]), int(hits[q, -1])
        assert (o["score"] <= worst).all()
        assert not ((o["score"] == worst) & (others < worst_t)).any()
