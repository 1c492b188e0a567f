"""User-extensible scoring on the GPU against the oracle.  Random profiles
(one int8 row per query residue) in database search (every mode, the
batched and plain forms, int16 and forced int32, inter-sequence, wavefront
and strip-pipelined units, queries over 1,024 rows), top-K with the hits'
traceback, and pairwise alignment with traceback on both pair kernels; a
profile made of the matrix rows gives the matrix results.  Custom matrices
over 33 to 64 letters (the int32 kernels) in search, top-K with traceback
and pairwise alignment."""
import numpy as np
import pytest

import oracle
from gpu_util import compare_search, log
from workloads import gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu

ROUTES = [None, "wavefront", "pipelined"]


def _route(monkeypatch, route):
    if route is not None:
        monkeypatch.setenv("DSA_INTRA_BUDGET", "1")
        monkeypatch.setenv("DSA_KS_BUDGET", "0" if route == "wavefront" else str(1 << 40))


def _profile(rng, Q, A, lo=-6, hi=9):
    return rng.integers(lo, hi, size=(len(Q.codes), A)).astype(np.int8)


def _search(Q, T, S, o, e, mode, pssm, **kw):
    import torch
    import paper_1701_01575_amd as dsa
    db = dsa.Database.from_seqset(T, S.shape[0])
    r = dsa.align(Q, db=db, matrix=S, gap_open=o, gap_extend=e, mode=mode, pssm=pssm, **kw)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in r.items() if hasattr(v, "cpu")}
    db.close()
    return got


@pytest.mark.parametrize("route", ROUTES, ids=["inter", "wavefront", "pipelined"])
@pytest.mark.parametrize("mode", ["local", "global", "semiglobal"])
def test_search_random_profiles(mode, route, blosum, monkeypatch):
    _route(monkeypatch, route)
    rng = np.random.default_rng([170101575, 120])
    c = gen.cfg2(n_targets=900, query_lengths=(33, 300, 1100))
    Q, T = c["queries"], c["targets"]
    P = _profile(rng, Q, blosum.shape[0])
    log(f"pssm search {mode} route={route}")
    got = _search(Q, T, blosum, 11, 1, mode, P)
    exp = oracle.search(Q, T, blosum, 11, 1, mode=mode, pssm=P)
    compare_search(got, exp, len(Q), len(T), label=f"pssm {mode} {route}")


@pytest.mark.parametrize("form", ["plain", "int32"])
def test_search_profiles_plain_and_int32(form, blosum):
    rng = np.random.default_rng([170101575, 121])
    c = gen.cfg2(n_targets=700, query_lengths=(64, 500))
    Q, T = c["queries"], c["targets"]
    P = _profile(rng, Q, blosum.shape[0], -4, 12)
    kw = {"plain": True} if form == "plain" else {"force_int32": True}
    for mode in ("local", "global"):
        got = _search(Q, T, blosum, 10, 2, mode, P, **kw)
        exp = oracle.search(Q, T, blosum, 10, 2, mode=mode, pssm=P)
        compare_search(got, exp, len(Q), len(T), label=f"pssm {form} {mode}")


def test_profile_of_matrix_rows_gives_matrix_results(blosum):
    c = gen.cfg2(n_targets=800, query_lengths=(80, 400))
    Q, T = c["queries"], c["targets"]
    a = _search(Q, T, blosum, 11, 1, "local", None)
    b = _search(Q, T, np.zeros_like(blosum), 11, 1, "local", blosum[Q.codes])
    for f in ("score", "q_end", "t_end"):
        assert (a[f] == b[f]).all(), f


@pytest.mark.parametrize("mode", ["local", "semiglobal"])
def test_topk_traceback_with_profiles(mode, blosum):
    import torch
    import paper_1701_01575_amd as dsa
    rng = np.random.default_rng([170101575, 122])
    c = gen.cfg2(n_targets=1200, query_lengths=(50, 350, 900))
    Q, T = c["queries"], c["targets"]
    P = _profile(rng, Q, blosum.shape[0], -5, 11)
    db = dsa.Database.from_seqset(T, blosum.shape[0])
    r = dsa.align(Q, db=db, matrix=blosum, gap_open=11, gap_extend=1, mode=mode, top_k=8, traceback=True,
                  pssm=P)
    torch.cuda.synchronize()
    full = oracle.search(Q, T, blosum, 11, 1, mode=mode, pssm=P)
    nq, nt = len(Q), len(T)
    hits = r["t_index"].cpu().numpy().reshape(nq, 8)
    for q in range(nq):
        exp = oracle.top_k(full["score"][q * nt:(q + 1) * nt], 8, positive_only=(mode == "local"))
        assert list(hits[q][:len(exp)]) == list(exp)
    valid = hits.reshape(-1) >= 0
    qi = np.repeat(np.arange(nq), 8)[valid]
    tr = oracle.align_index(qi, hits.reshape(-1)[valid], Q, T, blosum, 11, 1, mode=mode, traceback=True,
                            pssm=P)
    cig = dsa.cigars(r)
    pos = np.nonzero(valid)[0]
    for f in ("score", "q_begin", "q_end", "t_begin", "t_end"):
        assert (r[f].cpu().numpy()[pos] == np.asarray(tr[f])).all(), f
    for j, oi in enumerate(pos):
        assert (cig[oi] == tr["cigars"][j]).all(), oi
    db.close()


@pytest.mark.parametrize("kind", ["lane", "wavefront"])
@pytest.mark.parametrize("mode", ["local", "global", "semiglobal"])
def test_pairs_with_profiles(mode, kind, blosum, monkeypatch):
    import torch
    import paper_1701_01575_amd as dsa
    monkeypatch.setenv("DSA_PAIR_WF_ROWS", "100000" if kind == "lane" else "1")
    monkeypatch.setenv("DSA_PAIR_WF_CELLS", "0")
    rng = np.random.default_rng([170101575, 123])
    c = gen.cfg4(n_pairs=160)
    Q, T = c["queries"], c["targets"]
    P = _profile(rng, Q, blosum.shape[0])
    log(f"pssm pairs {mode} {kind}")
    r = dsa.align(Q, targets=T, matrix=blosum, gap_open=10, gap_extend=1, mode=mode, traceback=True, pssm=P)
    torch.cuda.synchronize()
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode=mode, traceback=True, pssm=P)
    cig = dsa.cigars(r)
    for f in ("score", "q_begin", "q_end", "t_begin", "t_end"):
        assert (r[f].cpu().numpy() == np.asarray(exp[f])).all(), f
    for k in range(len(Q)):
        assert (cig[k] == exp["cigars"][k]).all(), k


def _big_alphabet_case(seed, A, nq_lens, n_t):
    rng = np.random.default_rng([170101575, seed])
    S = rng.integers(-5, 8, size=(A, A)).astype(np.int8)
    S[np.arange(A), np.arange(A)] = rng.integers(6, 12, size=A)
    T = SeqSet.from_list([rng.integers(0, A, size=int(L)).astype(np.uint8)
                          for L in rng.integers(0, 500, size=n_t)])
    Q = SeqSet.from_list([rng.integers(0, A, size=L).astype(np.uint8) for L in nq_lens])
    return S, Q, T


@pytest.mark.parametrize("A", [33, 48, 64])
def test_alphabets_beyond_32_codes(A):
    """A custom matrix over 33 to 64 letters: database search (int32
    kernels), top-K with the hits' traceback, and pairwise alignment with
    traceback, against the oracle."""
    import torch
    import paper_1701_01575_amd as dsa
    S, Q, T = _big_alphabet_case(124 + A, A, (40, 260, 700), 600)
    log(f"alphabet of {A} letters")
    for mode in ("local", "global"):
        got = _search(Q, T, S, 9, 2, mode, None)
        exp = oracle.search(Q, T, S, 9, 2, mode=mode)
        compare_search(got, exp, len(Q), len(T), label=f"A={A} {mode}")
    db = dsa.Database.from_seqset(T, A)
    r = dsa.align(Q, db=db, matrix=S, gap_open=9, gap_extend=2, top_k=5, traceback=True)
    torch.cuda.synchronize()
    hits = r["t_index"].cpu().numpy()
    full = oracle.search(Q, T, S, 9, 2)
    nt = len(T)
    for q in range(len(Q)):
        exp = oracle.top_k(full["score"][q * nt:(q + 1) * nt], 5)
        assert list(hits[q * 5:q * 5 + len(exp)]) == list(exp)
    db.close()
    P2 = SeqSet.from_list([T[k] for k in range(20)])
    Q2 = SeqSet.from_list([Q[k % len(Q)][:300] for k in range(20)])
    r = dsa.align(Q2, targets=P2, matrix=S, gap_open=9, gap_extend=2, mode="global", traceback=True)
    torch.cuda.synchronize()
    exp = oracle.align_pairs(Q2, P2, S, 9, 2, mode="global", traceback=True)
    cig = dsa.cigars(r)
    assert (r["score"].cpu().numpy() == exp["score"]).all()
    for k in range(20):
        assert (cig[k] == exp["cigars"][k]).all(), k


def test_template_class_subclass_with_profile(blosum):
    """The paper's algorithm template: a DSW subclass that overrides the
    scoring with a profile built from the queries gives the oracle's results
    for that profile; DNW and DSG give the global and semi-global results."""
    import torch
    import paper_1701_01575_amd as dsa
    rng = np.random.default_rng([170101575, 125])
    c = gen.cfg2(n_targets=600, query_lengths=(70, 420))
    Q, T = c["queries"], c["targets"]
    bonus = rng.integers(0, 4, size=len(Q.codes)).astype(np.int8)

    class Weighted(dsa.DSW):
        def profile(self, queries):  # the matrix row of each residue plus a per-position bonus
            return (self.matrix()[queries.codes] + bonus[:, None]).astype(np.int8)

    db = dsa.Database.from_seqset(T, blosum.shape[0])
    for alg, mode, P in ((Weighted(blosum, 11, 1), "local", (blosum[Q.codes] + bonus[:, None]).astype(np.int8)),
                         (dsa.DNW(blosum, 11, 1), "global", None), (dsa.DSG(blosum, 11, 1), "semiglobal", None)):
        r = alg.align(Q, db=db)
        torch.cuda.synchronize()
        exp = oracle.search(Q, T, blosum, 11, 1, mode=mode, pssm=P)
        got = {k: v.cpu().numpy() for k, v in r.items() if hasattr(v, "cpu")}
        compare_search(got, exp, len(Q), len(T), label=f"template {mode}")
    db.close()
