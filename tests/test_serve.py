"""The chunk-step serving loop on the CPU: requests join at step boundaries
while others are active, every query sees each database chunk once and its
merged K best equal the K best over the whole database (with the traced
alignment of each hit), admission follows arrival order within the HBM
budget, a request that can never fit is refused, and a failing request does
not take others down.  The backend is the tests' own: it answers each chunk
scan and each traceback with the oracle on a small database, so the
scheduler runs without a GPU."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1701_01575_amd.serve import AdmissionError, Seqs, Server, merge_topk
from workloads import gen
from workloads.gen import SeqSet


class OracleStepBackend:
    def __init__(self, targets, S, k=3, chunks=4, per_query_bytes=100, base=50, delay=0.0, poison=None):
        self.T, self.S, self.top_k = targets, S, k
        self.positive_only = True
        n = len(targets)
        self.bounds = np.linspace(0, n, chunks + 1).astype(int)
        self.n_chunks = chunks
        self.per_q, self.base = per_query_bytes, base
        self.delay, self.poison = delay, poison
        self.scans = []          # (chunk, number of queries)
        self.lock = threading.Lock()

    def footprint(self, lens):
        return self.base + self.per_q * len(lens) if len(lens) else 0

    def _check(self, queries):
        if self.poison is not None:
            for q in range(len(queries)):
                if len(queries[q]) == self.poison and (queries[q] == 1).all():
                    raise RuntimeError("poisoned query")

    def search(self, chunk, queries):
        time.sleep(self.delay)
        self._check(queries)
        lo, hi = self.bounds[chunk], self.bounds[chunk + 1]
        sub = self.T.subset(range(lo, hi))
        r = oracle.search(queries, sub, self.S, 11, 1, threads=2)
        nt = hi - lo
        out = []
        for q in range(len(queries)):
            sc = r["score"][q * nt:(q + 1) * nt]
            idx = oracle.top_k(sc, self.top_k)
            out.append((idx + lo, sc[idx]))
        with self.lock:
            self.scans.append((chunk, len(queries)))
        return out

    def collect(self, handle):
        return handle

    def trace(self, queries, hits):
        out = []
        for q in range(len(queries)):
            t = np.asarray(hits[q], np.int64)
            r = oracle.align_index(np.zeros(len(t), np.int64), t, SeqSet.from_list([queries[q]]), self.T,
                                   self.S, 11, 1, mode="local", traceback=True, threads=2)
            out.append({"t_index": t, "score": r["score"], "q_begin": r["q_begin"], "cigars": r["cigars"]})
        return out

    def collect_trace(self, handle):
        return handle


def expected(queries, T, S, k):
    r = oracle.search(queries, T, S, 11, 1, threads=2)
    nt = len(T)
    out = []
    for q in range(len(queries)):
        sc = r["score"][q * nt:(q + 1) * nt]
        idx = oracle.top_k(sc, k)
        out.append((idx, sc[idx]))
    return out


def _requests(n, seed=0):
    rng = np.random.default_rng([170101575, 80, seed])
    reqs = []
    for _ in range(n):
        nq = int(rng.integers(1, 5))
        qs = [gen.background_residues(rng, int(rng.integers(5, 40))) for _ in range(nq)]
        offs = np.concatenate([[0], np.cumsum([len(x) for x in qs])])
        reqs.append(Seqs(np.concatenate(qs), offs))
    return reqs


@pytest.fixture(scope="module")
def db():
    return gen.random_protein_set(np.random.default_rng(5).integers(10, 60, size=40),
                                  np.random.default_rng(6))


def test_merge_topk_order():
    idx, sc = merge_topk([7, 3, 9, 1, 4], [5, 5, 8, 0, -2], 3)
    assert list(idx) == [9, 3, 7] and list(sc) == [8, 5, 5]
    idx, _ = merge_topk([2, 1], [-3, -3], 5, positive_only=False)
    assert list(idx) == [1, 2]


def test_steps_merge_to_whole_database_topk(db, blosum):
    """Requests arriving while others run join at later steps; each query's
    merged per-chunk hits equal the oracle's K best over all 40 targets,
    and each hit's traced alignment is the oracle's."""
    reqs = _requests(12)
    be = OracleStepBackend(db, blosum, k=3, chunks=4, delay=0.02)
    srv = Server(None, hbm_budget_bytes=10_000, backend=be).start()
    futs = []
    for r in reqs:
        futs.append(srv.submit(r))
        time.sleep(0.015)
    got = [f.result(timeout=60) for f in futs]
    srv.stop()
    for r, g in zip(reqs, got):
        exp = expected(r, db, blosum, 3)
        assert len(g) == len(r)
        for q, (x_idx, x_sc) in enumerate(exp):
            assert list(g[q]["t_index"]) == list(x_idx)
            assert list(g[q]["score"]) == list(x_sc)
            tr = oracle.align_index(np.zeros(len(x_idx), np.int64), x_idx, SeqSet.from_list([r[q]]), db,
                                    blosum, 11, 1, mode="local", traceback=True)
            assert list(g[q]["q_begin"]) == list(tr["q_begin"])
            for a, b in zip(g[q]["cigars"], tr["cigars"]):
                assert (a == b).all()
    st = srv.stats()
    assert st["completed"] == 12 and st["rejected"] == 0 and st["errors"] == 0
    # continuous batching: some step admitted queries while others were active
    assert any(joined > 0 and n_active > joined for _, _, n_active, joined, _ in srv.steps)
    # every scan covers one chunk; chunks go round in order
    assert [c for _, c, n, _, _ in srv.steps] == [s % 4 for s, _, _, _, _ in srv.steps]
    assert st["p99_s"] >= st["p50_s"] > 0 and st["n"] == 12


def test_each_query_scans_every_chunk_once(db, blosum):
    reqs = _requests(5, seed=4)
    be = OracleStepBackend(db, blosum, k=2, chunks=3)
    srv = Server(None, hbm_budget_bytes=10_000, backend=be)
    futs = [srv.submit(r) for r in reqs]
    srv.start()
    for f in futs:
        f.result(timeout=60)
    srv.stop()
    total_queries = sum(len(r) for r in reqs)
    assert sum(n for _, n in be.scans) == 3 * total_queries


def test_budget_bounds_active_queries_fifo(db, blosum):
    """At 100 bytes per query plus 50, a 450-byte budget holds at most 4
    active queries; requests are admitted in arrival order."""
    reqs = _requests(8, seed=1)
    be = OracleStepBackend(db, blosum, k=2, chunks=2, delay=0.005)
    srv = Server(None, hbm_budget_bytes=450, backend=be)
    futs = [srv.submit(r) for r in reqs]
    srv.start()
    for f in futs:
        f.result(timeout=60)
    srv.stop()
    assert max(n for _, _, n, _, _ in srv.steps) <= 4
    assert srv.peak_footprint <= 450
    starts = [r.start for r in sorted(srv.completed, key=lambda r: r.rid)]
    assert starts == sorted(starts)


def test_oversized_request_rejected_others_served(db, blosum):
    be = OracleStepBackend(db, blosum, per_query_bytes=200)
    srv = Server(None, hbm_budget_bytes=1000, backend=be).start()
    small = _requests(3, seed=2)   # at most 4 queries: <= 850 bytes
    big = Seqs(np.zeros(100, np.uint8), np.arange(0, 101, 10))
    f_small = [srv.submit(r) for r in small[:2]]
    f_big = srv.submit(big)   # 10 queries x 200 + 50 > 1000: can never fit
    f_last = srv.submit(small[2])
    with pytest.raises(AdmissionError):
        f_big.result(timeout=60)
    for f in f_small + [f_last]:
        f.result(timeout=60)
    srv.stop()
    assert srv.stats()["rejected"] == 1


def test_error_isolated_to_failing_request(db, blosum):
    reqs = _requests(5, seed=3)
    bad_len = 7
    bad = Seqs(np.ones(bad_len, np.uint8), np.array([0, bad_len]))
    be = OracleStepBackend(db, blosum, poison=bad_len)
    srv = Server(None, hbm_budget_bytes=100_000, backend=be)
    futs = [srv.submit(r) for r in reqs[:2]] + [srv.submit(bad)] + [srv.submit(r) for r in reqs[2:]]
    srv.start()
    results = []
    for f in futs:
        try:
            results.append(f.result(timeout=60))
        except RuntimeError:
            results.append(None)
    srv.stop()
    assert results[2] is None
    assert all(r is not None for k, r in enumerate(results) if k != 2)
    assert srv.stats()["errors"] == 1


def test_server_needs_db_and_matrix():
    with pytest.raises(ValueError):
        Server(None, 1 << 30)
