"""Serving loop on the CPU: FIFO admission by HBM budget, continuous
batching over several slots, overlap, rejection of requests that can never
fit, per-request error isolation, and results that are the same alone and
in the mix.  The backend here is the tests' own: it answers with the oracle's
top-K hits on a tiny database, so the scheduling logic runs without a GPU."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1701_01575_amd.serve import AdmissionError, Server, Seqs
from workloads import gen


class OracleBackend:
    def __init__(self, targets, S, k=3, per_query_bytes=100, base=50, delay=0.0, poison=None):
        self.T, self.S, self.k = targets, S, k
        self.per_q, self.base = per_query_bytes, base
        self.delay, self.poison = delay, poison
        self.running = 0
        self.max_running = 0
        self.lock = threading.Lock()

    def footprint(self, queries):
        return self.base + self.per_q * len(queries)

    def run(self, queries, stream):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
        try:
            time.sleep(self.delay)
            if self.poison is not None and any(len(queries[q]) == self.poison and (queries[q] == 1).all()
                                               for q in range(len(queries))):
                raise RuntimeError("poisoned query")
            r = oracle.search(queries, self.T, self.S, 11, 1, threads=2)
            nt = len(self.T)
            out = []
            for q in range(len(queries)):
                sc = r["score"][q * nt:(q + 1) * nt]
                idx = oracle.top_k(sc, self.k)
                out.append({"t_index": idx, "score": sc[idx]})
            return out
        finally:
            with self.lock:
                self.running -= 1


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


def test_mix_equals_alone_and_budget_respected(db, blosum):
    reqs = _requests(14)
    be = OracleBackend(db, blosum, delay=0.01)
    alone = [be.run(r, None) for r in reqs]
    srv = Server(be, hbm_budget_bytes=900, slots=3, max_batch_queries=6).start()
    futs = [srv.submit(r) for r in reqs]
    mixed = [f.result(timeout=60) for f in futs]
    srv.stop()
    for a, m in zip(alone, mixed):
        assert len(a) == len(m)
        for x, y in zip(a, m):
            assert (x["t_index"] == y["t_index"]).all() and (x["score"] == y["score"]).all()
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert srv.peak_in_flight <= 900
    assert st["batches"] < len(reqs)          # requests were batched together
    assert be.max_running >= 2                # batches overlapped on the slots
    assert st["p99_s"] >= st["p50_s"] > 0


def test_fifo_dispatch_order(db, blosum):
    be = OracleBackend(db, blosum, delay=0.005)
    srv = Server(be, hbm_budget_bytes=10_000, slots=1, max_batch_queries=1)
    futs = [srv.submit(r) for r in _requests(6, seed=1)]
    srv.start()
    for f in futs:
        f.result(timeout=60)
    srv.stop()
    order = [ids[0] for ids, _ in srv.batches]
    assert order == sorted(order)


def test_oversized_request_rejected_others_served(db, blosum):
    be = OracleBackend(db, blosum, per_query_bytes=200)
    srv = Server(be, hbm_budget_bytes=1000, slots=2).start()
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
    be = OracleBackend(db, blosum, poison=bad_len)
    srv = Server(be, hbm_budget_bytes=100_000, slots=1, max_batch_queries=64)
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
