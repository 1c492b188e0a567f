"""Serving on the GPU: a resident database (the serving recipe at reduced
size), requests batched continuously over two streams; every request's
top-K hits with traceback are bit-identical alone and in the mix, and match
the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import log
from workloads import gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu


def test_serving_mix_equals_alone_and_oracle():
    import torch
    import paper_1701_01575_amd as dsa
    from paper_1701_01575_amd.serve import GpuBackend, Server
    c = gen.cfg5_db(n_targets=20000)
    T, S = c["targets"], c["matrix"]
    db = dsa.Database.from_seqset(T, S.shape[0])
    rng = np.random.default_rng([170101575, 90])
    reqs = []
    for _ in range(10):
        nq = int(rng.integers(1, 5))
        lens = gen.loguniform_lengths(rng, nq, 30, 600)
        reqs.append(gen.random_protein_set(lens, rng))
    be = GpuBackend(db, S, 11, 1, top_k=10, traceback=True)
    stream = be.make_stream()
    log("serving: 10 requests alone")
    alone = [be.run(r, stream) for r in reqs]
    srv = Server(be, hbm_budget_bytes=64 << 30, slots=2, max_batch_queries=8).start()
    log("serving: 10 requests through the server")
    futs = [srv.submit(r) for r in reqs]
    mixed = [f.result(timeout=300) for f in futs]
    srv.stop()
    assert srv.stats()["completed"] == 10 and srv.stats()["batches"] < 10
    for a, m in zip(alone, mixed):
        for x, y in zip(a, m):
            for f in ("t_index", "score", "q_begin", "q_end", "t_begin", "t_end"):
                assert (x[f] == y[f]).all(), f
            for cx, cy in zip(x["cigars"], y["cigars"]):
                assert (cx == cy).all()
    # oracle check of the first request's hits
    r0, q0 = alone[0], reqs[0]
    for q in range(len(q0)):
        hits = r0[q]["t_index"]
        valid = hits >= 0
        if not valid.any():
            continue
        Q1 = SeqSet.from_list([q0[q]])
        exp = oracle.align_index(np.zeros(valid.sum(), np.int64), hits[valid], Q1, T, S, 11, 1,
                                 mode="local", traceback=True)
        assert (exp["score"] == r0[q]["score"][valid]).all()
        assert (exp["q_begin"] == r0[q]["q_begin"][valid]).all()
        for k, j in enumerate(np.nonzero(valid)[0]):
            assert (exp["cigars"][k] == r0[q]["cigars"][j]).all()
        full = oracle.search(Q1, T, S, 11, 1)
        assert (oracle.top_k(full["score"], 10) == hits[valid]).all()
