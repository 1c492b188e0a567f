"""Serving on the GPU: a resident database (the serving recipe at reduced
size) in chunks, requests joining at step boundaries while others run; every
request's top-K hits with traceback are bit-identical to the same queries
searched alone against the whole database in one call (top-K with hit
traceback), and match the oracle."""
import time

import numpy as np
import pytest

import oracle
from gpu_util import log
from workloads import gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu

FIELDS = ("t_index", "score", "q_begin", "q_end", "t_begin", "t_end")


def _alone(dsa, db, S, queries):
    import torch
    r = dsa.align(queries, db=db, matrix=S, gap_open=11, gap_extend=1, top_k=10, traceback=True)
    torch.cuda.synchronize()
    host = {f: r[f].cpu().numpy() for f in FIELDS}
    cig = dsa.cigars(r)
    out = []
    for q in range(len(queries)):
        sl = slice(q * 10, (q + 1) * 10)
        d = {f: host[f][sl] for f in FIELDS}
        d["cigars"] = cig[sl]
        out.append(d)
    return out


def test_serving_mix_equals_alone_and_oracle():
    import paper_1701_01575_amd as dsa
    c = gen.cfg5_db(n_targets=20000)
    T, S = c["targets"], c["matrix"]
    db = dsa.Database.from_seqset(T, S.shape[0])
    rng = np.random.default_rng([170101575, 90])
    reqs = []
    for _ in range(10):
        nq = int(rng.integers(1, 5))
        lens = gen.loguniform_lengths(rng, nq, 30, 600)
        reqs.append(gen.random_protein_set(lens, rng))
    log("serving: 10 requests alone (one top-K + traceback call each)")
    alone = [_alone(dsa, db, S, r) for r in reqs]
    srv = dsa.Server(db, 64 << 30, matrix=S, gap_open=11, gap_extend=1, top_k=10, chunks=4).start()
    log("serving: 10 requests through the chunk-step server")
    futs = []
    for r in reqs:
        futs.append(srv.submit(r))
        time.sleep(0.01)
    mixed = [f.result(timeout=300) for f in futs]
    srv.stop()
    st = srv.stats()
    assert st["completed"] == 10 and st["errors"] == 0
    for a, m in zip(alone, mixed):
        for x, y in zip(a, m):
            for f in FIELDS:
                assert (x[f] == y[f]).all(), f
            for cx, cy in zip(x["cigars"], y["cigars"]):
                assert (cx == cy).all()
    # oracle check of the first request's hits
    r0, q0 = alone[0], reqs[0]
    for q in range(len(q0)):
        hits = r0[q]["t_index"]
        valid = hits >= 0
        Q1 = SeqSet.from_list([q0[q]])
        full = oracle.search(Q1, T, S, 11, 1)
        assert (oracle.top_k(full["score"], 10) == hits[valid]).all()
        if not valid.any():
            continue
        exp = oracle.align_index(np.zeros(valid.sum(), np.int64), hits[valid], Q1, T, S, 11, 1,
                                 mode="local", traceback=True)
        assert (exp["score"] == r0[q]["score"][valid]).all()
        assert (exp["q_begin"] == r0[q]["q_begin"][valid]).all()
        for k, j in enumerate(np.nonzero(valid)[0]):
            assert (exp["cigars"][k] == r0[q]["cigars"][j]).all()
    srv.backend.close()
    db.close()
