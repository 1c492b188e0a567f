"""The boundary's memory rules on the GPU: a database whose device buffers
come from the caller's allocator (torch's caching allocator through
dsa_allocator) gives the same results as one from hipMalloc and hands every
buffer back on destroy; and two calls in flight at once on two streams, each
with its own workspace, both match the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import log
from workloads import gen

pytestmark = pytest.mark.gpu


def test_database_from_torch_allocator(blosum):
    import torch
    import paper_1701_01575_amd as dsa
    c = gen.cfg2(n_targets=3000, query_lengths=(100, 700))
    Q, T = c["queries"], c["targets"]
    before = torch.cuda.memory_allocated()
    db_t = dsa.Database.from_seqset(T, blosum.shape[0], allocator="torch")
    n_t, n_res, dev_bytes = db_t.info()
    assert (n_t, n_res) == (len(T), int(T.lengths.sum()))
    assert db_t.allocator.bytes_held() == dev_bytes > 0
    assert torch.cuda.memory_allocated() - before >= dev_bytes
    db_h = dsa.Database.from_seqset(T, blosum.shape[0], allocator=None)
    assert db_h.allocator is None and db_h.info()[2] == dev_bytes
    log("search through the torch-allocated and the hipMalloc-allocated database")
    r_t = dsa.align(Q, db=db_t, matrix=blosum, gap_open=11, gap_extend=1)
    r_h = dsa.align(Q, db=db_h, matrix=blosum, gap_open=11, gap_extend=1)
    torch.cuda.synchronize()
    exp = oracle.search(Q, T, blosum, 11, 1)
    for f in ("score", "q_end", "t_end"):
        assert (r_t[f].cpu().numpy() == exp[f]).all(), f
        assert (r_h[f].cpu().numpy() == exp[f]).all(), f
    db_t.close()
    db_h.close()
    assert db_t.allocator.bytes_held() == 0


def test_two_streams_in_flight(blosum):
    """A long search on one stream and a pairwise batch on another are both
    enqueued before either is waited for; each call's workspace comes from
    torch's caching allocator on its own stream, so neither overwrites the
    other's tables or boundary rows."""
    import torch
    import paper_1701_01575_amd as dsa
    c = gen.cfg2(n_targets=4000, query_lengths=(300, 1500, 2500))
    Q, T = c["queries"], c["targets"]
    p = gen.cfg4(n_pairs=400)
    db = dsa.Database.from_seqset(T, blosum.shape[0])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    log("two calls in flight on two streams")
    torch.cuda.synchronize()
    r1 = dsa.align(Q, db=db, matrix=blosum, gap_open=11, gap_extend=1, stream=s1)
    r2 = dsa.align(p["queries"], targets=p["targets"], matrix=blosum, gap_open=10, gap_extend=1,
                   mode="global", stream=s2)
    r3 = dsa.align(Q, db=db, matrix=blosum, gap_open=11, gap_extend=1, mode="semiglobal", stream=s2)
    s1.synchronize()
    s2.synchronize()
    exp1 = oracle.search(Q, T, blosum, 11, 1)
    exp2 = oracle.align_pairs(p["queries"], p["targets"], blosum, 10, 1, mode="global")
    exp3 = oracle.search(Q, T, blosum, 11, 1, mode="semiglobal")
    for r, exp, label in ((r1, exp1, "search"), (r2, exp2, "pairs"), (r3, exp3, "semi-global search")):
        for f in ("score", "q_end", "t_end"):
            got = r[f].cpu().numpy()[:len(exp[f])]
            assert (got == np.asarray(exp[f])).all(), (label, f)
    db.close()
