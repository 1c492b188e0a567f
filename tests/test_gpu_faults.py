"""Failure handling on the GPU, forced from the host with DSA_FAULT (every
kernel still runs to its normal end):

* ovf: every unit of a search is recomputed by the int32 rerun; results are
  unchanged and every one carries DSA_ST_INT32;
* alloc:N: a database whose Nth buffer fails gives every buffer it took back
  to the caller's allocator;
* launch:N: exactly the Nth call fails, the next one is correct;
* qlen:L: in the serving loop only the request holding a query of length L
  fails; every other request gets the same hits as a whole-database call."""
import numpy as np
import pytest

import oracle
from gpu_util import compare_search, log
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["local", "global"])
def test_forced_rerun_gives_same_results(mode, blosum, monkeypatch):
    import torch
    import paper_1701_01575_amd as dsa
    c = gen.cfg2(n_targets=3000, query_lengths=(90, 600, 2100))
    Q, T = c["queries"], c["targets"]
    db = dsa.Database.from_seqset(T, blosum.shape[0])
    monkeypatch.setenv("DSA_FAULT", "ovf")
    log(f"DSA_FAULT=ovf, {mode}")
    r = dsa.align(Q, db=db, matrix=blosum, gap_open=11, gap_extend=1, mode=mode)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in r.items() if hasattr(v, "cpu")}
    assert (got["status"] & dsa.DSA_ST_INT32).all()
    exp = oracle.search(Q, T, blosum, 11, 1, mode=mode)
    compare_search(got, exp, len(Q), len(T), label=f"ovf {mode}")
    db.close()


@pytest.mark.parametrize("n", [1, 4, 10])
def test_alloc_fault_gives_buffers_back(n, blosum, monkeypatch):
    import paper_1701_01575_amd as dsa
    from paper_1701_01575_amd import binding as B
    c = gen.cfg2(n_targets=1000, query_lengths=(50,))
    T = c["targets"]
    alloc = dsa.TorchAllocator(dsa._torch().device("cuda", 0))
    monkeypatch.setenv("DSA_FAULT", f"alloc:{n}")
    with pytest.raises(B.DsaError) as ei:
        dsa.Database.from_seqset(T, blosum.shape[0], allocator=alloc)
    assert ei.value.status == B.DSA_E_DEVICE and "injected" in str(ei.value)
    assert alloc.bytes_held() == 0 and not alloc.held
    monkeypatch.delenv("DSA_FAULT")
    db = dsa.Database.from_seqset(T, blosum.shape[0], allocator=alloc)
    assert alloc.bytes_held() == db.info()[2]
    db.close()
    assert alloc.bytes_held() == 0


def test_launch_fault_fails_one_call(blosum, monkeypatch):
    import torch
    import paper_1701_01575_amd as dsa
    from paper_1701_01575_amd import binding as B
    c = gen.cfg2(n_targets=800, query_lengths=(120,))
    Q, T = c["queries"], c["targets"]
    db = dsa.Database.from_seqset(T, blosum.shape[0])
    monkeypatch.setenv("DSA_FAULT", "launch:2")
    dsa.align(Q, db=db, matrix=blosum, gap_open=11, gap_extend=1)
    with pytest.raises(B.DsaError) as ei:
        dsa.align(Q, db=db, matrix=blosum, gap_open=11, gap_extend=1)
    assert ei.value.status == B.DSA_E_DEVICE
    r = dsa.align(Q, db=db, matrix=blosum, gap_open=11, gap_extend=1)
    torch.cuda.synchronize()
    exp = oracle.search(Q, T, blosum, 11, 1)
    assert (r["score"].cpu().numpy() == exp["score"]).all()
    db.close()


def test_serving_isolates_a_failing_request(blosum, monkeypatch):
    import torch
    import paper_1701_01575_amd as dsa
    from paper_1701_01575_amd import binding as B
    c = gen.cfg5_db(n_targets=6000)
    T, S = c["targets"], c["matrix"]
    db = dsa.Database.from_seqset(T, S.shape[0])
    rng = np.random.default_rng([170101575, 98])
    reqs = [gen.random_protein_set(gen.loguniform_lengths(rng, int(rng.integers(1, 4)), 30, 400), rng)
            for _ in range(6)]
    bad = gen.random_protein_set(np.array([100, 777]), rng)
    srv = dsa.Server(db, 32 << 30, matrix=S, top_k=5, chunks=3).start()
    monkeypatch.setenv("DSA_FAULT", "qlen:777")
    log("serving with one request holding a 777-residue query")
    futs = [srv.submit(r) for r in reqs[:3]] + [srv.submit(bad)] + [srv.submit(r) for r in reqs[3:]]
    results = []
    for f in futs:
        try:
            results.append(f.result(timeout=300))
        except B.DsaError as exc:
            results.append(exc)
    srv.stop()
    monkeypatch.delenv("DSA_FAULT")
    assert isinstance(results[3], B.DsaError) and results[3].status == B.DSA_E_DEVICE
    good = results[:3] + results[4:]
    for r, got in zip(reqs, good):
        one = dsa.align(r, db=db, matrix=S, gap_open=11, gap_extend=1, top_k=5, traceback=True)
        torch.cuda.synchronize()
        idx = one["t_index"].cpu().numpy().reshape(len(r), 5)
        sc = one["score"].cpu().numpy().reshape(len(r), 5)
        for q in range(len(r)):
            assert (got[q]["t_index"] == idx[q]).all() and (got[q]["score"] == sc[q]).all()
    assert srv.stats()["errors"] == 1
    srv.backend.close()
    db.close()
