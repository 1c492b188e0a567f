"""The allocation-free entry point dsa_align_batch_noalloc, called through
the C ABI: on two calls in a row (the second with a smaller input) its
results equal dsa_align_batch's, field by field and CIGAR by CIGAR, for a
database search, a top-K search with hit traceback and a pairwise batch
with traceback; it leaves the device's free memory unchanged; and a call
that needs more than the static scratch is refused before any device work."""
import numpy as np
import pytest

import oracle
from gpu_util import log
from workloads import gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu

FIELDS = ("score", "q_begin", "q_end", "t_begin", "t_end", "status", "t_index")


def _call(entry, queries, db=None, targets=None, S=None, o=11, e=1, mode="local", traceback=False,
          top_k=0):
    """One call through the C ABI with fresh outputs; the existing entry point
    gets a workspace of dsa_workspace_size bytes."""
    import torch
    import paper_1701_01575_amd as dsa
    from paper_1701_01575_amd import binding as B
    device = torch.device("cuda", torch.cuda.current_device())
    qc, qo = dsa.device_queries(queries, device)
    tc = to = None
    if targets is not None:
        tc, to = dsa.device_queries(targets, device)
    a = dsa.make_args(qc, qo, S, o, e, mode, db, tc, to, None, traceback, top_k, False, False, None)
    nq = len(qo) - 1
    n = nq if targets is not None else (nq * top_k if top_k else nq * db.n_targets)
    out, res = dsa._outputs(a, device, n)
    ws = None
    if entry == "batch":
        need = B.dsa_workspace_size(a)
        ws = torch.empty(need + 256, dtype=torch.uint8, device=device)
        a.workspace = (ws.data_ptr() + 255) // 256 * 256
        a.workspace_bytes = need
        st = B.dsa_align_batch(a, out)
    else:
        a.workspace = None
        a.workspace_bytes = 0
        st = B.dsa_align_batch_noalloc(a, out)
    torch.cuda.synchronize()
    got = {k: v[:n].cpu().numpy() for k, v in res.items() if k != "cigar_ops"}
    if traceback:
        got["cigars"] = dsa.cigars(res)
    del ws, qc, tc
    return got, st


def _same(x, y, label):
    for f in FIELDS:
        if f in x or f in y:
            assert (x[f] == y[f]).all(), f"{label}: field {f} differs"
    if "cigars" in x:
        assert len(x["cigars"]) == len(y["cigars"])
        for k, (cx, cy) in enumerate(zip(x["cigars"], y["cigars"])):
            assert (cx == cy).all(), f"{label}: CIGAR {k} differs"


def _search_case(n_targets, query_lengths, seed):
    c = gen.cfg2(n_targets=n_targets, query_lengths=query_lengths)
    return c["queries"], c["targets"]


def test_noalloc_search_two_calls(blosum):
    import paper_1701_01575_amd as dsa
    for label, n_t, ql in (("first", 2000, (64, 300, 900)), ("second, smaller", 700, (150,))):
        Q, T = _search_case(n_t, ql, 0)
        log(f"noalloc search {label}: {len(Q)} queries x {n_t} targets")
        db = dsa.Database.from_seqset(T, blosum.shape[0])
        ref, st0 = _call("batch", Q, db=db, S=blosum)
        got, st1 = _call("noalloc", Q, db=db, S=blosum)
        assert st0 == st1 == 0
        _same(got, ref, label)
        exp = oracle.search(Q, T, blosum, 11, 1)
        for f in ("score", "q_end", "t_end"):
            assert (got[f].astype(np.int64) == exp[f]).all(), f"{label}: {f} vs oracle"
        db.close()


def test_noalloc_topk_traceback_two_calls(blosum):
    import paper_1701_01575_amd as dsa
    for label, n_t, ql in (("first", 1500, (40, 500)), ("second, smaller", 400, (120,))):
        Q, T = _search_case(n_t, ql, 1)
        log(f"noalloc top-10 + traceback {label}: {len(Q)} queries x {n_t} targets")
        db = dsa.Database.from_seqset(T, blosum.shape[0])
        ref, st0 = _call("batch", Q, db=db, S=blosum, traceback=True, top_k=10)
        got, st1 = _call("noalloc", Q, db=db, S=blosum, traceback=True, top_k=10)
        assert st0 == st1 == 0
        _same(got, ref, label)
        db.close()


def test_noalloc_pairs_traceback_two_calls(blosum, dna):
    cases = (
        ("first: protein global", gen.cfg4(n_pairs=300), blosum, 10, 1, "global"),
        ("second, smaller: DNA local", gen.cfg3(n_pairs=200), dna, 5, 2, "local"),
    )
    for label, c, S, o, e, mode in cases:
        Q, T = c["queries"], c["targets"]
        log(f"noalloc pairs {label}: {len(Q)} pairs")
        ref, st0 = _call("batch", Q, targets=T, S=S, o=o, e=e, mode=mode, traceback=True)
        got, st1 = _call("noalloc", Q, targets=T, S=S, o=o, e=e, mode=mode, traceback=True)
        assert st0 == st1 == 0
        _same(got, ref, label)


def test_noalloc_leaves_free_memory_unchanged(blosum):
    import torch
    import paper_1701_01575_amd as dsa
    Q, T = _search_case(800, (100, 400), 2)
    db = dsa.Database.from_seqset(T, blosum.shape[0])
    _call("noalloc", Q, db=db, S=blosum)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        _call("noalloc", Q, db=db, S=blosum)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    db.close()


def test_noalloc_rejects_calls_beyond_the_scratch(blosum):
    """About 100,000 targets of 90 residues: one query's boundary rows alone
    exceed the 64 MiB scratch, so the call is refused in planning."""
    import torch
    import paper_1701_01575_amd as dsa
    from paper_1701_01575_amd import binding as B
    rng = np.random.default_rng([170101575, 91])
    T = SeqSet.from_list([gen.background_residues(rng, 90) for _ in range(100_000)])
    Q = SeqSet.from_list([gen.background_residues(rng, 50)])
    db = dsa.Database.from_seqset(T, blosum.shape[0])
    device = torch.device("cuda", torch.cuda.current_device())
    qc, qo = dsa.device_queries(Q, device)
    a = dsa.make_args(qc, qo, blosum, 11, 1, "local", db)
    assert B.dsa_workspace_size(a) > B.NOALLOC_SCRATCH_BYTES
    out, _ = dsa._outputs(a, device, db.n_targets)
    with pytest.raises(B.DsaError) as ei:
        B.dsa_align_batch_noalloc(a, out)
    assert ei.value.status == B.DSA_E_WORKSPACE
    assert "static scratch" in str(ei.value)
    db.close()
