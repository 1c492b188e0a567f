"""Recorded batches (dsa_graph_create / dsa_graph_launch): every replay of a
graph must give exactly the eager call's results.  Each test replays several
times with eager library calls, torch work and synchronizations in between,
clears the outputs before every replay, and changes the query residues (same
lengths) between replays to check that a replay reads its inputs afresh."""
import numpy as np
import pytest

import oracle
from gpu_util import log
from workloads import gen
from workloads.gen import SeqSet

pytestmark = pytest.mark.gpu

FIELDS = ("score", "q_end", "t_end", "q_begin", "t_begin", "status")


def _host(res, fields):
    return {k: res[k].cpu().numpy().copy() for k in fields if k in res}


def _mutate(Q, seed, alphabet):
    rng = np.random.default_rng([170101575, seed])
    return SeqSet(rng.integers(0, alphabet, size=len(Q.codes)).astype(np.uint8), Q.offsets.copy())


def _replay_and_check(rec, queries_seq, eager_fn, fields, tb=False):
    import torch
    import paper_1701_01575_amd as dsa
    qdev = rec._keep[0]
    for k, Q in enumerate(queries_seq):
        exp = eager_fn(Q)
        torch.cuda.synchronize()
        with torch.cuda.stream(rec.stream):
            qdev[:len(Q.codes)].copy_(torch.from_numpy(Q.codes))
            for f in fields:
                if f in rec.results():
                    v = rec.results()[f]
                    v.fill_(7 if v.dtype == torch.uint8 else -7)
            # unrelated device work between replays
            x = torch.randn(1 << 16, device=rec.device)
            (x * 2).sum().item()
            rec.run()
        rec.stream.synchronize()
        got = _host(rec.results(), fields)
        for f in fields:
            if f not in exp:
                continue
            bad = np.nonzero(got[f] != exp[f])[0]
            assert len(bad) == 0, f"replay {k} field {f}: {len(bad)} mismatches, first {bad[0]}"
        if tb:
            a, b = dsa.cigars(rec.results()), exp["cigars"]
            for r in range(len(b)):
                assert len(a[r]) == len(b[r]) and (a[r] == b[r]).all(), f"replay {k} cigar {r}"


@pytest.mark.parametrize("mode,top_k,route", [
    ("local", 0, None), ("global", 0, None), ("semiglobal", 0, None), ("local", 5, None),
    ("local", 0, "wavefront"), ("local", 0, "pipelined"), ("local", 5, "pipelined")])
def test_graph_search(mode, top_k, route, blosum, monkeypatch):
    """Replays of a recorded search; the routed cases send every group at
    least 128 columns wide to the wavefront or the strip-pipelined units,
    which then run inside the recorded persistent launch."""
    import torch
    import paper_1701_01575_amd as dsa
    if route is not None:
        monkeypatch.setenv("DSA_INTRA_BUDGET", "1")
        monkeypatch.setenv("DSA_KS_BUDGET", "0" if route == "wavefront" else str(1 << 40))
    c = gen.cfg2(n_targets=3000, query_lengths=(20, 144, 700))
    Q, T = c["queries"], c["targets"]
    db = dsa.Database.from_seqset(T, blosum.shape[0])
    log(f"graph search mode={mode} top_k={top_k} route={route}")

    def eager(Qx):
        r = dsa.align(Qx, db=db, matrix=blosum, gap_open=11, gap_extend=1, mode=mode, top_k=top_k)
        torch.cuda.synchronize()
        out = _host(r, FIELDS + ("t_index",))
        return out

    rec = dsa.Recorded(Q, db=db, matrix=blosum, gap_open=11, gap_extend=1, mode=mode, top_k=top_k)
    seq = [Q, _mutate(Q, 90, 20), Q, _mutate(Q, 91, 20)]
    _replay_and_check(rec, seq, eager, FIELDS + ("t_index",))
    # the recorded query set once more, against the oracle
    if not top_k:
        exp = oracle.search(Q, T, blosum, 11, 1, mode=mode)
        with torch.cuda.stream(rec.stream):
            rec._keep[0][:len(Q.codes)].copy_(torch.from_numpy(Q.codes))
            rec.run()
        rec.stream.synchronize()
        got = rec.results()
        for f in ("score", "q_end", "t_end"):
            assert (got[f].cpu().numpy() == exp[f]).all(), f
    rec.close()
    db.close()


@pytest.mark.parametrize("mode", ["local", "global", "semiglobal"])
def test_graph_pairs_traceback(mode, blosum, monkeypatch):
    """Lane-group and wavefront pairs together (two streams inside the graph),
    direction codes in several chunks."""
    import torch
    import paper_1701_01575_amd as dsa
    monkeypatch.setenv("DSA_TB_BUDGET", str(1 << 20))
    Q1, T1 = gen.random_pairs(21, 100, 90, 20, min_len=0)
    Q2, T2 = gen.related_pairs(22, 60, 100, 900)
    Q = SeqSet.from_list([Q1[k] for k in range(len(Q1))] + [Q2[k] for k in range(len(Q2))])
    T = SeqSet.from_list([T1[k] for k in range(len(T1))] + [T2[k] for k in range(len(T2))])
    log(f"graph pairs mode={mode} n={len(Q)}")

    def eager(Qx):
        r = dsa.align(Qx, targets=T, matrix=blosum, gap_open=10, gap_extend=1, mode=mode, traceback=True)
        torch.cuda.synchronize()
        out = _host(r, FIELDS)
        out["cigars"] = dsa.cigars(r)
        return out

    rec = dsa.Recorded(Q, targets=T, matrix=blosum, gap_open=10, gap_extend=1, mode=mode, traceback=True)
    assert rec.capacity_ok
    seq = [Q, _mutate(Q, 92, 20), Q]
    _replay_and_check(rec, seq, eager, FIELDS, tb=True)
    exp = oracle.align_pairs(Q, T, blosum, 10, 1, mode=mode, traceback=True)
    got = rec.results()
    assert (got["score"].cpu().numpy() == exp["score"]).all()
    rec.close()


def test_graph_topk_traceback_not_recordable(blosum):
    import paper_1701_01575_amd as dsa
    c = gen.cfg2(n_targets=300, query_lengths=(50,))
    db = dsa.Database.from_seqset(c["targets"], blosum.shape[0])
    with pytest.raises(dsa.DsaError) as ei:
        dsa.Recorded(c["queries"], db=db, matrix=blosum, top_k=3, traceback=True)
    assert ei.value.status == dsa.binding.DSA_E_NOTSUP
    db.close()
