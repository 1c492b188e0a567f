"""dsa_autotune on the GPU: the choice comes from the candidate set, the
results of the class are the same before and after tuning (tuning only moves
work between kernels and launch shapes), and the JSON cache holds the class."""
import json

import numpy as np
import pytest

import oracle
from gpu_util import log
from workloads import gen

pytestmark = pytest.mark.gpu


def _host(r, fields=("score", "q_end", "t_end", "q_begin", "t_begin")):
    return {k: r[k].cpu().numpy() for k in fields if k in r}


@pytest.mark.parametrize("plain", [False, True], ids=["batched", "plain"])
def test_autotune_search(plain, blosum, tmp_path):
    import torch
    import paper_1701_01575_amd as dsa
    c = gen.cfg2(n_targets=4000, query_lengths=(144, 700))
    Q, T = c["queries"], c["targets"]
    db = dsa.Database.from_seqset(T, blosum.shape[0])
    before = _host(dsa.align(Q, db=db, matrix=blosum, plain=plain))
    path = str(tmp_path / "tune.json")
    log(f"autotune search plain={plain}")
    ch = dsa.autotune(Q, db=db, matrix=blosum, plain=plain, cache_path=path)
    assert ch["strip"] in (16, 32) and ch["waves"] in (2, 4, 8) and ch["ms"] > 0
    now = dsa.tuning(Q, db=db, matrix=blosum, plain=plain)
    assert (now["strip"], now["waves"], now["intra_budget"], now["ks_budget"]) == \
        (ch["strip"], ch["waves"], ch["intra_budget"], ch["ks_budget"])
    assert ch["ks_budget"] >= 0 and (ch["ks_budget"] == 0 or (not plain and ch["strip"] == 16))
    after = _host(dsa.align(Q, db=db, matrix=blosum, plain=plain))
    torch.cuda.synchronize()
    for k in before:
        assert (before[k] == after[k]).all(), k
    exp = oracle.search(Q, T, blosum, 11, 1, mode="local")
    assert (after["score"] == exp["score"]).all() and (after["t_end"] == exp["t_end"]).all()
    entries = json.load(open(path))
    assert [e["key"] for e in entries] == [now["key"]]
    db.close()


def test_autotune_pairs(blosum, tmp_path):
    import paper_1701_01575_amd as dsa
    Q, T = gen.related_pairs(23, 300, 40, 700)
    before = dsa.align(Q, targets=T, matrix=blosum, gap_open=10, gap_extend=1, mode="global", traceback=True)
    bc = dsa.cigars(before)
    before = _host(before)
    path = str(tmp_path / "tune.json")
    log("autotune pairs")
    ch = dsa.autotune(Q, targets=T, matrix=blosum, gap_open=10, gap_extend=1, mode="global",
                      traceback=True, cache_path=path)
    assert ch["pair_rows"] in (48, 64, 96, 128, 192, 256, 512, 1 << 30)
    after = dsa.align(Q, targets=T, matrix=blosum, gap_open=10, gap_extend=1, mode="global", traceback=True)
    ac = dsa.cigars(after)
    after = _host(after)
    for k in before:
        assert (before[k] == after[k]).all(), k
    assert all(len(x) == len(y) and (x == y).all() for x, y in zip(ac, bc))
    assert json.load(open(path))[0]["pair_rows"] == ch["pair_rows"]
