"""Full parity at full size, in the launch configuration the benchmark times
(one batched call per workload), against the oracle on the host's cores:

* protein database search: 5 queries (144, 464, 1000, 2000, 5000 residues)
  against 200,000 log-normal targets, local, every one of the 1,000,000
  results (score, query end, target end);
* read mapping: all 100,000 DNA read / window pairs, local, with begins and
  CIGAR;
* protein pairs: all 50,000 pairs in global and in semi-global mode, with
  begins and CIGAR.

Each workload runs once on the GPU (module fixtures); the oracle checks it in
slices, each a test of well under a minute on 16 threads, so that progress is
printed as it goes."""
import numpy as np
import pytest

import oracle
from gpu_util import log
from test_gpu_pairs import compare_pairs, gpu_pairs
from workloads import gen

pytestmark = [pytest.mark.gpu, pytest.mark.fullsize]

SEARCH_SLICES = 8
PAIR_SLICES = 2


@pytest.fixture(scope="module")
def search_cfg():
    import torch
    import paper_1701_01575_amd as dsa
    c = gen.cfg2()
    Q, T = c["queries"], c["targets"]
    log("full size: 5 queries x 200,000 targets on the GPU")
    db = dsa.Database.from_seqset(T, c["matrix"].shape[0])
    r = dsa.align(Q, db=db, matrix=c["matrix"], gap_open=11, gap_extend=1, mode="local")
    torch.cuda.synchronize()
    got = {k: r[k].cpu().numpy().reshape(len(Q), len(T)) for k in ("score", "q_end", "t_end", "status")}
    db.close()
    return c, got


@pytest.mark.parametrize("part", range(SEARCH_SLICES))
def test_search_full_parity(search_cfg, part):
    """Targets [part * 25,000, (part + 1) * 25,000) against all 5 queries."""
    c, got = search_cfg
    Q, T = c["queries"], c["targets"]
    nq, nt = len(Q), len(T)
    lo, hi = part * nt // SEARCH_SLICES, (part + 1) * nt // SEARCH_SLICES
    qi = np.repeat(np.arange(nq), hi - lo)
    ti = np.tile(np.arange(lo, hi), nq)
    log(f"oracle: targets {lo}..{hi - 1} x {nq} queries")
    exp = oracle.align_index(qi, ti, Q, T, c["matrix"], 11, 1, mode="local")
    for f in ("score", "q_end", "t_end"):
        g = got[f][:, lo:hi].reshape(-1).astype(np.int64)
        x = np.asarray(exp[f]).astype(np.int64)
        bad = np.nonzero(g != x)[0]
        assert len(bad) == 0, (f"{f}: {len(bad)} mismatches; first query {qi[bad[0]]} target {ti[bad[0]]}: "
                               f"gpu {g[bad[0]]} oracle {x[bad[0]]}")


@pytest.fixture(scope="module")
def read_mapping():
    c = gen.cfg3()
    log("full size: 100,000 read / window pairs on the GPU")
    got = gpu_pairs(c["queries"], c["targets"], c["matrix"], 5, 2, "local")
    assert got["capacity_ok"]
    return c, got


def test_read_mapping_full_parity(read_mapping):
    c, got = read_mapping
    log("oracle: all 100,000 pairs with traceback")
    exp = oracle.align_pairs(c["queries"], c["targets"], c["matrix"], 5, 2, mode="local", traceback=True)
    compare_pairs(got, exp, True, "read mapping")


_PROTEIN = {}


def _protein_pairs(mode):
    if mode not in _PROTEIN:
        c = _PROTEIN.get("inputs") or gen.cfg4()
        _PROTEIN["inputs"] = c
        log(f"full size: 50,000 protein pairs, {mode}, on the GPU")
        got = gpu_pairs(c["queries"], c["targets"], c["matrix"], 10, 1, mode)
        assert got["capacity_ok"]
        _PROTEIN.pop("global" if mode == "semiglobal" else "semiglobal", None)
        _PROTEIN[mode] = got
    return _PROTEIN["inputs"], _PROTEIN[mode]


@pytest.mark.parametrize("part", range(PAIR_SLICES))
@pytest.mark.parametrize("mode", ["global", "semiglobal"])
def test_protein_pairs_full_parity(mode, part):
    c, got = _protein_pairs(mode)
    n = len(c["queries"])
    lo, hi = part * n // PAIR_SLICES, (part + 1) * n // PAIR_SLICES
    idx = np.arange(lo, hi)
    log(f"oracle: protein pairs {lo}..{hi - 1}, {mode}, with traceback")
    exp = oracle.align_index(idx, idx, c["queries"], c["targets"], c["matrix"], 10, 1, mode=mode,
                             traceback=True)
    sub = {k: v[lo:hi] for k, v in got.items() if isinstance(v, np.ndarray)}
    sub["cigars"] = got["cigars"][lo:hi]
    compare_pairs(sub, exp, True, f"protein pairs {mode}")
