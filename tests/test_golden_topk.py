"""The oracle's top-K order (Section II.B.2: the K best alignments of a
query by maximum score) against hand-worked selections in
tests/golden/topk_handworked.txt: ties on score in ascending original
index, non-positive local scores excluded, fewer than K hits, K above the
number of targets, and every target counting in global mode."""
import os

import numpy as np
import pytest

import oracle
from golden_cases import matrix
from workloads import encode
from workloads.gen import SeqSet

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "topk_handworked.txt")


def _ints(field):
    return [int(x) for x in field.split()]


def load():
    lists, searches = [], []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = [x.strip() for x in line.split("|")]
            if f[0] == "search":
                searches.append(dict(query=f[1], K=int(f[2]), targets=f[3].split(),
                                     scores=_ints(f[4]), expected=_ints(f[5])))
            else:
                lists.append(dict(name=f[0], K=int(f[1]), positive_only=bool(int(f[2])),
                                  scores=_ints(f[3]), expected=_ints(f[4])))
    return lists, searches


LISTS, SEARCHES = load()


def test_fixture_is_complete():
    assert len(LISTS) >= 8 and len(SEARCHES) >= 2


@pytest.mark.parametrize("c", LISTS, ids=[c["name"] for c in LISTS])
def test_topk_order(c):
    got = oracle.top_k(np.array(c["scores"], np.int64), c["K"], positive_only=c["positive_only"])
    assert [int(x) for x in got] == c["expected"]


@pytest.mark.parametrize("c", SEARCHES, ids=[f"K{c['K']}" for c in SEARCHES])
def test_search_topk(c):
    S, alpha = matrix("dna23")
    Q = SeqSet.from_list([encode(c["query"], alpha)])
    T = SeqSet.from_list([encode(t, alpha) for t in c["targets"]])
    r = oracle.search(Q, T, S, 5, 2, mode="local", threads=1)
    assert [int(x) for x in r["score"]] == c["scores"]
    got = oracle.top_k(r["score"], c["K"], positive_only=True)
    assert [int(x) for x in got] == c["expected"]
