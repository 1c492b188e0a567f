"""Invariants of the alignment scores, checked on the oracle with hypothesis.

local >= 0; global <= semi-global(target ends free) <= local; swap symmetry
under a symmetric matrix (local, global; semi-global with free target ends
vs free query ends); reversal symmetry (local, global, all-ends-free
semi-global); scores never increase with the gap open or extend penalty;
local(a, b) >= local(a, b') for b' a substring of b; local is bounded by the
sum of positive row maxima and of positive column maxima.  Every CIGAR the
oracle emits rescores to its score.  Every prefix of a local alignment that
ends on an =/X column scores above zero (the traceback stops at a zero
cell before it takes any other step).
"""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from brute import score_columns, ops_to_cols
from workloads.gen import SeqSet

SETTINGS = dict(max_examples=60, deadline=None, derandomize=True)

seq = st.lists(st.integers(0, 19), min_size=0, max_size=40).map(lambda v: np.array(v, np.uint8))
gaps = st.tuples(st.integers(0, 12), st.integers(0, 12)).map(lambda t: (max(t), min(t)))


def one(a, b, S, o, e, mode, ends=None, tb=False):
    r = oracle.align_pairs(SeqSet.from_list([a]), SeqSet.from_list([b]), S, o, e, mode=mode,
                           ends=ends, traceback=tb, threads=1)
    return {k: (v[0] if not isinstance(v, list) else v[0]) for k, v in r.items()}


@settings(**SETTINGS)
@given(seq, seq, gaps)
def test_mode_ordering(a, b, g):
    from workloads import blosum62
    S = blosum62()
    o, e = g
    loc = one(a, b, S, o, e, "local")["score"]
    glo = one(a, b, S, o, e, "global")["score"]
    semi = one(a, b, S, o, e, "semiglobal")["score"]
    assert loc >= 0
    assert glo <= semi <= loc


@settings(**SETTINGS)
@given(seq, seq, gaps)
def test_swap_symmetry(a, b, g):
    from workloads import blosum62
    S = blosum62()
    o, e = g
    for mode in ("local", "global"):
        assert one(a, b, S, o, e, mode)["score"] == one(b, a, S, o, e, mode)["score"]
    assert one(a, b, S, o, e, "semiglobal", ends=oracle.TB | oracle.TE)["score"] == \
        one(b, a, S, o, e, "semiglobal", ends=oracle.QB | oracle.QE)["score"]


@settings(**SETTINGS)
@given(seq, seq, gaps)
def test_reversal_symmetry(a, b, g):
    from workloads import blosum62
    S = blosum62()
    o, e = g
    ra, rb = a[::-1].copy(), b[::-1].copy()
    for mode, ends in (("local", None), ("global", None), ("semiglobal", 15)):
        assert one(a, b, S, o, e, mode, ends)["score"] == one(ra, rb, S, o, e, mode, ends)["score"]


@settings(**SETTINGS)
@given(seq, seq, gaps, st.integers(0, 5))
def test_monotone_in_penalties(a, b, g, d):
    from workloads import blosum62
    S = blosum62()
    o, e = g
    for mode in ("local", "global", "semiglobal"):
        base = one(a, b, S, o, e, mode)["score"]
        assert one(a, b, S, o + d, e, mode)["score"] <= base
        assert one(a, b, S, o + d, min(e + d, o + d), mode)["score"] <= base


@settings(**SETTINGS)
@given(seq, seq, gaps, st.integers(0, 40), st.integers(0, 40))
def test_local_substring_and_bounds(a, b, g, i, j):
    from workloads import blosum62
    S = blosum62()
    o, e = g
    lo, hi = sorted((min(i, len(b)), min(j, len(b))))
    full = one(a, b, S, o, e, "local")["score"]
    assert full >= one(a, b[lo:hi].copy(), S, o, e, "local")["score"]
    rowmax = sum(max(0, int(S[x].max())) for x in a)
    colmax = sum(max(0, int(S[:, y].max())) for y in b)
    assert full <= min(rowmax, colmax)


@settings(**SETTINGS)
@given(seq, seq, gaps, st.sampled_from(["local", "global", "semiglobal"]))
def test_cigar_rescores(a, b, g, mode):
    from workloads import blosum62
    S = blosum62()
    o, e = g
    r = one(a, b, S, o, e, mode, tb=True)
    runs = [(int(x) >> 4, oracle.OP_CHARS[int(x) & 15]) for x in r["cigars"]]
    if mode == "local" and r["score"] == 0:
        assert runs == [] and r["q_end"] == -1
        return
    cols = ops_to_cols(runs)
    sc, i1, j1 = score_columns([int(x) for x in a], [int(x) for x in b], S, o, e,
                               int(r["q_begin"]), int(r["t_begin"]), cols)
    assert sc == r["score"]
    assert (i1 - 1, j1 - 1) == (r["q_end"], r["t_end"])
    if mode == "global":
        assert (r["q_begin"], r["t_begin"]) == (0, 0)
        assert (r["q_end"], r["t_end"]) == (len(a) - 1, len(b) - 1)
    if mode == "semiglobal":
        assert r["q_begin"] == 0 and r["q_end"] == len(a) - 1
    if mode == "local":
        assert runs[0][1] in "=X" and runs[-1][1] in "=X"


dna_seq = st.lists(st.integers(0, 3), min_size=0, max_size=40).map(lambda v: np.array(v, np.uint8))


@settings(**SETTINGS)
@given(st.one_of(st.tuples(seq, seq, st.just("protein")), st.tuples(dna_seq, dna_seq, st.just("dna"))),
       gaps)
def test_local_positive_prefixes(ab, g):
    """Scored from the definition (brute.score_columns), each prefix of the
    reported local alignment that ends on a match or mismatch column is
    positive: the traceback stops at a zero cell before any other step, so
    it never passes through a cell whose best score is <= 0.  Each suffix
    that starts on such a column is positive too: otherwise the part before
    it would score at least as much and end at a smaller target position,
    which the end-cell rule (smallest target end among the best) would have
    chosen."""
    from workloads import blosum62, dna_matrix
    a, b, kind = ab
    S = blosum62() if kind == "protein" else dna_matrix(2, -3)
    o, e = g
    r = one(a, b, S, o, e, "local", tb=True)
    if r["score"] == 0:
        return
    cols = ops_to_cols([(int(x) >> 4, oracle.OP_CHARS[int(x) & 15]) for x in r["cigars"]])
    A, B = [int(x) for x in a], [int(x) for x in b]
    i0, j0 = int(r["q_begin"]), int(r["t_begin"])
    for k in range(1, len(cols) + 1):
        if cols[k - 1] == "M":
            sc, _, _ = score_columns(A, B, S, o, e, i0, j0, cols[:k])
            assert sc > 0, (cols, k, sc)
    i, j = i0, j0
    for k in range(len(cols)):
        if cols[k] == "M":
            sc, _, _ = score_columns(A, B, S, o, e, i, j, cols[k:])
            assert sc > 0, (cols, k, sc)
        i += cols[k] in "MI"
        j += cols[k] in "MD"
