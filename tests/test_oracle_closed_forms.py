"""Pin the oracle to closed forms and textbook special cases.

* all-gap alignments: global("", b) = -(o + (n-1)e), and the empty cases of
  every mode;
* self-alignment = sum of the diagonal substitution scores when the matrix
  satisfies S[x][y] <= (S[x][x] + S[y][y]) / 2 and S[x][x] > 0;
* o = e = 0, match 1, mismatch 0, global  -> longest common subsequence;
* o = e = 1, match 0, mismatch -1, global -> minus the Levenshtein distance;
* o = e = g -> linear-gap Needleman-Wunsch / Smith-Waterman;
* gaps priced out (o = e huge): local = best diagonal run (Kadane), global
  of equal lengths = sum along the main diagonal.
"""
import numpy as np
import pytest

import oracle
from textbook import kadane_diagonals, lcs_length, levenshtein, linear_nw, linear_sw
from workloads.gen import SeqSet


def run(qs, ts, S, o, e, mode, ends=None, tb=False):
    return oracle.align_pairs(SeqSet.from_list(qs), SeqSet.from_list(ts), S, o, e,
                              mode=mode, ends=ends, traceback=tb, threads=4)


def rand_seqs(seed, n, lo, hi, alphabet):
    rng = np.random.default_rng([170101575, 11, seed])
    return [rng.integers(0, alphabet, size=int(rng.integers(lo, hi + 1))).astype(np.uint8)
            for _ in range(n)]


@pytest.mark.parametrize("o,e", [(11, 1), (10, 1), (5, 2), (3, 3)])
def test_all_gap_closed_forms(o, e, blosum):
    lens = [0, 1, 2, 7, 40]
    emp = np.zeros(0, np.uint8)
    seqs = [np.full(L, 4, np.uint8) for L in lens]
    g = lambda L: 0 if L == 0 else o + (L - 1) * e
    r = run([emp] * len(seqs), seqs, blosum, o, e, "global", tb=True)
    assert list(r["score"]) == [-g(L) for L in lens]
    for k, L in enumerate(lens):
        assert oracle.cigar_string(r["cigars"][k]) == (f"{L}D" if L else "")
    r = run(seqs, [emp] * len(seqs), blosum, o, e, "global")
    assert list(r["score"]) == [-g(L) for L in lens]
    # local with an empty side: no alignment
    r = run([emp] * len(seqs), seqs, blosum, o, e, "local")
    assert list(r["score"]) == [0] * len(lens)
    assert list(r["q_end"]) == [-1] * len(lens)
    # semi-global with free target ends: ("", b) = 0 and (a, "") = -(o+(m-1)e)
    r = run([emp] * len(seqs), seqs, blosum, o, e, "semiglobal")
    assert list(r["score"]) == [0] * len(lens)
    r = run(seqs, [emp] * len(seqs), blosum, o, e, "semiglobal")
    assert list(r["score"]) == [-g(L) for L in lens]


def test_blosum62_satisfies_self_alignment_condition(blosum):
    S = blosum[:20, :20].astype(int)
    for x in range(20):
        assert S[x, x] > 0
        for y in range(20):
            assert 2 * S[x, y] <= S[x, x] + S[y, y]
    # the condition fails for X, whose diagonal is negative
    assert blosum[22, 22] < 0


@pytest.mark.parametrize("mode", ["local", "global", "semiglobal"])
def test_self_alignment_blosum(mode, blosum):
    seqs = rand_seqs(1, 60, 1, 120, 20)
    r = run(seqs, seqs, blosum, 11, 1, mode, tb=True)
    for k, a in enumerate(seqs):
        assert r["score"][k] == sum(int(blosum[c, c]) for c in a)
        assert oracle.cigar_string(r["cigars"][k]) == f"{len(a)}="
        assert (r["q_begin"][k], r["q_end"][k], r["t_begin"][k], r["t_end"][k]) == (0, len(a) - 1, 0, len(a) - 1)


def test_self_alignment_dna(dna):
    seqs = rand_seqs(2, 60, 1, 200, 4)
    r = run(seqs, seqs, dna, 5, 2, "local")
    assert list(r["score"]) == [2 * len(a) for a in seqs]


def test_lcs_reduction():
    S = np.array([[1 if x == y else 0 for y in range(4)] for x in range(4)], dtype=np.int8)
    qs = rand_seqs(3, 80, 0, 25, 4)
    ts = rand_seqs(4, 80, 0, 25, 4)
    r = run(qs, ts, S, 0, 0, "global")
    assert list(r["score"]) == [lcs_length(list(a), list(b)) for a, b in zip(qs, ts)]


def test_levenshtein_reduction():
    S = np.array([[0 if x == y else -1 for y in range(4)] for x in range(4)], dtype=np.int8)
    qs = rand_seqs(5, 80, 0, 25, 4)
    ts = rand_seqs(6, 80, 0, 25, 4)
    r = run(qs, ts, S, 1, 1, "global")
    assert list(r["score"]) == [-levenshtein(list(a), list(b)) for a, b in zip(qs, ts)]


@pytest.mark.parametrize("g", [1, 4, 8])
def test_linear_gap_reduction(g, blosum):
    qs = rand_seqs(7 + g, 50, 0, 30, 20)
    ts = rand_seqs(17 + g, 50, 0, 30, 20)
    r = run(qs, ts, blosum, g, g, "global")
    assert list(r["score"]) == [linear_nw(a, b, blosum, g) for a, b in zip(qs, ts)]
    r = run(qs, ts, blosum, g, g, "local")
    assert list(r["score"]) == [linear_sw(a, b, blosum, g) for a, b in zip(qs, ts)]


def test_gaps_priced_out(blosum):
    big = 1_000_000
    qs = rand_seqs(30, 60, 1, 30, 20)
    ts = rand_seqs(31, 60, 1, 30, 20)
    r = run(qs, ts, blosum, big, big, "local")
    assert list(r["score"]) == [kadane_diagonals(a, b, blosum) for a, b in zip(qs, ts)]
    ts_eq = [t[:len(q)] if len(t) >= len(q) else np.resize(t, len(q)) for q, t in zip(qs, ts)]
    r = run(qs, ts_eq, blosum, big, big, "global")
    assert list(r["score"]) == [sum(int(blosum[x, y]) for x, y in zip(a, b)) for a, b in zip(qs, ts_eq)]
