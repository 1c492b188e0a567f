"""Pin the CPU oracle to the definition by enumerating every alignment.

For tiny sequences the brute force lists all alignments allowed by the mode
(local / global / semi-global with free-end flags) and scores each from the
definition.  The oracle must return the best score, the end cell the stated
rule picks among the optimal ones (smallest target end, then smallest query
end), and a CIGAR that is one of the optimal alignments.  The pure-Python
reference must agree with the C oracle exactly, traceback included.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle.pyref import ref_align
from brute import brute, lexmin_end, ops_to_cols, score_columns
from workloads.gen import SeqSet

LOCAL, GLOBAL, SEMI = 0, 1, 2
QB, QE, TB, TE = 1, 2, 4, 8

MODES = [
    ("local", LOCAL, 0),
    ("global", GLOBAL, 0),
    ("semi_tb_te", SEMI, TB | TE),
    ("semi_qb_qe", SEMI, QB | QE),
    ("semi_all", SEMI, QB | QE | TB | TE),
    ("semi_qb_te", SEMI, QB | TE),
]

BIN_SYM = np.array([[2, -1], [-1, 1]], dtype=np.int8)
BIN_ASYM = np.array([[1, -2], [0, 3]], dtype=np.int8)   # row = query code


def _runs(ops):
    return [(int(x) >> 4, oracle.OP_CHARS[int(x) & 15]) for x in ops]


def _check_batch(qs, ts, S, o, e, mode, ends):
    Q = SeqSet.from_list(qs)
    T = SeqSet.from_list(ts)
    res = oracle.align_pairs(Q, T, S, o, e, mode=mode, ends=ends, traceback=True, threads=4)
    for k, (a, b) in enumerate(zip(qs, ts)):
        best, end_set, paths = brute(a, b, S, o, e, mode, ends)
        sc = int(res["score"][k])
        assert sc == best, (a, b, mode, ends, sc, best)
        runs = _runs(res["cigars"][k])
        if mode == LOCAL and best == 0:
            assert (res["q_end"][k], res["t_end"][k], res["q_begin"][k], res["t_begin"][k]) == (-1, -1, -1, -1)
            assert runs == []
            continue
        end = (int(res["q_end"][k]) + 1, int(res["t_end"][k]) + 1)
        assert end == lexmin_end(end_set), (a, b, mode, ends, end, sorted(end_set))
        start = (int(res["q_begin"][k]), int(res["t_begin"][k]))
        cols = ops_to_cols(runs)
        assert (start, cols) in paths, (a, b, mode, ends, start, cols)
        # rescoring the emitted path gives the score, and it ends at the end cell
        r, i1, j1 = score_columns([int(x) for x in a], [int(x) for x in b], S, o, e,
                                  start[0], start[1], cols)
        assert r == sc and (i1, j1) == end
        # '=' exactly where the residues are identical
        i, j = start
        for L, c in runs:
            for _ in range(L):
                if c in "=X":
                    assert (a[i] == b[j]) == (c == "=")
                    i += 1
                    j += 1
                elif c == "I":
                    i += 1
                else:
                    j += 1
        # the separately written Python reference agrees exactly
        py = ref_align(a, b, S, o, e, mode, ends, traceback=True)
        assert py["score"] == sc
        assert (py["q_begin"], py["q_end"], py["t_begin"], py["t_end"]) == (
            start[0], end[0] - 1, start[1], end[1] - 1)
        assert "".join(py["ops"]) == "".join(c * L for L, c in runs)


def _all_binary(maxlen):
    out = []
    for L in range(maxlen + 1):
        out.extend([np.array(t, dtype=np.uint8) for t in itertools.product([0, 1], repeat=L)])
    return out


@pytest.mark.parametrize("name,mode,ends", MODES)
@pytest.mark.parametrize("S", [BIN_SYM, BIN_ASYM], ids=["sym", "asym"])
@pytest.mark.parametrize("o,e", [(2, 1), (1, 1), (0, 0)])
def test_exhaustive_binary(name, mode, ends, S, o, e):
    seqs = _all_binary(3)
    pairs = [(a, b) for a in seqs for b in seqs]
    qs, ts = zip(*pairs)
    _check_batch(list(qs), list(ts), S, o, e, mode, ends)


@pytest.mark.parametrize("name,mode,ends", MODES)
def test_random_dna_len6(name, mode, ends, dna):
    rng = np.random.default_rng([170101575, 7, mode, ends])
    qs, ts = [], []
    for _ in range(40):
        qs.append(rng.integers(0, 5, size=int(rng.integers(0, 7))).astype(np.uint8))
        ts.append(rng.integers(0, 5, size=int(rng.integers(0, 7))).astype(np.uint8))
    _check_batch(qs, ts, dna, 5, 2, mode, ends)


@pytest.mark.parametrize("name,mode,ends", MODES)
def test_random_blosum_len5(name, mode, ends, blosum):
    rng = np.random.default_rng([170101575, 8, mode, ends])
    qs, ts = [], []
    for _ in range(40):
        # a small sub-alphabet makes equal scores (ties) frequent
        qs.append(rng.choice([0, 9, 10, 18], size=int(rng.integers(0, 6))).astype(np.uint8))
        ts.append(rng.choice([0, 9, 10, 18], size=int(rng.integers(0, 6))).astype(np.uint8))
    _check_batch(qs, ts, blosum, 3, 1, mode, ends)


def test_local_never_ends_with_gap_even_when_gaps_are_free():
    S = np.array([[1, -1], [-1, 1]], dtype=np.int8)
    seqs = _all_binary(3)
    pairs = [(a, b) for a in seqs for b in seqs]
    qs, ts = zip(*pairs)
    res = oracle.align_pairs(SeqSet.from_list(qs), SeqSet.from_list(ts), S, 0, 0,
                             mode="local", traceback=True)
    for k in range(len(qs)):
        runs = _runs(res["cigars"][k])
        if runs:
            assert runs[0][1] in "=X" and runs[-1][1] in "=X"
