"""Position-specific scoring in the oracle (a row of scores per query
position in place of the matrix row of its residue; the scoring extension
next to the paper's user-defined algorithm template, Section II.C.2), pinned
by: the profile made of each residue's matrix row gives exactly the matrix
results (score, four coordinates, CIGAR; several queries in one batch, so each
query's rows start at its own offset), brute force over every alignment of
tiny pairs with random profiles (best score, the end cell the rule picks, an
optimal CIGAR), and the separately written Python DP with random profiles."""
import numpy as np
import pytest

import oracle
from brute import brute, lexmin_end, ops_to_cols, score_columns
from oracle.pyref import ref_align, rle
from workloads.gen import SeqSet, random_pairs

CASES = [("local", None), ("global", None), ("semiglobal", None), ("semiglobal", 15),
         ("semiglobal", oracle.QB | oracle.TE)]


def _runs(ops):
    return [(int(x) >> 4, oracle.OP_CHARS[int(x) & 15]) for x in ops]


@pytest.mark.parametrize("mode,ends", CASES)
def test_profile_of_matrix_rows_equals_matrix(mode, ends, blosum):
    Q, T = random_pairs(11, 40, 60, 24, min_len=0)
    prof = blosum[Q.codes]              # row of each query residue
    a = oracle.align_pairs(Q, T, blosum, 11, 1, mode=mode, ends=ends, traceback=True)
    zero = np.zeros_like(blosum)        # the matrix must not be read at all
    b = oracle.align_pairs(Q, T, zero, 11, 1, mode=mode, ends=ends, traceback=True, pssm=prof)
    for f in ("score", "q_begin", "q_end", "t_begin", "t_end"):
        assert (a[f] == b[f]).all(), f
    for x, y in zip(a["cigars"], b["cigars"]):
        assert (x == y).all()
    # search layout: every query against every target, rows by query offset
    s1 = oracle.search(Q.subset(range(5)), T.subset(range(7)), blosum, 11, 1, mode=mode, ends=ends)
    Q5 = Q.subset(range(5))
    s2 = oracle.search(Q5, T.subset(range(7)), zero, 11, 1, mode=mode, ends=ends, pssm=blosum[Q5.codes])
    assert (s1["score"] == s2["score"]).all() and (s1["t_end"] == s2["t_end"]).all()


MODES = [(0, 0), (1, 0), (2, 4 | 8), (2, 1 | 2), (2, 15)]


@pytest.mark.parametrize("mode,ends", MODES)
def test_brute_force_random_profiles(mode, ends):
    rng = np.random.default_rng([170101575, 110, mode, ends])
    S = np.zeros((3, 3), np.int8)
    for _ in range(40):
        m, n = int(rng.integers(0, 5)), int(rng.integers(0, 5))
        a = rng.integers(0, 3, size=m).astype(np.uint8)
        b = rng.integers(0, 3, size=n).astype(np.uint8)
        P = rng.integers(-4, 5, size=(m, 3)).astype(np.int8)
        o = int(rng.integers(0, 5))
        e = int(rng.integers(0, o + 1))
        r = oracle.align_pairs(SeqSet.from_list([a]), SeqSet.from_list([b]), S, o, e, mode=mode,
                               ends=ends or None, traceback=True, threads=1, pssm=P)
        best, end_set, paths = brute(a, b, S, o, e, mode, ends, pssm=P)
        assert int(r["score"][0]) == best
        if mode == 0 and best == 0:
            assert r["q_end"][0] == -1 and len(r["cigars"][0]) == 0
            continue
        i1, j1 = lexmin_end(end_set)
        assert (int(r["q_end"][0]), int(r["t_end"][0])) == (i1 - 1, j1 - 1)
        cols = ops_to_cols(_runs(r["cigars"][0]))
        start = (int(r["q_begin"][0]), int(r["t_begin"][0]))
        assert (start, cols) in paths
        sc, _, _ = score_columns([int(x) for x in a], [int(x) for x in b], S, o, e, start[0], start[1], cols,
                                 pssm=P)
        assert sc == best


@pytest.mark.parametrize("mode,ends", CASES)
def test_c_and_python_agree_with_random_profiles(mode, ends):
    rng = np.random.default_rng([170101575, 111])
    Q, T = random_pairs(12, 30, 40, 20, min_len=1)
    P = rng.integers(-6, 9, size=(len(Q.codes), 20)).astype(np.int8)
    S = np.zeros((20, 20), np.int8)
    r = oracle.align_pairs(Q, T, S, 7, 2, mode=mode, ends=ends, traceback=True, pssm=P)
    m = oracle.MODES[mode]
    for k in range(len(Q)):
        rows = P[Q.offsets[k]:Q.offsets[k + 1]]
        py = ref_align(Q[k], T[k], S, 7, 2, m, oracle.default_ends(m, ends), traceback=True, pssm=rows)
        got = (int(r["score"][k]), int(r["q_begin"][k]), int(r["q_end"][k]), int(r["t_begin"][k]),
               int(r["t_end"][k]))
        assert got == (py["score"], py["q_begin"], py["q_end"], py["t_begin"], py["t_end"]), k
        assert _runs(r["cigars"][k]) == rle(py["ops"]), k
