"""The C oracle and the separately written Python reference agree exactly
(score, four coordinates, CIGAR) on random and related pairs, every mode."""
import numpy as np
import pytest

import oracle
from oracle.pyref import ref_align, rle
from workloads.gen import SeqSet, random_pairs, related_pairs

CASES = [
    ("local", None), ("global", None), ("semiglobal", None),
    ("semiglobal", oracle.QB | oracle.QE), ("semiglobal", 15), ("semiglobal", oracle.TB | oracle.QE),
]


def _compare(Q, T, S, o, e, mode, ends):
    r = oracle.align_pairs(Q, T, S, o, e, mode=mode, ends=ends, traceback=True, threads=8)
    m = oracle.MODES[mode]
    for k in range(len(Q)):
        py = ref_align(Q[k], T[k], S, o, e, m, oracle.default_ends(m, ends), traceback=True)
        got = (int(r["score"][k]), int(r["q_begin"][k]), int(r["q_end"][k]),
               int(r["t_begin"][k]), int(r["t_end"][k]))
        exp = (py["score"], py["q_begin"], py["q_end"], py["t_begin"], py["t_end"])
        assert got == exp, (k, mode, ends, got, exp)
        runs = [(int(x) >> 4, oracle.OP_CHARS[int(x) & 15]) for x in r["cigars"][k]]
        assert runs == rle(py["ops"]), (k, mode, ends)


@pytest.mark.parametrize("mode,ends", CASES)
def test_random_protein(mode, ends, blosum):
    Q, T = random_pairs(1, 60, 40, 24)
    _compare(Q, T, blosum, 11, 1, mode, ends)


@pytest.mark.parametrize("mode,ends", CASES)
def test_related_protein(mode, ends, blosum):
    Q, T = related_pairs(2, 25, 20, 80)
    _compare(Q, T, blosum, 10, 1, mode, ends)


@pytest.mark.parametrize("mode,ends", CASES)
def test_random_dna_small_alphabet(mode, ends, dna):
    Q, T = random_pairs(3, 80, 30, 2)
    _compare(Q, T, dna, 5, 2, mode, ends)


def test_search_layout_is_query_major(blosum):
    Q, T = random_pairs(4, 3, 20, 20, min_len=1)
    r = oracle.search(Q, T, blosum, 11, 1)
    for q in range(3):
        for t in range(3):
            py = ref_align(Q[q], T[t], blosum, 11, 1, 0, 0, traceback=False)
            assert r["score"][q * 3 + t] == py["score"]
