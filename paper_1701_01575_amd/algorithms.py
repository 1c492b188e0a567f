"""The alignment algorithms as a template class (Section II.C.2: the API
offers distributed Smith-Waterman, Needleman-Wunsch and semi-global
alignment, and lets users define their own algorithm by extending a template
class and overriding its implementation).

`Alignment` is the template: an algorithm is its mode, its free ends, its
gap penalties and its scoring, which is a substitution matrix or, per call,
a position-specific profile built from the queries.  `DSW`, `DNW` and `DSG`
are the paper's three algorithms.  A subclass overrides `profile` (or
`matrix`, `mode`, `free_ends`, `gaps`) and every call runs on the same
kernels:

    class ProfileSearch(DSW):
        def profile(self, queries):          # one int8 row per query residue
            return my_pssm(queries)

    hits = ProfileSearch(blosum62).align(queries, db=db, top_k=10, traceback=True)
"""
from __future__ import annotations

import numpy as np


class Alignment:
    """Template of an affine-gap alignment algorithm."""

    mode = "local"
    free_ends = None            # semi-global: a mask of QB | QE | TB | TE

    def __init__(self, matrix, gap_open: int = 11, gap_extend: int = 1):
        self._matrix = np.ascontiguousarray(matrix, dtype=np.int8)
        self.gap_open, self.gap_extend = int(gap_open), int(gap_extend)

    # -- the parts a subclass overrides ---------------------------------
    def matrix(self) -> np.ndarray:
        """Substitution scores, row = query code, column = target code."""
        return self._matrix

    def profile(self, queries):
        """Position-specific scores for these queries (one row of alphabet
        size scores per query residue, in the order of queries.codes), or
        None to score with the matrix."""
        return None

    def gaps(self):
        """(open, extend): a gap of L columns costs open + (L - 1) * extend."""
        return self.gap_open, self.gap_extend

    # -- the call ----------------------------------------------------------
    def align(self, queries, db=None, targets=None, top_k=0, traceback=False, **kw) -> dict:
        from . import align
        o, e = self.gaps()
        return align(queries, db=db, targets=targets, matrix=self.matrix(), gap_open=o, gap_extend=e,
                     mode=self.mode, free_ends=self.free_ends, traceback=traceback, top_k=top_k,
                     pssm=self.profile(queries), **kw)


class DSW(Alignment):
    """Smith-Waterman: the best local alignment."""
    mode = "local"


class DNW(Alignment):
    """Needleman-Wunsch: both sequences end to end."""
    mode = "global"


class DSG(Alignment):
    """Semi-global: the query end to end, the target's ends free (by default)."""
    mode = "semiglobal"

    def __init__(self, matrix, gap_open: int = 11, gap_extend: int = 1, free_ends=None):
        super().__init__(matrix, gap_open, gap_extend)
        self.free_ends = free_ends
