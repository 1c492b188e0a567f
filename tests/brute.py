"""Brute-force enumeration of every alignment of two tiny sequences.

An alignment is a string of columns: M (a_i against b_j), I (a_i against a
gap) or D (a gap against b_j).  Its score is the sum of the substitution
scores of its M columns minus open + (L-1)*extend for every maximal run of
I's and every maximal run of D's (an I-run next to a D-run counts as two
gaps).  Which alignments are allowed depends on the mode:

* global      a[1..m] against b[1..n] in full;
* local       any substring of a against any substring of b (the empty
              alignment, score 0, included);
* semiglobal  starts at (0,0), at (i,0) if the query begin is free (QB) or at
              (0,j) if the target begin is free (TB); ends at (m,n), at (m,j)
              if the target end is free (TE) or at (i,n) if the query end is
              free (QE).

This is the definition itself; it shares nothing with the dynamic programs.
"""
from __future__ import annotations

LOCAL, GLOBAL, SEMIGLOBAL = 0, 1, 2
QB, QE, TB, TE = 1, 2, 4, 8


def _sub(a, b, S, pssm, i, j):
    """Score of a[i] against b[j]: S[a[i]][b[j]], or with a position-specific
    profile pssm[i][b[j]]."""
    return int(pssm[i][b[j]]) if pssm is not None else int(S[a[i]][b[j]])


def score_columns(a, b, S, o, e, i0, j0, cols, pssm=None):
    """Score of the column string `cols` starting at cell (i0, j0)."""
    i, j = i0, j0
    total = 0
    prev = None
    for c in cols:
        if c == "M":
            total += _sub(a, b, S, pssm, i, j)
            i += 1
            j += 1
        elif c == "I":
            total -= e if prev == "I" else o
            i += 1
        else:
            total -= e if prev == "D" else o
            j += 1
        prev = c
    return total, i, j


def enumerate_alignments(a, b, S, o, e, mode, ends=0, pssm=None):
    """Yield (score, start(i0,j0), end(i1,j1), cols) for every allowed alignment.

    Coordinates are DP cells: the alignment consumes a[i0..i1) and b[j0..j1)."""
    m, n = len(a), len(b)
    if mode == SEMIGLOBAL and not ends:
        ends = TB | TE
    if mode == LOCAL:
        starts = [(i, j) for i in range(m + 1) for j in range(n + 1)]
    elif mode == GLOBAL:
        starts = [(0, 0)]
    else:
        starts = {(0, 0)}
        if ends & QB:
            starts |= {(i, 0) for i in range(m + 1)}
        if ends & TB:
            starts |= {(0, j) for j in range(n + 1)}
        starts = sorted(starts)

    def end_ok(i, j):
        if mode == LOCAL:
            return True
        if (i, j) == (m, n):
            return True
        if mode == SEMIGLOBAL:
            if (ends & TE) and i == m:
                return True
            if (ends & QE) and j == n:
                return True
        return False

    for (i0, j0) in starts:
        # depth-first over column strings, scoring incrementally
        stack = [(i0, j0, None, 0, "")]
        while stack:
            i, j, prev, sc, cols = stack.pop()
            if end_ok(i, j):
                yield sc, (i0, j0), (i, j), cols
            if i < m and j < n:
                stack.append((i + 1, j + 1, "M", sc + _sub(a, b, S, pssm, i, j), cols + "M"))
            if i < m:
                stack.append((i + 1, j, "I", sc - (e if prev == "I" else o), cols + "I"))
            if j < n:
                stack.append((i, j + 1, "D", sc - (e if prev == "D" else o), cols + "D"))


def brute(a, b, S, o, e, mode, ends=0, pssm=None):
    """Best score, the set of end cells attaining it, and the set of optimal
    (start, cols) paths.  Local: score 0 means no alignment (empty sets)."""
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    best = None
    ends_set = set()
    paths = set()
    for sc, st, en, cols in enumerate_alignments(a, b, S, o, e, mode, ends, pssm):
        if best is None or sc > best:
            best = sc
            ends_set = {en}
            paths = {(st, cols)}
        elif sc == best:
            ends_set.add(en)
            paths.add((st, cols))
    if mode == LOCAL:
        if best is None or best <= 0:
            return 0, set(), set()
        # the empty alignment does not define an end cell
    return best, ends_set, paths


def lexmin_end(ends_set):
    """The end cell the stated rule selects: smallest j, then smallest i."""
    return min(ends_set, key=lambda c: (c[1], c[0]))


def ops_to_cols(cigar_runs):
    """[(len, '='|'X'|'I'|'D')] -> column string over M/I/D."""
    out = []
    for L, c in cigar_runs:
        out.append(("M" if c in "=X" else c) * L)
    return "".join(out)
