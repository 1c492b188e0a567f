"""Textbook routines the affine-gap method reduces to in special cases.

Each is written here from its own classic definition, independently of the
oracle:

* longest common subsequence length (global, match 1, mismatch 0, o = e = 0);
* Levenshtein distance (global, match 0, mismatch -1, o = e = 1, negated);
* linear-gap Needleman-Wunsch / Smith-Waterman (o = e);
* Kadane's maximum subarray over every diagonal (local with gaps priced out).
"""
from __future__ import annotations


def lcs_length(a, b):
    m, n = len(a), len(b)
    L = [[0] * (n + 1) for _ in range(m + 1)]
    for i in range(m):
        for j in range(n):
            if a[i] == b[j]:
                L[i + 1][j + 1] = L[i][j] + 1
            else:
                L[i + 1][j + 1] = max(L[i][j + 1], L[i + 1][j])
    return L[m][n]


def levenshtein(a, b):
    m, n = len(a), len(b)
    prev = list(range(n + 1))
    for i in range(1, m + 1):
        cur = [i] + [0] * n
        for j in range(1, n + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (0 if a[i - 1] == b[j - 1] else 1))
        prev = cur
    return prev[n]


def linear_nw(a, b, S, g):
    """Global alignment, each gapped residue costs g."""
    m, n = len(a), len(b)
    D = [[0] * (n + 1) for _ in range(m + 1)]
    for i in range(1, m + 1):
        D[i][0] = -g * i
    for j in range(1, n + 1):
        D[0][j] = -g * j
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            D[i][j] = max(D[i - 1][j - 1] + int(S[a[i - 1]][b[j - 1]]),
                          D[i - 1][j] - g, D[i][j - 1] - g)
    return D[m][n]


def linear_sw(a, b, S, g):
    """Local alignment, each gapped residue costs g."""
    m, n = len(a), len(b)
    D = [[0] * (n + 1) for _ in range(m + 1)]
    best = 0
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            D[i][j] = max(0, D[i - 1][j - 1] + int(S[a[i - 1]][b[j - 1]]),
                          D[i - 1][j] - g, D[i][j - 1] - g)
            best = max(best, D[i][j])
    return best


def kadane_diagonals(a, b, S):
    """max over diagonals of the maximum-sum contiguous run (empty run = 0)."""
    m, n = len(a), len(b)
    best = 0
    for d in range(-m + 1, n):
        run = 0
        for i in range(m):
            j = i + d
            if 0 <= j < n:
                run = max(0, run + int(S[a[i]][b[j]]))
                best = max(best, run)
    return best
