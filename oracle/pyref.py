"""Second, separately written oracle in pure Python (small inputs only).

TEST INFRASTRUCTURE ONLY.  It exists to cross-check ``gotoh.c``: same
definitions (affine gaps costing open + (L-1)*extend; local, global and
semi-global with free-end flags; end cell = best score, then smallest target
end, then smallest query end; traceback priority zero > diagonal > D > I with
open winning ties), written with a different structure: the three matrices
are filled column by column, and the path is recovered by a state machine
over explicit predecessor tests.
"""
from __future__ import annotations

LOCAL, GLOBAL, SEMIGLOBAL = 0, 1, 2
QB, QE, TB, TE = 1, 2, 4, 8
NEG = -(1 << 60)


def _gap(o, e, L):
    return 0 if L == 0 else o + (L - 1) * e


def ref_align(a, b, S, o, e, mode=LOCAL, ends=0, traceback=True, pssm=None):
    """Returns dict(score, q_begin, q_end, t_begin, t_end, ops) where ops is
    a forward list of op characters ('=', 'X', 'I', 'D') or None.  With pssm
    (a row of scores per query position) residue i of a scores pssm[i][c]
    against target code c instead of S[a[i]][c]."""
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    if pssm is None:
        def sub(i, j):  # 1-based cell
            return int(S[a[i - 1]][b[j - 1]])
    else:
        def sub(i, j):
            return int(pssm[i - 1][b[j - 1]])
    m, n = len(a), len(b)
    if mode == SEMIGLOBAL and not ends:
        ends = TB | TE
    if mode != SEMIGLOBAL:
        ends = 0
    loc = mode == LOCAL

    def top(j):  # H[0][j]
        if j == 0 or loc or (ends & TB):
            return 0
        return -_gap(o, e, j)

    def left(i):  # H[i][0]
        if i == 0 or loc or (ends & QB):
            return 0
        return -_gap(o, e, i)

    H = [[0] * (n + 1) for _ in range(m + 1)]
    E = [[NEG] * (n + 1) for _ in range(m + 1)]
    F = [[NEG] * (n + 1) for _ in range(m + 1)]
    for j in range(n + 1):
        H[0][j] = top(j)
    for i in range(m + 1):
        H[i][0] = left(i)
    for j in range(1, n + 1):          # column by column
        for i in range(1, m + 1):
            E[i][j] = max(E[i][j - 1] - e, H[i][j - 1] - o)
            F[i][j] = max(F[i - 1][j] - e, H[i - 1][j] - o)
            cand = [H[i - 1][j - 1] + sub(i, j), E[i][j], F[i][j]]
            if loc:
                cand.append(0)
            H[i][j] = max(cand)

    # candidate end cells in (j, i) order; strictly-greater keeps the first
    if loc:
        cells = [(i, j) for j in range(1, n + 1) for i in range(1, m + 1)]
    else:
        cs = {(m, n)}
        if ends & TE:
            cs |= {(m, j) for j in range(n + 1)}
        if ends & QE:
            cs |= {(i, n) for i in range(m + 1)}
        cells = sorted(cs, key=lambda c: (c[1], c[0]))
    best, end = None, None
    for (i, j) in cells:
        if best is None or H[i][j] > best:
            best, end = H[i][j], (i, j)
    if loc and best is not None and best <= 0:
        best = None
    if best is None:
        if loc:
            return dict(score=0, q_begin=-1, q_end=-1, t_begin=-1, t_end=-1,
                        ops=[] if traceback else None)
    score = best
    i, j = end
    out = dict(score=score, q_end=i - 1, t_end=j - 1, q_begin=-1, t_begin=-1, ops=None)
    if not traceback:
        return out

    ops = []
    state = "H"
    while True:
        if state == "H":
            h = H[i][j]
            if loc and h == 0:
                break
            if i == 0 or j == 0:
                if i == 0 and j == 0:
                    break
                if i == 0:
                    if ends & TB:
                        break
                    ops.extend("D" * j)
                    j = 0
                else:
                    if ends & QB:
                        break
                    ops.extend("I" * i)
                    i = 0
                break
            s = sub(i, j)
            if h == H[i - 1][j - 1] + s:
                ops.append("=" if a[i - 1] == b[j - 1] else "X")
                i, j = i - 1, j - 1
            elif h == E[i][j]:
                state = "E"
            else:
                assert h == F[i][j]
                state = "F"
        elif state == "E":
            ops.append("D")
            opened = E[i][j] == H[i][j - 1] - o
            assert opened or E[i][j] == E[i][j - 1] - e
            j -= 1
            if opened:
                state = "H"
        else:
            ops.append("I")
            opened = F[i][j] == H[i - 1][j] - o
            assert opened or F[i][j] == F[i - 1][j] - e
            i -= 1
            if opened:
                state = "H"
    ops.reverse()
    out.update(q_begin=i, t_begin=j, ops=ops)
    return out


def rle(ops):
    """Forward op characters -> list of (length, char)."""
    runs = []
    for c in ops:
        if runs and runs[-1][1] == c:
            runs[-1][0] += 1
        else:
            runs.append([1, c])
    return [(k, c) for k, c in runs]
