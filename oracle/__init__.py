"""CPU oracle for affine-gap alignment (local, global, semi-global).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library.

Two independent implementations live here:

* ``gotoh.c`` (built into ``liboracle.so`` with gcc): plain int64 O(m*n)
  dynamic programming, full matrices for traceback, a pthread pool over pairs.
* ``pyref.py``: a separately written pure-Python version (small inputs only)
  used to cross-check the C code, including its traceback.

Conventions (the paper leaves them open; see the module docstring of
``gotoh.c``): a gap of length L costs open + (L-1)*extend; end cell = best
score, then smallest target end, then smallest query end; traceback priority
zero > diagonal > D > I, open wins ties; CIGAR ops use the BAM numbering
(= 7, X 8, I 1, D 2), len << 4 | op.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

LOCAL, GLOBAL, SEMIGLOBAL = 0, 1, 2
QB, QE, TB, TE = 1, 2, 4, 8
MODES = {"local": LOCAL, "global": GLOBAL, "semiglobal": SEMIGLOBAL}
OP_I, OP_D, OP_EQ, OP_X = 1, 2, 7, 8
OP_CHARS = {OP_I: "I", OP_D: "D", OP_EQ: "=", OP_X: "X"}

_lib = None


SAN_LIB_PATH = os.path.join(HERE, "liboracle_san.so")


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile gotoh.c into liboracle.so with gcc (with sanitize: an
    AddressSanitizer + UndefinedBehaviorSanitizer build, liboracle_san.so)."""
    src = os.path.join(HERE, "gotoh.c")
    path = SAN_LIB_PATH if sanitize else LIB_PATH
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        tmp = path + ".tmp"
        flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
        subprocess.check_call(["gcc", *flags, "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-o", tmp, src])
        os.replace(tmp, path)
    return path


def lib():
    """The oracle library; DSA_ORACLE_SANITIZED=1 loads the sanitizer build
    (the process must preload the sanitizer runtimes)."""
    global _lib
    if _lib is None:
        san = os.environ.get("DSA_ORACLE_SANITIZED") == "1"
        path = build(sanitize=san)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.or_align_batch.restype = ctypes.c_int
        L.or_align_batch.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, P, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def default_threads() -> int:
    """Worker threads of a batch: the cores this process may run on, at most
    DSA_ORACLE_THREADS (default 16, a one-GPU machine's share of its host)."""
    cap = int(os.environ.get("DSA_ORACLE_THREADS", "16"))
    return max(1, min(len(os.sched_getaffinity(0)), cap))


def default_ends(mode: int, ends) -> int:
    if mode == SEMIGLOBAL:
        return TB | TE if not ends else int(ends)
    return 0


def align_index(qi, ti, queries, targets, matrix, gap_open, gap_extend, mode="local",
                ends=None, traceback=False, threads=None, pssm=None) -> dict:
    """Align pairs (queries[qi[k]], targets[ti[k]]) with the C oracle.

    queries/targets: objects with .codes (uint8) and .offsets (int64, n+1).
    pssm: optional (total query residues, alphabet) int8 scores, one row per
    query residue in the order of queries.codes, used instead of the matrix.
    Returns a dict of numpy arrays: score (int64), q_begin, q_end, t_begin,
    t_end (int32) and, with traceback, cigars (list of uint32 arrays)."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    qi = np.ascontiguousarray(qi, dtype=np.int64)
    ti = np.ascontiguousarray(ti, dtype=np.int64)
    n = len(qi)
    S = np.ascontiguousarray(matrix, dtype=np.int8)
    A = S.shape[0]
    if pssm is not None:
        pssm = np.ascontiguousarray(pssm, dtype=np.int8)
        if pssm.shape != (len(queries.codes), A):
            raise ValueError("pssm must have one row of alphabet-size scores per query residue")
    if threads is None:
        threads = default_threads()
    score = np.zeros(n, np.int64)
    coords = np.zeros((n, 4), np.int32)
    n_ops = np.zeros(n, np.int32)
    status = np.zeros(n, np.int32)
    cig = cig_off = cig_cap = None
    if traceback:
        ql = (queries.offsets[qi + 1] - queries.offsets[qi])
        tl = (targets.offsets[ti + 1] - targets.offsets[ti])
        cig_cap = (ql + tl + 1).astype(np.int64)
        cig_off = np.zeros(n, np.int64)
        if n:
            cig_off[1:] = np.cumsum(cig_cap)[:-1]
        cig = np.zeros(int(cig_cap.sum()) if n else 1, np.uint32)
    rc = lib().or_align_batch(n, _ptr(qi), _ptr(ti), _ptr(queries.codes), _ptr(queries.offsets),
                              _ptr(targets.codes), _ptr(targets.offsets), _ptr(S), _ptr(pssm), A,
                              int(gap_open), int(gap_extend), m, default_ends(m, ends),
                              1 if traceback else 0, int(threads), _ptr(score), _ptr(coords),
                              _ptr(n_ops), _ptr(status), _ptr(cig), _ptr(cig_off), _ptr(cig_cap))
    if rc != 0:
        raise RuntimeError(f"oracle failed with code {rc}")
    out = dict(score=score, q_begin=coords[:, 0].copy(), q_end=coords[:, 1].copy(),
               t_begin=coords[:, 2].copy(), t_end=coords[:, 3].copy())
    if traceback:
        out["cigars"] = [cig[cig_off[k]:cig_off[k] + n_ops[k]].copy() for k in range(n)]
    return out


def align_pairs(queries, targets, matrix, gap_open, gap_extend, mode="local", ends=None,
                traceback=False, threads=None, pssm=None) -> dict:
    """Pairwise: queries[k] vs targets[k]."""
    n = len(queries.offsets) - 1
    idx = np.arange(n, dtype=np.int64)
    return align_index(idx, idx, queries, targets, matrix, gap_open, gap_extend, mode, ends,
                       traceback, threads, pssm)


def search(queries, targets, matrix, gap_open, gap_extend, mode="local", ends=None,
           traceback=False, threads=None, pssm=None) -> dict:
    """Every query vs every target, results query-major (n_q * n_t)."""
    nq = len(queries.offsets) - 1
    nt = len(targets.offsets) - 1
    qi = np.repeat(np.arange(nq, dtype=np.int64), nt)
    ti = np.tile(np.arange(nt, dtype=np.int64), nq)
    return align_index(qi, ti, queries, targets, matrix, gap_open, gap_extend, mode, ends,
                       traceback, threads, pssm)


def cigar_string(ops) -> str:
    return "".join(f"{int(x) >> 4}{OP_CHARS[int(x) & 15]}" for x in ops)


def top_k(scores: np.ndarray, k: int, positive_only: bool = True):
    """Top-k target indices of one query (Section II.B.2: the k best
    alignments by maximum score), by (score desc, index asc): a full stable
    sort of the oracle's per-target scores.  With positive_only (local mode)
    scores <= 0, which mean "no alignment", are left out; in global and
    semi-global mode every target counts."""
    scores = np.asarray(scores).astype(np.int64)
    order = np.lexsort((np.arange(len(scores)), -scores))
    if positive_only:
        order = order[scores[order] > 0]
    return order[:k]
