"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare element by element."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_search(queries, targets, S, o, e, mode="local", ends=None, plain=False,
               force_int32=False, db=None):
    import torch
    import paper_1701_01575_amd as dsa
    if db is None:
        db = dsa.Database.from_seqset(targets, S.shape[0])
    r = dsa.align(queries, db=db, matrix=S, gap_open=o, gap_extend=e, mode=mode,
                  free_ends=ends, plain=plain, force_int32=force_int32)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items() if hasattr(v, "cpu")}, db


def compare_search(got, exp, nq, nt, fields=("score", "q_end", "t_end"), label=""):
    for f in fields:
        g = got[f].astype(np.int64).reshape(nq, nt)
        x = np.asarray(exp[f]).astype(np.int64).reshape(nq, nt)
        bad = np.argwhere(g != x)
        if len(bad):
            q, t = bad[0]
            for qq, tt in bad[:6]:
                print(f"  mismatch q={qq} t={tt}: gpu " +
                      str([int(got[k].reshape(nq, nt)[qq, tt]) for k in ("score", "q_end", "t_end")]) +
                      " oracle " + str([int(np.asarray(exp[k]).reshape(nq, nt)[qq, tt])
                                        for k in ("score", "q_end", "t_end")]), flush=True)
            raise AssertionError(
                f"{label} field {f}: {len(bad)} mismatches; first at query {q} target {t}: "
                f"gpu {g[q, t]} oracle {x[q, t]} (score gpu {got['score'].reshape(nq, nt)[q, t]} "
                f"oracle {np.asarray(exp['score']).reshape(nq, nt)[q, t]})")
