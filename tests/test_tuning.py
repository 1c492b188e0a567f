"""Tuning table and its JSON cache (host logic; no GPU): a cache file named
by DSA_AUTOTUNE_CACHE is read once and applies to calls of the same shape
class only, environment variables override it, and text the reader does not
understand is skipped.  Pairwise planning needs no device, so the effect is
visible through dsa_tuning_get and dsa_workspace_size."""
import ctypes
import json
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ARGS_SRC = textwrap.dedent("""
    import ctypes, sys, json
    import numpy as np
    sys.path.insert(0, {root!r})
    from paper_1701_01575_amd import binding as B

    def make(m, n, k):
        a = B.dsa_args()
        qo = np.arange(k + 1, dtype=np.int64) * m
        to = np.arange(k + 1, dtype=np.int64) * n
        S = np.eye(4, dtype=np.int8) * 3 - 1
        a.q_codes = 1  # planning never reads device memory
        a.q_offsets = qo.ctypes.data
        a.n_q = k
        a.t_codes = 1
        a.t_offsets = to.ctypes.data
        a.subst = S.ctypes.data
        a.alphabet_size = 4
        a.gap_open = 5
        a.gap_extend = 2
        a.mode = B.DSA_GLOBAL
        a.flags = B.DSA_TRACEBACK
        a._keep = (qo, to, S)
        return a

    def ws(a):
        n = ctypes.c_size_t()
        assert B.lib().dsa_workspace_size(ctypes.byref(a), ctypes.byref(n)) == 0, B.dsa_last_error()
        return n.value
""")


def _run(code, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    src = ARGS_SRC.format(root=ROOT) + textwrap.dedent(code)
    r = subprocess.run([sys.executable, "-c", src], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_key_and_defaults():
    out = _run("""
        a, b = make(300, 400, 5), make(40, 50, 5)
        print(json.dumps({"ka": B.dsa_tuning_key(a), "kb": B.dsa_tuning_key(b),
                          "ta": B.dsa_tuning_get(a), "wsa": ws(a)}))
    """, {})
    assert out["ka"].startswith("pairs/") and out["ka"] != out["kb"]
    assert out["ta"]["pair_rows"] == 48 and out["ta"]["pair_cells"] == 32768 and out["ta"]["ms"] == 0


def test_cache_applies_to_its_class_only(tmp_path):
    keys = _run("""
        print(json.dumps({"ka": B.dsa_tuning_key(make(300, 400, 5)), "kb": B.dsa_tuning_key(make(40, 50, 5)),
                          "wsa": ws(make(300, 400, 5))}))
    """, {})
    cache = tmp_path / "tune.json"
    entries = [{"key": keys["ka"], "strip": 0, "waves": 0, "intra_budget": -1, "pair_rows": 1 << 30,
                "pair_cells": 0, "ms": 1.25},
               {"key": "pairs/something/else", "pair_rows": 7}]
    cache.write_text("garbage before\n" + json.dumps(entries, indent=1) + "\n{not an entry}\n")
    out = _run("""
        a, b = make(300, 400, 5), make(40, 50, 5)
        print(json.dumps({"ta": B.dsa_tuning_get(a), "tb": B.dsa_tuning_get(b), "wsa": ws(a)}))
    """, {"DSA_AUTOTUNE_CACHE": str(cache)})
    assert out["ta"]["pair_rows"] == 1 << 30 and out["ta"]["pair_cells"] == 0 and out["ta"]["ms"] == 1.25
    assert out["tb"]["pair_rows"] == 48  # other class: defaults
    # every pair now goes to the lane-per-pair kernel: a different workspace
    assert out["wsa"] != keys["wsa"]


def test_environment_overrides_cache(tmp_path):
    key = _run("""print(json.dumps({"k": B.dsa_tuning_key(make(300, 400, 5))}))""", {})["k"]
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps([{"key": key, "pair_rows": 1 << 30, "pair_cells": 0}]))
    out = _run("""print(json.dumps(B.dsa_tuning_get(make(300, 400, 5))))""",
               {"DSA_AUTOTUNE_CACHE": str(cache), "DSA_PAIR_WF_ROWS": "128"})
    assert out["pair_rows"] == 128 and out["pair_cells"] == 0


def test_missing_cache_file_is_ignored(tmp_path):
    out = _run("""print(json.dumps(B.dsa_tuning_get(make(300, 400, 5))))""",
               {"DSA_AUTOTUNE_CACHE": str(tmp_path / "absent.json")})
    assert out["pair_rows"] == 48
