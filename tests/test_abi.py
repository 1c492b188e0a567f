"""The C ABI: the library loads, exports every function include/dsa.h
declares, and rejects bad arguments with the documented status before any
device work (these calls need no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dsa.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*|int32_t)\s*\*?\s*(dsa_\w+)\(", src, re.M)))


@pytest.fixture(scope="module")
def B():
    from paper_1701_01575_amd import binding
    return binding


def test_every_declared_symbol_is_exported(B):
    names = _declared()
    assert {"dsa_align_batch", "dsa_db_create", "dsa_workspace_size"} <= set(names)
    L = B.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(B.EXPORTS) == names
    assert B.dsa_abi_version() == B.ABI_VERSION == 4


def test_strerror(B):
    assert B.dsa_strerror(0) == "ok"
    assert B.dsa_strerror(B.DSA_E_NOTSUP) == "not supported"


def _args(B, **kw):
    a = B.dsa_args()
    qo = np.array([0, 3], np.int64)
    S = np.zeros((4, 4), np.int8)
    a.q_codes = 1  # never dereferenced by the checks below
    a.q_offsets = qo.ctypes.data
    a.n_q = 1
    a.t_codes = 1
    a.t_offsets = qo.ctypes.data
    a.subst = S.ctypes.data
    a.alphabet_size = 4
    a.gap_open = 5
    a.gap_extend = 2
    a.mode = B.DSA_LOCAL
    for k, v in kw.items():
        setattr(a, k, v)
    a._keep = (qo, S)
    return a


@pytest.mark.parametrize("kw,status", [
    (dict(gap_extend=6), 1),
    (dict(gap_open=-1), 1),
    (dict(mode=7), 1),
    (dict(alphabet_size=70), 1),
    (dict(free_ends=4), 1),          # free ends outside semiglobal
    (dict(flags=64), 1),
    (dict(n_q=0), 1),
])
def test_invalid_arguments(B, kw, status):
    a = _args(B, **kw)
    n = ctypes.c_size_t()
    assert B.lib().dsa_workspace_size(ctypes.byref(a), ctypes.byref(n)) == status
    assert B.dsa_last_error()


def test_db_create_validates_before_allocating(B):
    codes = np.array([0, 1, 9], np.uint8)
    offs = np.array([0, 3], np.int64)
    h = ctypes.c_void_p()
    st = B.lib().dsa_db_create(codes.ctypes.data, offs.ctypes.data, 1, 4, None, None, ctypes.byref(h))
    assert st == B.DSA_E_INVAL and "alphabet" in B.dsa_last_error()
    bad = np.array([0, 5, 3], np.int64)
    st = B.lib().dsa_db_create(codes.ctypes.data, bad.ctypes.data, 2, 16, None, None, ctypes.byref(h))
    assert st == B.DSA_E_INVAL


def test_db_create_allocator_needs_both_functions(B):
    """An allocator without a free function is refused before any device
    work; the callbacks are never called."""
    codes = np.array([0, 1, 2], np.uint8)
    offs = np.array([0, 3], np.int64)
    calls = []
    alloc = B.ALLOC_FN(lambda n, ctx: calls.append(n) or None)
    half = B.dsa_allocator(alloc, B.FREE_FN(), None)
    h = ctypes.c_void_p()
    st = B.lib().dsa_db_create(codes.ctypes.data, offs.ctypes.data, 1, 4, ctypes.byref(half), None,
                               ctypes.byref(h))
    assert st == B.DSA_E_INVAL and "allocator" in B.dsa_last_error()
    assert calls == [] and not h.value


def test_length_limit(B):
    """Sequences up to 65,532 residues are supported; longer ones are
    rejected with DSA_E_NOTSUP before any device work."""
    codes = np.zeros(65533, np.uint8)
    offs = np.array([0, 65533], np.int64)
    h = ctypes.c_void_p()
    st = B.lib().dsa_db_create(codes.ctypes.data, offs.ctypes.data, 1, 4, None, None, ctypes.byref(h))
    assert st == B.DSA_E_NOTSUP and "65532" in B.dsa_last_error()
    n = ctypes.c_size_t()
    qo = np.array([0, 65533], np.int64)
    to = np.array([0, 10], np.int64)
    a = _args(B, q_offsets=qo.ctypes.data, t_offsets=to.ctypes.data)
    assert B.lib().dsa_workspace_size(ctypes.byref(a), ctypes.byref(n)) == B.DSA_E_NOTSUP
    qo[1] = 65532
    assert B.lib().dsa_workspace_size(ctypes.byref(a), ctypes.byref(n)) == B.DSA_OK


def test_no_cpu_fallback():
    import torch
    import paper_1701_01575_amd as dsa
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        dsa.Database(np.zeros(4, np.uint8), np.array([0, 4]), 4)
