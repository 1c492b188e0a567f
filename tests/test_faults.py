"""Fault injection (DSA_FAULT) on the CPU: an align call that the variable
names fails with DSA_E_DEVICE before any device work, counts start again when
the variable changes, and a query length can be named.  The calls carry a
one-byte workspace, so a call the fault does not name stops at the workspace check
(DSA_E_WORKSPACE): no call here reaches the device, with or without a GPU."""
import ctypes

import numpy as np
import pytest


@pytest.fixture()
def B(monkeypatch):
    from paper_1701_01575_amd import binding
    monkeypatch.delenv("DSA_FAULT", raising=False)
    return binding


def _pair_args(B, qlens=(3, 5)):
    qo = np.concatenate([[0], np.cumsum(qlens)]).astype(np.int64)
    S = np.eye(4, dtype=np.int8) * 2 - 1
    a = B.dsa_args()
    a.q_codes = 1  # never dereferenced before the fault
    a.q_offsets = qo.ctypes.data
    a.n_q = len(qlens)
    a.t_codes = 1
    a.t_offsets = qo.ctypes.data
    a.subst = S.ctypes.data
    a.alphabet_size = 4
    a.gap_open = 5
    a.gap_extend = 2
    a.workspace = 256      # never dereferenced: one byte is below any plan's size
    a.workspace_bytes = 1
    a._keep = (qo, S)
    out = B.dsa_out()
    score = np.zeros(len(qlens), np.int32)
    out.score = score.ctypes.data
    out._keep = score
    return a, out


def _call(B, a, out):
    return B.lib().dsa_align_batch(ctypes.byref(a), ctypes.byref(out))


def test_launch_fault_counts_calls(B, monkeypatch):
    a, out = _pair_args(B)
    monkeypatch.setenv("DSA_FAULT", "launch:2")
    assert _call(B, a, out) == B.DSA_E_WORKSPACE
    assert _call(B, a, out) == B.DSA_E_DEVICE and "injected fault" in B.dsa_last_error()
    assert _call(B, a, out) == B.DSA_E_WORKSPACE
    # a new text starts the count again
    monkeypatch.setenv("DSA_FAULT", "launch:1")
    assert _call(B, a, out) == B.DSA_E_DEVICE and "injected fault" in B.dsa_last_error()


def test_qlen_fault_names_a_query(B, monkeypatch):
    a, out = _pair_args(B, qlens=(3, 777))
    monkeypatch.setenv("DSA_FAULT", "qlen:777")
    assert _call(B, a, out) == B.DSA_E_DEVICE and "injected fault" in B.dsa_last_error()
    a2, out2 = _pair_args(B, qlens=(3, 776))
    assert _call(B, a2, out2) == B.DSA_E_WORKSPACE
