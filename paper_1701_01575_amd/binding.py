"""ctypes binding of libdsa.so: the C ABI of include/dsa.h, same names.

Argument marshalling only; every step of the alignment runs in the HIP
library.  Loading fails loudly when libdsa.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# DSA_LIBRARY names another build of the library (the host-sanitized one of
# the CPU sanitizer tests); by default the in-tree build is loaded
LIB_PATH = os.environ.get("DSA_LIBRARY") or os.path.join(PKG, "libdsa.so")
ABI_VERSION = 4  # DSA_ABI_VERSION of the include/dsa.h the structs here mirror

DSA_OK, DSA_E_INVAL, DSA_E_RANGE, DSA_E_WORKSPACE, DSA_E_CAPACITY, DSA_E_DEVICE, DSA_E_NOTSUP = range(7)
DSA_LOCAL, DSA_GLOBAL, DSA_SEMIGLOBAL = 0, 1, 2
DSA_QB, DSA_QE, DSA_TB, DSA_TE = 1, 2, 4, 8
DSA_TRACEBACK, DSA_PLAIN, DSA_FORCE_INT32 = 1, 2, 4
DSA_ST_INT32, DSA_ST_TRUNCATED = 1, 2
DSA_ALPHA_PROTEIN, DSA_ALPHA_DNA = 1, 2
DSA_FORMAT_NONE, DSA_FORMAT_FASTA, DSA_FORMAT_FASTQ = 0, 1, 2

EXPORTS = ["dsa_db_create", "dsa_db_destroy", "dsa_db_info", "dsa_workspace_size",
           "dsa_cigar_capacity", "dsa_align_batch", "dsa_align_batch_noalloc", "dsa_graph_create", "dsa_graph_launch",
           "dsa_graph_destroy", "dsa_autotune", "dsa_tuning_get", "dsa_tuning_key",
           "dsa_timing_enable", "dsa_timing_read",
           "dsa_timing_reset",
           "dsa_probe",
           "dsa_seqset_create", "dsa_seqset_feed", "dsa_seqset_finish", "dsa_seqset_read_file",
           "dsa_seqset_info", "dsa_seqset_codes", "dsa_seqset_name", "dsa_seqset_destroy",
           "dsa_strerror", "dsa_last_error", "dsa_abi_version"]


class DsaError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: status {status}: {detail}")


class dsa_args(ctypes.Structure):
    _fields_ = [
        ("q_codes", ctypes.c_void_p),
        ("q_offsets", ctypes.c_void_p),
        ("n_q", ctypes.c_int64),
        ("db", ctypes.c_void_p),
        ("t_codes", ctypes.c_void_p),
        ("t_offsets", ctypes.c_void_p),
        ("subst", ctypes.c_void_p),
        ("pssm", ctypes.c_void_p),
        ("alphabet_size", ctypes.c_int32),
        ("gap_open", ctypes.c_int32),
        ("gap_extend", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("free_ends", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("top_k", ctypes.c_int32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class dsa_allocator(ctypes.Structure):
    _fields_ = [
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("ctx", ctypes.c_void_p),
    ]


class dsa_out(ctypes.Structure):
    _fields_ = [
        ("score", ctypes.c_void_p),
        ("q_begin", ctypes.c_void_p),
        ("q_end", ctypes.c_void_p),
        ("t_begin", ctypes.c_void_p),
        ("t_end", ctypes.c_void_p),
        ("t_index", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("cigar_off", ctypes.c_void_p),
        ("cigar_len", ctypes.c_void_p),
        ("cigar_ops", ctypes.c_void_p),
        ("cigar_capacity", ctypes.c_int64),
    ]


_lib = None


def lib():
    """Load libdsa.so (built by __graft_entry__.build()); raise if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.dsa_db_create.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(dsa_allocator), P,
                                    ctypes.POINTER(ctypes.c_void_p)]
        L.dsa_db_destroy.argtypes = [P]
        L.dsa_db_info.argtypes = [P, P, P, P]
        L.dsa_workspace_size.argtypes = [ctypes.POINTER(dsa_args), ctypes.POINTER(ctypes.c_size_t)]
        L.dsa_cigar_capacity.argtypes = [ctypes.POINTER(dsa_args), ctypes.POINTER(ctypes.c_int64)]
        L.dsa_align_batch.argtypes = [ctypes.POINTER(dsa_args), ctypes.POINTER(dsa_out)]
        L.dsa_align_batch_noalloc.argtypes = [ctypes.POINTER(dsa_args), ctypes.POINTER(dsa_out)]
        L.dsa_timing_enable.argtypes = [ctypes.c_int]
        L.dsa_timing_read.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]
        L.dsa_timing_reset.argtypes = []
        L.dsa_probe.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
        L.dsa_seqset_create.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
        L.dsa_seqset_feed.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
        L.dsa_seqset_finish.argtypes = [P]
        L.dsa_seqset_read_file.argtypes = [P, ctypes.c_char_p]
        L.dsa_seqset_info.argtypes = [P, P, P, P]
        L.dsa_seqset_codes.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]
        L.dsa_seqset_name.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_int64)]
        L.dsa_seqset_destroy.argtypes = [P]
        L.dsa_strerror.argtypes = [ctypes.c_int]
        L.dsa_strerror.restype = ctypes.c_char_p
        L.dsa_last_error.argtypes = []
        L.dsa_last_error.restype = ctypes.c_char_p
        L.dsa_abi_version.restype = ctypes.c_int32
        if L.dsa_abi_version() != ABI_VERSION:  # the structs below mirror that version of dsa.h
            raise RuntimeError(f"{LIB_PATH}: ABI version {L.dsa_abi_version()}, the binding expects "
                               f"{ABI_VERSION}; rebuild with __graft_entry__.build()")
        for name in EXPORTS:
            if name not in ("dsa_strerror", "dsa_last_error", "dsa_abi_version"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != DSA_OK:
        detail = lib().dsa_last_error().decode(errors="replace")
        raise DsaError(status, where, detail)


def dsa_db_create(codes_ptr, offsets_ptr, n_targets, alphabet_size, stream, allocator=None):
    """allocator: a dsa_allocator (kept alive by the caller) or None for hipMalloc."""
    handle = ctypes.c_void_p()
    check(lib().dsa_db_create(codes_ptr, offsets_ptr, n_targets, alphabet_size,
                              ctypes.byref(allocator) if allocator is not None else None, stream,
                              ctypes.byref(handle)), "dsa_db_create")
    return handle.value


def dsa_db_destroy(handle):
    check(lib().dsa_db_destroy(handle), "dsa_db_destroy")


def dsa_db_info(handle):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(lib().dsa_db_info(handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "dsa_db_info")
    return a.value, b.value, c.value


def dsa_workspace_size(args: dsa_args) -> int:
    n = ctypes.c_size_t()
    check(lib().dsa_workspace_size(ctypes.byref(args), ctypes.byref(n)), "dsa_workspace_size")
    return n.value


def dsa_cigar_capacity(args: dsa_args) -> int:
    n = ctypes.c_int64()
    check(lib().dsa_cigar_capacity(ctypes.byref(args), ctypes.byref(n)), "dsa_cigar_capacity")
    return n.value


def dsa_align_batch(args: dsa_args, out: dsa_out) -> int:
    """Returns the status (DSA_OK or DSA_E_CAPACITY); raises on other errors."""
    st = lib().dsa_align_batch(ctypes.byref(args), ctypes.byref(out))
    if st not in (DSA_OK, DSA_E_CAPACITY):
        check(st, "dsa_align_batch")
    return st


NOALLOC_SCRATCH_BYTES = 64 << 20  # DSA_NOALLOC_SCRATCH_BYTES


def dsa_align_batch_noalloc(args: dsa_args, out: dsa_out) -> int:
    """dsa_align_batch on the library's static scratch (args.workspace is
    ignored).  Returns the status (DSA_OK or DSA_E_CAPACITY); raises on
    other errors."""
    st = lib().dsa_align_batch_noalloc(ctypes.byref(args), ctypes.byref(out))
    if st not in (DSA_OK, DSA_E_CAPACITY):
        check(st, "dsa_align_batch_noalloc")
    return st


def dsa_graph_create(args: dsa_args, out: dsa_out):
    """Record the call (args, out) into a graph; returns (handle, status)."""
    g = ctypes.c_void_p()
    st = lib().dsa_graph_create(ctypes.byref(args), ctypes.byref(out), ctypes.byref(g))
    if st not in (DSA_OK, DSA_E_CAPACITY):
        check(st, "dsa_graph_create")
    return g, st


def dsa_graph_launch(graph, stream) -> None:
    check(lib().dsa_graph_launch(graph, ctypes.c_void_p(stream)), "dsa_graph_launch")


def dsa_graph_destroy(graph) -> None:
    check(lib().dsa_graph_destroy(graph), "dsa_graph_destroy")


class dsa_tuning(ctypes.Structure):
    _fields_ = [
        ("strip", ctypes.c_int32),
        ("waves", ctypes.c_int32),
        ("intra_budget", ctypes.c_int64),
        ("ks_budget", ctypes.c_int64),
        ("pair_rows", ctypes.c_int64),
        ("pair_cells", ctypes.c_int64),
        ("ms", ctypes.c_double),
    ]


def _tuning_dict(t: dsa_tuning) -> dict:
    return {f: getattr(t, f) for f, _ in dsa_tuning._fields_}


def dsa_autotune(args: dsa_args, cache_path: str | None = None) -> dict:
    t = dsa_tuning()
    path = cache_path.encode() if cache_path else None
    check(lib().dsa_autotune(ctypes.byref(args), path, ctypes.byref(t)), "dsa_autotune")
    return _tuning_dict(t)


def dsa_tuning_get(args: dsa_args) -> dict:
    t = dsa_tuning()
    check(lib().dsa_tuning_get(ctypes.byref(args), ctypes.byref(t)), "dsa_tuning_get")
    return _tuning_dict(t)


def dsa_tuning_key(args: dsa_args) -> str:
    buf = ctypes.create_string_buffer(256)
    check(lib().dsa_tuning_key(ctypes.byref(args), buf, ctypes.c_size_t(256)), "dsa_tuning_key")
    return buf.value.decode()


def dsa_timing_enable(on: bool):
    check(lib().dsa_timing_enable(1 if on else 0), "dsa_timing_enable")


TIMING_SPAN, TIMING_INTER, TIMING_INTRA, TIMING_PAIR_LANE, TIMING_PAIR_WF = 0, 1, 2, 3, 4


def dsa_timing_read(kind: int = TIMING_SPAN):
    """(summed milliseconds, launch count) of one timing kind."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    check(lib().dsa_timing_read(kind, ctypes.byref(ms), ctypes.byref(n)), "dsa_timing_read")
    return ms.value, n.value


def dsa_timing_reset():
    check(lib().dsa_timing_reset(), "dsa_timing_reset")


def dsa_probe(which: int, size: int) -> float:
    r = ctypes.c_double()
    check(lib().dsa_probe(which, size, ctypes.byref(r)), "dsa_probe")
    return r.value


def dsa_seqset_create(alphabet: int):
    h = ctypes.c_void_p()
    check(lib().dsa_seqset_create(alphabet, ctypes.byref(h)), "dsa_seqset_create")
    return h.value


def dsa_seqset_feed(handle, data: bytes) -> None:
    check(lib().dsa_seqset_feed(handle, data, len(data)), "dsa_seqset_feed")


def dsa_seqset_finish(handle) -> None:
    check(lib().dsa_seqset_finish(handle), "dsa_seqset_finish")


def dsa_seqset_read_file(handle, path: str) -> None:
    check(lib().dsa_seqset_read_file(handle, os.fsencode(path)), "dsa_seqset_read_file")


def dsa_seqset_info(handle):
    n, r, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    check(lib().dsa_seqset_info(handle, ctypes.byref(n), ctypes.byref(r), ctypes.byref(f)), "dsa_seqset_info")
    return n.value, r.value, f.value


def dsa_seqset_codes(handle):
    """(codes address, offsets address) borrowed from the set."""
    c, o = ctypes.c_void_p(), ctypes.c_void_p()
    check(lib().dsa_seqset_codes(handle, ctypes.byref(c), ctypes.byref(o)), "dsa_seqset_codes")
    return c.value, o.value


def dsa_seqset_name(handle, k: int) -> bytes:
    p, n = ctypes.c_void_p(), ctypes.c_int64()
    check(lib().dsa_seqset_name(handle, k, ctypes.byref(p), ctypes.byref(n)), "dsa_seqset_name")
    return ctypes.string_at(p.value, n.value) if n.value else b""


def dsa_seqset_destroy(handle) -> None:
    check(lib().dsa_seqset_destroy(handle), "dsa_seqset_destroy")


def dsa_strerror(status: int) -> str:
    return lib().dsa_strerror(status).decode()


def dsa_last_error() -> str:
    return lib().dsa_last_error().decode(errors="replace")


def dsa_abi_version() -> int:
    return int(lib().dsa_abi_version())
