"""MI355X affine-gap sequence alignment (local, global, semi-global).

The alignment itself runs in libdsa.so (hand-written HIP kernels for
gfx950); this module marshals arguments and uses torch only to own device
memory and streams.  There is no CPU fallback: without the built library
or a GPU every call raises.

    db = Database(codes, offsets, alphabet_size=24)
    res = align(queries, db=db, matrix=blosum62, gap_open=11, gap_extend=1)
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import binding as B
from .binding import (  # noqa: F401
    DSA_FORCE_INT32, DSA_GLOBAL, DSA_LOCAL, DSA_PLAIN, DSA_QB, DSA_QE, DSA_SEMIGLOBAL,
    DSA_ST_INT32, DSA_ST_TRUNCATED, DSA_TB, DSA_TE, DSA_TRACEBACK, DsaError,
)

MODES = {"local": DSA_LOCAL, "global": DSA_GLOBAL, "semiglobal": DSA_SEMIGLOBAL}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the alignment kernels need an MI355X (gfx950)")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class TorchAllocator:
    """A dsa_allocator backed by torch's caching allocator: every device
    buffer of a database is a uint8 tensor that this object holds until the
    library gives the buffer back."""

    def __init__(self, device):
        self.device = device
        self.held = {}
        self._alloc = B.ALLOC_FN(self._on_alloc)
        self._free = B.FREE_FN(self._on_free)
        self.c = B.dsa_allocator(self._alloc, self._free, None)

    def _on_alloc(self, nbytes, ctx):
        import torch
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:
            return None
        self.held[t.data_ptr()] = t
        return t.data_ptr()

    def _on_free(self, ptr, ctx):
        self.held.pop(ptr, None)

    def bytes_held(self) -> int:
        return sum(t.numel() for t in self.held.values())


class Database:
    """A target database packed into device memory (dsa_db_create).

    allocator="torch" (the default) takes the database's device buffers from
    torch's caching allocator (a TorchAllocator may be passed to share one);
    allocator=None lets the library use hipMalloc."""

    def __init__(self, codes, offsets, alphabet_size: int, device=None, allocator="torch"):
        torch = _torch()
        if device is None:
            device = torch.cuda.current_device()
        self.device = device if isinstance(device, torch.device) else torch.device("cuda", int(device))
        with torch.cuda.device(self.device):
            self._codes = _host(codes, np.uint8)
            self._offsets = _host(offsets, np.int64)
            self.n_targets = len(self._offsets) - 1
            self.alphabet_size = int(alphabet_size)
            if isinstance(allocator, TorchAllocator):
                self.allocator = allocator
            else:
                self.allocator = TorchAllocator(self.device) if allocator == "torch" else None
            stream = torch.cuda.current_stream().cuda_stream
            self.handle = B.dsa_db_create(self._codes.ctypes.data_as(ctypes.c_void_p),
                                          self._offsets.ctypes.data_as(ctypes.c_void_p),
                                          self.n_targets, self.alphabet_size, ctypes.c_void_p(stream),
                                          self.allocator.c if self.allocator is not None else None)
        self.lengths = np.diff(self._offsets)

    @classmethod
    def from_seqset(cls, s, alphabet_size: int, device=None, allocator="torch"):
        return cls(s.codes, s.offsets, alphabet_size, device, allocator)

    @classmethod
    def from_file(cls, path, alphabet="protein", device=None, allocator="torch"):
        """Read a FASTA or FASTQ file with the library's ingest and pack it;
        the record names are kept in `names`."""
        seqs = Sequences.from_file(path, alphabet)
        db = cls(seqs.codes, seqs.offsets, 24 if alphabet == "protein" else 5, device, allocator)
        db.names = seqs.names
        return db

    def info(self):
        return B.dsa_db_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            B.dsa_db_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


ALPHABETS = {"protein": B.DSA_ALPHA_PROTEIN, "dna": B.DSA_ALPHA_DNA}


class Sequences:
    """Sequences read from FASTA or FASTQ text by the library's ingest
    (dsa_seqset_*): uint8 codes, int64 offsets (n + 1) and record names.
    Works without a GPU; feed Database(...) or align(...) with it."""

    def __init__(self, codes, offsets, names, fmt):
        self.codes = codes
        self.offsets = offsets
        self.names = names
        self.format = {B.DSA_FORMAT_FASTA: "fasta", B.DSA_FORMAT_FASTQ: "fastq"}.get(fmt, "none")

    def __len__(self):
        return len(self.offsets) - 1

    def __getitem__(self, k):
        return self.codes[self.offsets[k]:self.offsets[k + 1]]

    @property
    def lengths(self):
        return np.diff(self.offsets)

    @classmethod
    def _from_handle(cls, h):
        n, nres, fmt = B.dsa_seqset_info(h)
        cp, op = B.dsa_seqset_codes(h)
        offsets = np.ctypeslib.as_array((ctypes.c_int64 * (n + 1)).from_address(op)).copy()
        codes = (np.ctypeslib.as_array((ctypes.c_uint8 * nres).from_address(cp)).copy() if nres
                 else np.zeros(0, np.uint8))
        names = [B.dsa_seqset_name(h, k).decode(errors="replace") for k in range(n)]
        return cls(codes, offsets, names, fmt)

    @classmethod
    def from_file(cls, path, alphabet="protein"):
        """Read a FASTA or FASTQ file (streamed in 4 MiB pieces)."""
        h = B.dsa_seqset_create(ALPHABETS[alphabet])
        try:
            B.dsa_seqset_read_file(h, str(path))
            return cls._from_handle(h)
        finally:
            B.dsa_seqset_destroy(h)

    @classmethod
    def from_text(cls, pieces, alphabet="protein"):
        """Read FASTA or FASTQ text given as one str/bytes or an iterable of pieces."""
        if isinstance(pieces, (str, bytes)):
            pieces = [pieces]
        h = B.dsa_seqset_create(ALPHABETS[alphabet])
        try:
            for p in pieces:
                B.dsa_seqset_feed(h, p.encode() if isinstance(p, str) else bytes(p))
            B.dsa_seqset_finish(h)
            return cls._from_handle(h)
        finally:
            B.dsa_seqset_destroy(h)


def read_sequences(path, alphabet="protein") -> Sequences:
    return Sequences.from_file(path, alphabet)


def _workspace(nbytes: int, device):
    """A workspace from torch's caching allocator, taken on the current
    stream (the call's): once the caller drops it, torch hands the block out
    again only to later work on that stream, which runs after this call's
    kernels, so calls on different streams or threads never share one."""
    torch = _torch()
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    aligned = (t.data_ptr() + 255) // 256 * 256
    return t, aligned, t.numel() - (aligned - t.data_ptr())


def device_queries(queries, device):
    """Stage a SeqSet's codes on the device: returns (codes tensor, host offsets)."""
    torch = _torch()
    codes = torch.from_numpy(_host(queries.codes, np.uint8)).to(device) if len(queries.codes) else \
        torch.zeros(1, dtype=torch.uint8, device=device)
    return codes, _host(queries.offsets, np.int64)


def make_args(q_codes, q_offsets, matrix, gap_open, gap_extend, mode="local", db=None,
              t_codes=None, t_offsets=None, free_ends=None, traceback=False, top_k=0,
              plain=False, force_int32=False, stream=None, pssm=None):
    torch = _torch()
    a = B.dsa_args()
    q_offsets = _host(q_offsets, np.int64)
    S = _host(matrix, np.int8)
    if pssm is not None:
        pssm = _host(pssm, np.int8)
        if pssm.shape != (int(q_offsets[-1]), S.shape[0]):
            raise ValueError("pssm must hold one row of alphabet-size scores per query residue")
        a.pssm = pssm.ctypes.data
    a.q_codes = q_codes.data_ptr()
    a.q_offsets = q_offsets.ctypes.data
    a.n_q = len(q_offsets) - 1
    a.db = db.handle if db is not None else None
    keep = [q_offsets, S, pssm]
    if t_codes is not None:
        t_offsets = _host(t_offsets, np.int64)
        keep.append(t_offsets)
        a.t_codes = t_codes.data_ptr()
        a.t_offsets = t_offsets.ctypes.data
    a.subst = S.ctypes.data
    a.alphabet_size = S.shape[0]
    a.gap_open = int(gap_open)
    a.gap_extend = int(gap_extend)
    a.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    a.free_ends = int(free_ends or 0)
    a.flags = (DSA_TRACEBACK if traceback else 0) | (DSA_PLAIN if plain else 0) | \
        (DSA_FORCE_INT32 if force_int32 else 0)
    a.top_k = int(top_k)
    if stream is None:
        stream = torch.cuda.current_stream()
    a.stream = stream.cuda_stream
    a._keep = keep
    return a


def align_args(a, device, n_results, want_coords=True, want_begin=True, cigar_capacity=None):
    """Allocate outputs + workspace and call dsa_align_batch; returns tensors.
    Called with the call's stream current (align() arranges it)."""
    torch = _torch()
    need = B.dsa_workspace_size(a)
    ws_tensor, ws, ws_bytes = _workspace(need, device)
    a.workspace = ws
    a.workspace_bytes = ws_bytes
    out = B.dsa_out()
    i32 = dict(dtype=torch.int32, device=device)
    nr = max(n_results, 1)
    res = {"score": torch.empty(nr, **i32)}
    if want_coords:
        res["q_end"] = torch.empty(nr, **i32)
        res["t_end"] = torch.empty(nr, **i32)
    if want_begin:
        res["q_begin"] = torch.empty(nr, **i32)
        res["t_begin"] = torch.empty(nr, **i32)
    res["status"] = torch.empty(nr, dtype=torch.uint8, device=device)
    if a.top_k:
        res["t_index"] = torch.empty(nr, dtype=torch.int64, device=device)
    if a.flags & DSA_TRACEBACK:
        cap = B.dsa_cigar_capacity(a) if cigar_capacity is None else int(cigar_capacity)
        res["cigar_off"] = torch.empty(nr, dtype=torch.int64, device=device)
        res["cigar_len"] = torch.empty(nr, **i32)
        res["cigar_ops"] = torch.empty(max(cap, 1), dtype=torch.int32, device=device)
        out.cigar_capacity = cap
    for k in ("score", "q_begin", "q_end", "t_begin", "t_end", "status", "cigar_off", "cigar_len",
              "cigar_ops", "t_index"):
        if k in res:
            setattr(out, k, res[k].data_ptr())
    st = B.dsa_align_batch(a, out)
    del ws_tensor  # reusable by later work on this stream only
    res = {k: (v[:n_results] if k != "cigar_ops" else v) for k, v in res.items()}
    res["capacity_ok"] = st == B.DSA_OK
    return res


def _outputs(a, device, n_results, cigar_capacity=None):
    torch = _torch()
    out = B.dsa_out()
    i32 = dict(dtype=torch.int32, device=device)
    nr = max(n_results, 1)
    res = {k: torch.empty(nr, **i32) for k in ("score", "q_end", "t_end", "q_begin", "t_begin")}
    res["status"] = torch.empty(nr, dtype=torch.uint8, device=device)
    if a.top_k:
        res["t_index"] = torch.empty(nr, dtype=torch.int64, device=device)
    if a.flags & DSA_TRACEBACK:
        cap = B.dsa_cigar_capacity(a) if cigar_capacity is None else int(cigar_capacity)
        res["cigar_off"] = torch.empty(nr, dtype=torch.int64, device=device)
        res["cigar_len"] = torch.empty(nr, **i32)
        res["cigar_ops"] = torch.empty(max(cap, 1), dtype=torch.int32, device=device)
        out.cigar_capacity = cap
    for k, v in res.items():
        setattr(out, k, v.data_ptr())
    return out, res


class Recorded:
    """One batch recorded into a HIP graph (dsa_graph_create): `run()`
    replays every kernel of the call on the stream given at creation, with
    the same buffers, which this object keeps alive.  `results()` returns the
    output tensors (valid once the stream has finished the replay)."""

    def __init__(self, queries, db: Database = None, targets=None, matrix=None, gap_open=11,
                 gap_extend=1, mode="local", free_ends=None, traceback=False, top_k=0,
                 force_int32=False, stream=None):
        torch = _torch()
        self.device = db.device if db is not None else torch.device("cuda", torch.cuda.current_device())
        if stream is None:
            stream = torch.cuda.Stream(device=self.device)
        self.stream = stream
        with torch.cuda.stream(stream):
            qc, qo = device_queries(queries, self.device)
            tc = to = None
            if targets is not None:
                tc, to = device_queries(targets, self.device)
            a = make_args(qc, qo, matrix, gap_open, gap_extend, mode, db, tc, to, free_ends, traceback,
                          top_k, False, force_int32, stream)
            nq = len(qo) - 1
            n = nq if targets is not None else (nq * top_k if top_k else nq * db.n_targets)
            need = B.dsa_workspace_size(a)
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            a.workspace = (self._ws.data_ptr() + 255) // 256 * 256
            a.workspace_bytes = need
            out, res = _outputs(a, self.device, n)
        stream.synchronize()
        self._keep = (qc, tc, a, out, db)
        self._res = {k: (v[:n] if k != "cigar_ops" else v) for k, v in res.items()}
        self.handle, st = B.dsa_graph_create(a, out)
        self.capacity_ok = st == B.DSA_OK

    def run(self):
        B.dsa_graph_launch(self.handle, self.stream.cuda_stream)

    def results(self) -> dict:
        return self._res

    def close(self):
        if getattr(self, "handle", None):
            B.dsa_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(queries, db: Database = None, targets=None, matrix=None, gap_open=11, gap_extend=1,
             mode="local", free_ends=None, traceback=False, top_k=0, plain=False, cache_path=None) -> dict:
    """Time the launch candidates on these inputs (dsa_autotune) and keep the
    fastest for their shape class; returns the choice."""
    torch = _torch()
    device = db.device if db is not None else torch.device("cuda", torch.cuda.current_device())
    qc, qo = device_queries(queries, device)
    tc = to = None
    if targets is not None:
        tc, to = device_queries(targets, device)
    a = make_args(qc, qo, matrix, gap_open, gap_extend, mode, db, tc, to, free_ends, traceback, top_k,
                  plain, False, None)
    return B.dsa_autotune(a, cache_path)


def tuning(queries, db: Database = None, targets=None, matrix=None, gap_open=11, gap_extend=1,
           mode="local", free_ends=None, traceback=False, top_k=0, plain=False) -> dict:
    """The launch choices a call with these inputs would use now, and its class key."""
    torch = _torch()
    device = db.device if db is not None else torch.device("cuda", torch.cuda.current_device())
    qc, qo = device_queries(queries, device)
    tc = to = None
    if targets is not None:
        tc, to = device_queries(targets, device)
    a = make_args(qc, qo, matrix, gap_open, gap_extend, mode, db, tc, to, free_ends, traceback, top_k,
                  plain, False, None)
    out = B.dsa_tuning_get(a)
    out["key"] = B.dsa_tuning_key(a)
    return out


def cigars(res) -> list:
    """Per-result CIGAR runs (uint32 numpy arrays, (len << 4) | op) on the host."""
    ops = res["cigar_ops"].cpu().numpy().view(np.uint32)
    off = res["cigar_off"].cpu().numpy()
    ln = res["cigar_len"].cpu().numpy()
    return [ops[int(o):int(o) + int(n)].copy() for o, n in zip(off, ln)]


def align(queries, db: Database = None, targets=None, matrix=None, gap_open=11, gap_extend=1,
          mode="local", free_ends=None, traceback=False, top_k=0, plain=False,
          force_int32=False, stream=None, cigar_capacity=None, pssm=None) -> dict:
    """Align a SeqSet of queries against a Database (every query vs every
    target, query-major results) or against a SeqSet of targets pairwise.
    pssm: optional (total query residues, alphabet) int8 position-specific
    scores, used in place of the matrix rows.
    Returns a dict of device tensors (score, q_begin, q_end, t_begin, t_end,
    status)."""
    torch = _torch()
    device = db.device if db is not None else torch.device("cuda", torch.cuda.current_device())
    if stream is None:
        stream = torch.cuda.current_stream(device)
    with torch.cuda.device(device), torch.cuda.stream(stream):
        qc, qo = device_queries(queries, device)
        tc = to = None
        if targets is not None:
            tc, to = device_queries(targets, device)
        a = make_args(qc, qo, matrix, gap_open, gap_extend, mode, db, tc, to, free_ends, traceback,
                      top_k, plain, force_int32, stream, pssm)
        nq = len(qo) - 1
        n = nq * (db.n_targets if db is not None else 1) if not top_k else nq * top_k
        if targets is not None:
            n = nq
        res = align_args(a, device, n, cigar_capacity=cigar_capacity)
    res["_keep"] = (qc, tc)
    return res
from .serve import AdmissionError, Server  # noqa: F401,E402
from .algorithms import DNW, DSG, DSW, Alignment  # noqa: F401,E402
