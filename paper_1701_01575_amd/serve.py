"""Serving: a device-resident database answering a stream of requests (each
1..64 queries) with the K best local alignments per query, with traceback.

The paper keeps hot reference data in memory (Section II.A, the in-memory
store) and answers with the K best alignment objects per query
(Section II.B.2: per-partition K best, then one merge).  Here the database
stays resident in HBM, split into C chunks of about equal residues (each
packed as its own database), and the server runs in steps:

* step s scans chunk s mod C with every active query (one batched top-K
  search: every active query against the chunk);
* a query that joined at step s0 has seen every chunk after step s0 + C - 1;
  its per-chunk K best are merged by (score descending, original target index
  ascending), which gives exactly the K best over the whole database, and
  its hits are traced (one pairwise batch with traceback);
* requests join at step boundaries, in arrival order, as long as the step's
  device memory (search workspace, outputs and the hit traceback, as the
  backend reports them) fits the HBM budget; a request that cannot fit even
  alone is refused at once;
* the traceback of the queries that finished at step s runs on its own
  stream while step s + 1 scans, so the two overlap on the device.

A request completes when all its queries are traced.  Its latency is
completion minus arrival.  The backend (search, collect, trace, footprint)
is all the scheduler uses, so the scheduling logic runs on the CPU in the
tests with a backend of their own.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future

import numpy as np


class AdmissionError(RuntimeError):
    """The request can never fit in the HBM budget."""


class Seqs:
    """Concatenated sequences: uint8 codes plus int64 offsets (n + 1)."""

    def __init__(self, codes, offsets):
        self.codes = np.ascontiguousarray(codes, dtype=np.uint8)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)

    def __len__(self):
        return len(self.offsets) - 1

    def __getitem__(self, k):
        return self.codes[self.offsets[k]:self.offsets[k + 1]]

    @property
    def lengths(self):
        return np.diff(self.offsets)


def concat(seqs):
    """Sequences (arrays) or sequence sets -> one Seqs."""
    parts = []
    for s in seqs:
        if isinstance(s, np.ndarray):
            parts.append(np.asarray(s, dtype=np.uint8))
        else:
            parts.extend(np.asarray(s[k], dtype=np.uint8) for k in range(len(s)))
    offs = np.zeros(len(parts) + 1, np.int64)
    if parts:
        offs[1:] = np.cumsum([len(p) for p in parts])
    codes = np.concatenate(parts) if parts and offs[-1] else np.zeros(0, np.uint8)
    return Seqs(codes, offs)


def merge_topk(idx, score, k, positive_only=True):
    """The k best of (index, score) candidates: score descending, then index
    ascending; with positive_only, scores <= 0 are left out."""
    idx = np.asarray(idx, dtype=np.int64)
    score = np.asarray(score, dtype=np.int64)
    if positive_only:
        keep = score > 0
        idx, score = idx[keep], score[keep]
    order = np.lexsort((idx, -score))[:k]
    return idx[order], score[order]


@dataclasses.dataclass
class Request:
    rid: int
    queries: Seqs
    arrival: float
    future: Future
    left: int = 0               # queries not yet traced
    results: list = None
    start: float = 0.0          # step at which it joined (clock)
    done: float = 0.0


@dataclasses.dataclass
class Active:
    req: Request
    qi: int                     # query index within its request
    seq: np.ndarray
    joined: int                 # step at which the query joined
    hits_idx: np.ndarray = None
    hits_score: np.ndarray = None


class GpuBackend:
    """The resident database on libdsa, in chunks: top-K searches per chunk,
    pairwise traceback of the merged hits."""

    def __init__(self, db, matrix, gap_open=11, gap_extend=1, top_k=10, mode="local", chunks=8):
        import torch
        import paper_1701_01575_amd as dsa
        self.dsa = dsa
        self.device = db.device
        self.matrix = np.ascontiguousarray(matrix, dtype=np.int8)
        self.o, self.e, self.top_k, self.mode = gap_open, gap_extend, top_k, mode
        self.positive_only = mode == "local"
        codes, offs = db._codes, db._offsets
        n = len(offs) - 1
        self.t_codes, self.t_offsets = codes, offs
        # chunk bounds: contiguous index ranges of about equal residues, so a
        # chunk's local index + its first index is the original index
        cum = offs[1:]
        bounds = [0]
        for c in range(1, chunks):
            bounds.append(int(np.searchsorted(cum, offs[-1] * c / chunks)))
        bounds.append(n)
        bounds = sorted(set(min(max(b, 0), n) for b in bounds))
        self.chunks = []
        for lo, hi in zip(bounds[:-1], bounds[1:]):
            if hi <= lo:
                continue
            sub_off = offs[lo:hi + 1] - offs[lo]
            cdb = dsa.Database(codes[offs[lo]:offs[hi]], sub_off, db.alphabet_size, device=self.device)
            self.chunks.append((cdb, lo, int((offs[lo + 1:hi + 1] - offs[lo:hi]).max())))
        self.n_chunks = len(self.chunks)
        self.max_len = int(np.diff(offs).max()) if n else 0
        self.search_stream = torch.cuda.Stream(device=self.device)
        self.trace_stream = torch.cuda.Stream(device=self.device)
        self._ws_cache = {}

    # -- device memory of one step -----------------------------------------
    def footprint(self, query_lengths) -> int:
        """Bytes one step holds with these active queries: the largest chunk
        search (workspace from the library, outputs) plus the hit traceback
        (workspace bound: codes at half a byte per cell, CIGAR regions)."""
        from . import binding as B
        lens = np.asarray(query_lengths, np.int64)
        if len(lens) == 0:
            return 0
        key = (len(lens), int(lens.sum()), int(lens.max()))
        ws = self._ws_cache.get(key)
        if ws is None:
            import torch
            offs = np.concatenate([[0], np.cumsum(lens)])
            qc = torch.zeros(1, dtype=torch.uint8, device=self.device)
            ws = 0
            for cdb, _, _ in self.chunks:
                a = self.dsa.make_args(qc, offs, self.matrix, self.o, self.e, self.mode, db=cdb,
                                       top_k=self.top_k)
                ws = max(ws, B.dsa_workspace_size(a))
            self._ws_cache[key] = ws
        n_out = len(lens) * self.top_k
        trace = int(sum(self.top_k * (m * self.max_len // 2 + 4 * (m + self.max_len + 1) + 256)
                        for m in lens.tolist()))
        return int(ws + n_out * 64 + trace)

    # -- one chunk scan -----------------------------------------------------
    def search(self, chunk: int, queries: Seqs):
        import torch
        cdb, first, _ = self.chunks[chunk]
        with torch.cuda.stream(self.search_stream):
            r = self.dsa.align(queries, db=cdb, matrix=self.matrix, gap_open=self.o, gap_extend=self.e,
                               mode=self.mode, top_k=self.top_k, stream=self.search_stream)
            ev = torch.cuda.Event()
            ev.record(self.search_stream)
        return (r, ev, first, len(queries))

    def collect(self, handle):
        r, ev, first, nq = handle
        ev.synchronize()
        idx = r["t_index"].cpu().numpy().reshape(nq, self.top_k)
        sc = r["score"].cpu().numpy().reshape(nq, self.top_k).astype(np.int64)
        out = []
        for q in range(nq):
            valid = idx[q] >= 0
            out.append((idx[q][valid] + first, sc[q][valid]))
        return out

    # -- traceback of the final hits ------------------------------------------
    def trace(self, queries: Seqs, hits):
        import torch
        pq, pt, slot = [], [], []
        for q in range(len(queries)):
            for k, t in enumerate(hits[q]):
                pq.append(queries[q])
                pt.append(self.t_codes[self.t_offsets[t]:self.t_offsets[t + 1]])
                slot.append((q, k))
        if not pq:
            return (None, None, queries, hits, slot)
        with torch.cuda.stream(self.trace_stream):
            r = self.dsa.align(concat(pq), targets=concat(pt), matrix=self.matrix, gap_open=self.o,
                               gap_extend=self.e, mode=self.mode, traceback=True, stream=self.trace_stream)
            ev = torch.cuda.Event()
            ev.record(self.trace_stream)
        return (r, ev, queries, hits, slot)

    def collect_trace(self, handle):
        r, ev, queries, hits, slot = handle
        K = self.top_k
        out = []
        for q in range(len(queries)):
            d = {"t_index": np.full(K, -1, np.int64)}
            for f in ("score",):
                d[f] = np.zeros(K, np.int32)
            for f in ("q_begin", "q_end", "t_begin", "t_end"):
                d[f] = np.full(K, -1, np.int32)
            d["cigars"] = [np.zeros(0, np.uint32) for _ in range(K)]
            out.append(d)
        if r is None:
            return out
        ev.synchronize()
        host = {f: r[f].cpu().numpy() for f in ("score", "q_begin", "q_end", "t_begin", "t_end")}
        cig = self.dsa.cigars(r)
        for p, (q, k) in enumerate(slot):
            d = out[q]
            d["t_index"][k] = hits[q][k]
            for f in host:
                d[f][k] = host[f][p]
            d["cigars"][k] = cig[p]
        return out

    def close(self):
        for cdb, _, _ in self.chunks:
            cdb.close()


class Server:
    """Continuous batching in chunk steps over a resident database.

        srv = Server(db, hbm_budget_bytes, matrix=blosum62).start()
        fut = srv.submit(queries)        # a SeqSet-like set of 1..64 queries
        hits = fut.result()              # per query: t_index, score, begins, ends, cigars

    db is a Database (its targets are re-packed into `chunks` chunks), or
    None with backend= given (the tests' own backends)."""

    def __init__(self, db, hbm_budget_bytes: int, *, matrix=None, gap_open=11, gap_extend=1, top_k=10,
                 mode="local", chunks=8, max_active_queries=256, backend=None, clock=time.monotonic):
        if backend is None:
            if db is None or matrix is None:
                raise ValueError("Server needs a Database and a substitution matrix (or a backend)")
            backend = GpuBackend(db, matrix, gap_open, gap_extend, top_k, mode, chunks)
        self.backend = backend
        self.budget = int(hbm_budget_bytes)
        self.max_active = int(max_active_queries)
        self.clock = clock
        self.queue = collections.deque()
        self.cv = threading.Condition()
        self.active: list[Active] = []
        self.step = 0
        self.next_id = 0
        self.stopping = False
        self.completed = []
        self.rejected = 0
        self.errors = 0
        self.steps = []             # (step, chunk, active queries, joined, finished)
        self.peak_footprint = 0
        self._thread = None

    # -- client side ------------------------------------------------------
    def submit(self, queries, arrival: float | None = None) -> Future:
        fut = Future()
        q = queries if isinstance(queries, Seqs) else concat([queries])
        with self.cv:
            req = Request(self.next_id, q, self.clock() if arrival is None else arrival, fut,
                          left=len(q), results=[None] * len(q))
            self.next_id += 1
            self.queue.append(req)
            self.cv.notify_all()
        return fut

    def start(self):
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()
        return self

    def stop(self, wait: bool = True):
        with self.cv:
            self.stopping = True
            self.cv.notify_all()
        if wait and self._thread is not None:
            self._thread.join()

    # -- scheduling -------------------------------------------------------
    def _admit(self):
        """At a step boundary, with the lock held: move queued requests, in
        arrival order, into the active set while the step fits the budget."""
        joined = 0
        while self.queue:
            req = self.queue[0]
            lens = [len(a.seq) for a in self.active]
            alone = self.backend.footprint(list(req.queries.lengths))
            if alone > self.budget or len(req.queries) > self.max_active:
                self.queue.popleft()
                self.rejected += 1
                req.future.set_exception(AdmissionError(
                    f"request {req.rid} needs {alone} bytes for {len(req.queries)} queries; the budget is "
                    f"{self.budget} bytes and {self.max_active} active queries"))
                continue
            if len(req.queries) == 0:
                self.queue.popleft()
                req.start = req.done = self.clock()
                req.future.set_result([])
                self.completed.append(req)
                continue
            if len(lens) + len(req.queries) > self.max_active:
                break
            need = self.backend.footprint(lens + list(req.queries.lengths))
            if need > self.budget:
                break  # FIFO: later requests wait behind the head
            self.queue.popleft()
            req.start = self.clock()
            for k in range(len(req.queries)):
                self.active.append(Active(req, k, req.queries[k], self.step))
            joined += len(req.queries)
            self.peak_footprint = max(self.peak_footprint, need)
        return joined

    def _finish(self, finished, traced):
        now = self.clock()
        for a, res in zip(finished, traced):
            a.req.results[a.qi] = res
            a.req.left -= 1
            if a.req.left == 0:
                a.req.done = now
                a.req.future.set_result(a.req.results)
                self.completed.append(a.req)

    def _fail(self, group, exc):
        for a in group:
            if not a.req.future.done():
                a.req.done = self.clock()
                a.req.future.set_exception(exc)
                self.errors += 1
                self.completed.append(a.req)

    def _loop(self):
        be = self.backend
        pending = None  # (handle, finished actives): traceback in flight
        while True:
            with self.cv:
                joined = self._admit()
                while not self.active and pending is None and not self.stopping and not self.queue:
                    self.cv.wait()
                    joined += self._admit()
                if not self.active and pending is None:
                    if self.stopping or not self.queue:
                        if self.stopping:
                            for r in self.queue:
                                r.future.set_exception(RuntimeError("server stopped"))
                            self.queue.clear()
                            return
                        continue
                active = list(self.active)
            chunk = self.step % be.n_chunks
            live = [a for a in active if not a.req.future.done()]
            handle = None
            if live:
                try:
                    handle = be.search(chunk, concat([a.seq for a in live]))
                except Exception:
                    handle = None  # rescanned request by request below
            if pending is not None:  # overlaps this step's scan
                h, fin = pending
                pending = None
                try:
                    traced = be.collect_trace(h)
                    with self.cv:
                        self._finish(fin, traced)
                except Exception as exc:
                    with self.cv:
                        self._fail(fin, exc)
            finished = []
            if live:
                per_query = None
                if handle is not None:
                    try:
                        per_query = be.collect(handle)
                    except Exception:
                        per_query = None
                if per_query is None:
                    per_query = self._scan_isolated(chunk, live)
                for a, got in zip(live, per_query):
                    if got is None:
                        continue
                    idx, sc = got
                    if a.hits_idx is None:
                        a.hits_idx, a.hits_score = idx, sc
                    else:
                        a.hits_idx, a.hits_score = merge_topk(
                            np.concatenate([a.hits_idx, idx]), np.concatenate([a.hits_score, sc]),
                            be.top_k, be.positive_only)
                    if self.step - a.joined + 1 >= be.n_chunks:
                        finished.append(a)
            with self.cv:
                done_ids = set(id(a) for a in finished)
                self.active = [a for a in self.active if id(a) not in done_ids and not a.req.future.done()]
                self.steps.append((self.step, chunk, len(live), joined, len(finished)))
                self.step += 1
                self.cv.notify_all()
            if finished:
                try:
                    pending = (be.trace(concat([a.seq for a in finished]),
                                        [a.hits_idx for a in finished]), finished)
                except Exception as exc:
                    with self.cv:
                        self._fail(finished, exc)

    def _scan_isolated(self, chunk, live):
        """The step's scan failed: scan each request's queries alone, so only
        the requests that fail by themselves report the error."""
        be = self.backend
        out = [None] * len(live)
        groups = collections.OrderedDict()
        for k, a in enumerate(live):
            groups.setdefault(a.req.rid, []).append(k)
        for ks in groups.values():
            members = [live[k] for k in ks]
            try:
                res = be.collect(be.search(chunk, concat([a.seq for a in members])))
                for k, r in zip(ks, res):
                    out[k] = r
            except Exception as exc:
                with self.cv:
                    self._fail(members, exc)
        return out

    # -- statistics -------------------------------------------------------
    def latencies(self):
        return np.array([r.done - r.arrival for r in self.completed if r.future.done()
                         and r.future.exception() is None])

    def stats(self) -> dict:
        lat = self.latencies()
        out = {"completed": len(self.completed), "rejected": self.rejected, "errors": self.errors,
               "steps": len(self.steps), "peak_footprint_bytes": self.peak_footprint,
               "budget_bytes": self.budget, "n": int(len(lat))}
        if len(lat):
            out.update(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                       max_s=float(lat.max()), mean_s=float(lat.mean()))
        return out
