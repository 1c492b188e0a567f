"""Serving loop: a device-resident database, requests of 1..64 queries each,
HBM-budget admission and continuous batching over several device slots.

The paper keeps hot reference data in memory (Section II.A, the in-memory
store) and answers with the K best alignment objects per query
(Section II.B.2).  Here the packed database stays resident in HBM; requests
queue FIFO; a scheduler forms a batch from the queue head whenever a slot is
free, as long as the batch's device memory (workspace + outputs + CIGAR
buffer, as dsa_workspace_size / dsa_cigar_capacity report) fits in what the
budget has left.  Each slot is a worker thread with its own HIP stream, so
batches admitted while others run overlap on the device.  A request whose
own footprint exceeds the whole budget is rejected, never left waiting.
Results are per-query top-K hits with score, begins, ends and CIGAR.

The backend interface (footprint, run) is all the scheduler needs, so the
scheduling logic is tested on the CPU with a backend of the tests' own.
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


@dataclasses.dataclass
class Request:
    rid: int
    queries: object            # SeqSet-like: .codes, .offsets, __len__, __getitem__
    arrival: float
    future: Future
    start: float = 0.0
    done: float = 0.0


class Seqs:
    """Concatenated sequences: uint8 codes plus int64 offsets (n + 1)."""

    def __init__(self, codes, offsets):
        self.codes = np.ascontiguousarray(codes, dtype=np.uint8)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)

    def __len__(self):
        return len(self.offsets) - 1

    def __getitem__(self, k):
        return self.codes[self.offsets[k]:self.offsets[k + 1]]


def concat(seqsets):
    """Concatenate sequence sets; returns (Seqs, per-set query index ranges)."""
    codes, offs, ranges = [], [0], []
    n = 0
    for s in seqsets:
        lo = n
        for k in range(len(s)):
            codes.append(np.asarray(s[k], dtype=np.uint8))
            offs.append(offs[-1] + len(codes[-1]))
            n += 1
        ranges.append((lo, n))
    return Seqs(np.concatenate(codes) if codes else np.zeros(0, np.uint8), np.array(offs)), ranges


class GpuBackend:
    """Backend on libdsa: one top-K search with hit traceback per batch."""

    def __init__(self, db, matrix, gap_open=11, gap_extend=1, top_k=10, traceback=True, mode="local"):
        self.db = db
        self.matrix = np.ascontiguousarray(matrix, dtype=np.int8)
        self.o, self.e = gap_open, gap_extend
        self.k = top_k
        self.traceback = traceback
        self.mode = mode

    def _args(self, queries, qcodes=None, stream=None):
        import torch
        import paper_1701_01575_amd as dsa
        if qcodes is None:
            qcodes = torch.zeros(max(len(queries.codes), 1), dtype=torch.uint8, device=self.db.device)
        return dsa.make_args(qcodes, queries.offsets, self.matrix, self.o, self.e, self.mode, db=self.db,
                             traceback=self.traceback, top_k=self.k, stream=stream)

    def footprint(self, queries) -> int:
        from . import binding as B
        a = self._args(queries)
        ws = B.dsa_workspace_size(a)
        n = len(queries) * self.k
        cig = B.dsa_cigar_capacity(a) * 4 if self.traceback else 0
        return int(ws + n * (4 * 5 + 8 + 8 + 1) + cig)

    def run(self, queries, stream) -> list:
        import torch
        import paper_1701_01575_amd as dsa
        from . import binding as B
        with torch.cuda.stream(stream):
            qc, qo = dsa.device_queries(queries, self.db.device)
            a = self._args(queries, qc, stream)
            need = B.dsa_workspace_size(a)
            ws = torch.empty(need + 256, dtype=torch.uint8, device=self.db.device)
            a.workspace = (ws.data_ptr() + 255) // 256 * 256
            a.workspace_bytes = need
            nr = len(queries) * self.k
            i32 = dict(dtype=torch.int32, device=self.db.device)
            out = {f: torch.empty(nr, **i32) for f in ("score", "q_begin", "q_end", "t_begin", "t_end")}
            out["t_index"] = torch.empty(nr, dtype=torch.int64, device=self.db.device)
            out["status"] = torch.empty(nr, dtype=torch.uint8, device=self.db.device)
            o = B.dsa_out()
            if self.traceback:
                cap = B.dsa_cigar_capacity(a)
                out["cigar_off"] = torch.empty(nr, dtype=torch.int64, device=self.db.device)
                out["cigar_len"] = torch.empty(nr, **i32)
                out["cigar_ops"] = torch.empty(max(cap, 1), dtype=torch.int32, device=self.db.device)
                o.cigar_capacity = cap
            for f, v in out.items():
                setattr(o, f, v.data_ptr())
            B.dsa_align_batch(a, o)
            stream.synchronize()
            host = {f: v.cpu().numpy() for f, v in out.items() if f != "cigar_ops"}
            cig = dsa.cigars(out) if self.traceback else None
        res = []
        for q in range(len(queries)):
            sl = slice(q * self.k, (q + 1) * self.k)
            r = {f: host[f][sl] for f in ("t_index", "score", "q_begin", "q_end", "t_begin", "t_end")}
            if cig is not None:
                r["cigars"] = cig[sl]
            res.append(r)
        return res

    def make_stream(self):
        import torch
        return torch.cuda.Stream(device=self.db.device)


class Server:
    """FIFO admission by HBM budget, continuous batching over `slots` streams."""

    def __init__(self, backend, hbm_budget_bytes: int, slots: int = 2, max_batch_queries: int = 64,
                 clock=time.monotonic):
        self.backend = backend
        self.budget = int(hbm_budget_bytes)
        self.slots = slots
        self.max_q = max_batch_queries
        self.clock = clock
        self.queue = collections.deque()
        self.cv = threading.Condition()
        self.in_flight = 0          # bytes held by running batches
        self.busy = 0               # running batches
        self.peak_in_flight = 0
        self.next_id = 0
        self.stopping = False
        self.completed = []         # finished requests (for statistics)
        self.rejected = 0
        self.batches = []           # (request ids, footprint) in dispatch order
        self.errors = 0
        self._threads = []

    # -- client side ------------------------------------------------------
    def submit(self, queries, arrival: float | None = None) -> Future:
        fut = Future()
        with self.cv:
            req = Request(self.next_id, queries, self.clock() if arrival is None else arrival, fut)
            self.next_id += 1
            self.queue.append(req)
            self.cv.notify_all()
        return fut

    def start(self):
        for k in range(self.slots):
            t = threading.Thread(target=self._worker, args=(k,), daemon=True)
            t.start()
            self._threads.append(t)
        return self

    def stop(self, wait: bool = True):
        with self.cv:
            self.stopping = True
            self.cv.notify_all()
        if wait:
            for t in self._threads:
                t.join()

    # -- scheduling -------------------------------------------------------
    def _take_batch(self):
        """Called with the lock held: pop a FIFO batch that fits, or None."""
        while self.queue:
            head = self.queue[0]
            need = self.backend.footprint(head.queries)
            if need > self.budget:
                self.queue.popleft()
                self.rejected += 1
                head.future.set_exception(AdmissionError(
                    f"request {head.rid} needs {need} bytes, budget is {self.budget}"))
                continue
            if self.in_flight + need > self.budget:
                return None  # FIFO: wait until running batches free memory
            batch, nq = [self.queue.popleft()], len(head.queries)
            while self.queue and nq + len(self.queue[0].queries) <= self.max_q:
                cand = self.queue[0]
                trial = batch + [cand]
                merged, _ = concat([r.queries for r in trial])
                need2 = self.backend.footprint(merged)
                if self.in_flight + need2 > self.budget:
                    break
                batch.append(self.queue.popleft())
                nq += len(cand.queries)
                need = need2
            return batch, need
        return None

    def _worker(self, slot: int):
        stream = self.backend.make_stream() if hasattr(self.backend, "make_stream") else None
        while True:
            with self.cv:
                got = None
                while not self.stopping:
                    got = self._take_batch()
                    if got is not None:
                        break
                    self.cv.wait()
                if got is None:
                    return
                batch, need = got
                self.in_flight += need
                self.busy += 1
                self.peak_in_flight = max(self.peak_in_flight, self.in_flight)
                self.batches.append(([r.rid for r in batch], need))
            t0 = self.clock()
            for r in batch:
                r.start = t0
            try:
                merged, ranges = concat([r.queries for r in batch])
                results = self.backend.run(merged, stream)
                t1 = self.clock()
                for r, (lo, hi) in zip(batch, ranges):
                    r.done = t1
                    r.future.set_result(results[lo:hi])
            except Exception as exc:
                # isolate the failure: rerun each request of the batch alone so
                # only the requests that fail by themselves report an error
                for r in batch:
                    try:
                        if len(batch) == 1:
                            raise exc
                        res = self.backend.run(concat([r.queries])[0], stream)
                        r.done = self.clock()
                        r.future.set_result(res)
                    except Exception as exc1:
                        r.done = self.clock()
                        r.future.set_exception(exc1)
                        with self.cv:
                            self.errors += 1
            with self.cv:
                self.in_flight -= need
                self.busy -= 1
                self.completed.extend(batch)
                self.cv.notify_all()

    # -- statistics -------------------------------------------------------
    def latencies(self):
        return np.array([r.done - r.arrival for r in self.completed if r.future.done()
                         and r.future.exception() is None])

    def stats(self) -> dict:
        lat = self.latencies()
        out = {"completed": len(self.completed), "rejected": self.rejected, "errors": self.errors,
               "batches": len(self.batches), "peak_in_flight_bytes": self.peak_in_flight,
               "budget_bytes": self.budget}
        if len(lat):
            out.update(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                       mean_s=float(lat.mean()))
        return out
