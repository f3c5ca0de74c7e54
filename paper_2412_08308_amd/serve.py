"""Serving loop: continuous batching of database-search requests on one GPU.

Requests (single queries) arrive at any time through ``Server.submit``.  A
scheduler thread

* admits requests while the in-flight slot count and the device-memory
  budget allow (each batch needs its workspace from ``sw_workspace_bytes``,
  its score matrix and its query bytes), in order of deadline (``policy=
  "edf"``: arrival time plus the request's estimated service time, its cells
  over the device rate observed on completed batches, so a short request
  overtakes long ones that arrived about as early, while no deadline moves)
  or of arrival (``policy="fifo"``);
* groups admissible requests of similar size into one batched launch
  (``sw_db_search_batch``) on a free stream of a small stream pool, so batches
  that arrive while others run are searched concurrently on the device: a
  batch takes the first pending request and those within ``size_ratio`` of
  its cells (a short request never waits for a long one in its own batch),
  and requests longer than ``long_s`` of estimated device time may hold all
  but one of the in-flight slots, so a short request always finds a slot;
* the GPU backend cuts each batch's work into persistent launches of a few
  milliseconds (``slice_mcells``).  A batch holding a long request is
  *stepped*: the scheduler enqueues its launches itself, at most
  ``long_depth`` of them outstanding over all long batches (earliest deadline
  first), and none while a batch of short requests is in flight, so a short
  request waits at most for the long launches already queued instead of
  sharing the device with them for its whole run;
* records a completion event per batch (after an asynchronous copy of the
  scores to pinned host memory) and resolves each request's future when it
  fires, with the latency (completion - arrival) attached.

Scores are exact integers, so a request's result is identical whether it runs
alone or inside any batch.  ``GpuBackend`` does the device work through the
library; the scheduler itself only needs the small backend interface
(``need_bytes``, ``launch``, ``poll``, ``results``, ``cells``; stepped
batches also ``advance``, ``remaining`` and ``queued``).
"""
from __future__ import annotations

import collections
import itertools
import threading
import time
from concurrent.futures import Future
from typing import List, Optional, Sequence

import numpy as np


class Request:
    __slots__ = ("id", "query", "qlen", "arrival", "future", "started", "deadline")

    def __init__(self, rid, query, arrival):
        self.id = rid
        self.query = query
        self.qlen = int(len(query)) if not hasattr(query, "numel") else int(query.numel())
        self.arrival = arrival
        self.deadline = arrival
        self.future = Future()
        self.future.latency = None
        self.future.request_id = rid
        self.started = False


def percentiles(latencies: Sequence[float]):
    """(p50, p99) by linear interpolation between order statistics."""
    if len(latencies) == 0:
        return None, None
    x = np.sort(np.asarray(latencies, dtype=np.float64))
    return float(np.percentile(x, 50)), float(np.percentile(x, 99))


class GpuBackend:
    """Batched searches on a pool of HIP streams through ``Database.search_batch``."""

    def __init__(self, db, matrix, gap_open: int, gap_extend: int, mode="auto", n_streams: int = 4,
                 slice_mcells: int = 0, **opt_kw):
        import torch

        from . import options
        self.torch = torch
        self.db = db
        self.matrix = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
        self.go, self.ge = int(gap_open), int(gap_extend)
        self._opt_kw = dict(mode=mode, slice_mcells=slice_mcells, **opt_kw)
        self.opt = options(**self._opt_kw)
        self.device = db.device
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.nseq = db.nseq

    @property
    def slots(self) -> int:
        return len(self.streams)

    def need_bytes(self, qlens: Sequence[int]) -> int:
        ws = self.db.workspace_bytes(list(qlens), self.opt)
        return ws + 4 * len(qlens) * self.nseq + int(sum(qlens))

    def cells(self, qlens: Sequence[int]) -> int:
        return int(sum(qlens)) * self.db.total

    def launch(self, slot: int, queries: List[np.ndarray], stepped: bool = False):
        """Enqueue a batch on stream ``slot``: all of its launches, or with
        ``stepped`` (and slicing on) none yet -- ``advance`` enqueues them one
        at a time."""
        torch = self.torch
        s = self.streams[slot]
        lens = [len(q) for q in queries]
        offs = np.zeros(len(lens), dtype=np.int64)
        if len(lens) > 1:
            offs[1:] = np.cumsum(lens[:-1])
        with torch.cuda.stream(s):
            host = torch.from_numpy(np.concatenate(queries) if sum(lens) else np.zeros(1, np.uint8)).pin_memory()
            cat = host.to(self.device, non_blocking=True)
            ws = self.db.alloc_workspace(lens, self.opt)
            out = torch.empty((len(lens), self.nseq), dtype=torch.int32, device=self.device)
        h = {"stream": s, "args": (cat, offs, lens), "ws": ws, "out": out, "keep": (host,),
             "next": 0, "total": 1, "slice_events": collections.deque(), "event": None}
        if stepped and self.opt.slice_mcells > 0 and sum(lens) > 0:
            h["total"] = int(self.db.plan_info(lens, self.opt)["launches"])
        if h["total"] <= 1 or not stepped:
            self._enqueue(h, None)
        return h

    def _enqueue(self, h, k):
        """Enqueue launch k of the batch (None: all of them); after the last
        one, the status and score copies and the completion event."""
        torch = self.torch
        s = h["stream"]
        opt = self.opt if k is None else options_for(self._opt_kw, slice_begin=k, slice_count=1)
        with torch.cuda.stream(s):
            self.db.search_batch(h["args"], self.matrix, self.go, self.ge, opt=opt, out=h["out"],
                                 workspace=h["ws"], stream=s, check=False)
            h["next"] = h["total"] if k is None else k + 1
            ev = torch.cuda.Event()
            if h["next"] >= h["total"]:
                status = torch.zeros(4, dtype=torch.int32, pin_memory=True)
                self.db.status_async(h["ws"], status, stream=s)
                res = torch.empty(tuple(h["out"].shape), dtype=torch.int32, pin_memory=True)
                res.copy_(h["out"], non_blocking=True)
                h["status"], h["res"] = status, res
                ev.record(s)
                h["event"] = ev
            else:
                ev.record(s)
            h["slice_events"].append(ev)

    def advance(self, handle):
        """Enqueue the stepped batch's next launch."""
        if handle["next"] < handle["total"]:
            self._enqueue(handle, handle["next"])

    def remaining(self, handle) -> int:
        """Launches of the batch not enqueued yet."""
        return handle["total"] - handle["next"]

    def queued(self, handle) -> int:
        """Enqueued launches of the batch that have not finished."""
        q = handle["slice_events"]
        while q and q[0].query():
            q.popleft()
        return len(q)

    def poll(self, handle) -> bool:
        return handle["event"] is not None and handle["event"].query()

    def results(self, handle) -> List[np.ndarray]:
        """Score rows of a finished batch; raises the batch's status error (a
        residue code >= 32, an incomplete exact rescore) instead."""
        from . import status_error
        handle["event"].synchronize()
        err = status_error(handle["status"])
        if err is not None:
            raise err
        r = handle["res"].numpy()
        return [r[k].copy() for k in range(r.shape[0])]


def options_for(kw: dict, **more):
    from . import options
    return options(**{**kw, **more})


class Server:
    """Continuous-batching request loop (see module docstring)."""

    def __init__(self, backend, max_batch: int = 16, max_inflight: Optional[int] = None,
                 mem_budget: Optional[int] = None, poll_interval: float = 1e-4, clock=time.perf_counter,
                 policy: str = "edf", rate_guess: float = 1e12, size_ratio: float = 4.0,
                 long_s: float = 0.02, long_depth: int = 2):
        if policy not in ("edf", "fifo"):
            raise ValueError("policy must be 'edf' or 'fifo'")
        if long_depth < 1:
            raise ValueError("long_depth must be >= 1")
        self.policy = policy
        self.long_depth = int(long_depth)   # outstanding launches of stepped (long) batches
        self.stepping = all(hasattr(backend, f) for f in ("advance", "remaining", "queued"))
        self.size_ratio = float(size_ratio)   # 0: batch regardless of size
        self.long_s = float(long_s)           # estimated device time that makes a request long
        self.rate = float(rate_guess)       # cells per second, updated from completed batches
        self.nominal_rate = float(rate_guess)   # the rate that classes requests as long (fixed)
        self.backend = backend
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight or getattr(backend, "slots", 4))
        if mem_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            mem_budget = int(free * 0.5)
        self.mem_budget = int(mem_budget)
        self.poll_interval = poll_interval
        self.clock = clock
        self._ids = itertools.count()
        self._pending = collections.deque()
        self._inflight = []            # (slot, handle, requests, bytes, launch time)
        self._free_slots = list(range(self.max_inflight))
        self._in_use = 0
        self._cv = threading.Condition()
        self._running = False
        self._thread = None
        self.latencies = []
        self.by_qlen = []              # (query length, latency) of completed requests
        self.completed = 0
        self.cells_done = 0
        self.first_arrival = None
        self.last_completion = None
        self.max_in_use = 0
        self.batch_sizes = []
        self.errors = []
        self._failed = None            # the error that stopped the scheduler, if any
        self._stepped = set()          # ids of in-flight handles whose launches the scheduler enqueues

    # ------------------------------------------------------------------ client side

    def submit(self, query) -> Future:
        """Queue one query (uint8 codes < 32, numpy); returns a Future of its scores."""
        q = np.ascontiguousarray(np.asarray(query))
        if q.dtype != np.uint8 or q.ndim != 1:
            raise ValueError("query must be a 1-D uint8 array of residue codes")
        if len(q) and int(q.max()) >= 32:
            raise ValueError("query residue codes must be < 32")
        now = self.clock()
        req = Request(next(self._ids), q, now)
        req.deadline = now + self.backend.cells([req.qlen]) / self.rate
        need = self.backend.need_bytes([req.qlen])
        if need > self.mem_budget:
            req.future.set_exception(MemoryError(f"request needs {need} bytes, budget {self.mem_budget}"))
            return req.future
        with self._cv:
            if self._failed is not None:
                req.future.set_exception(RuntimeError(f"server stopped after an error: {self._failed!r}"))
                return req.future
            if self.first_arrival is None:
                self.first_arrival = now
            self._pending.append(req)
            self._cv.notify()
        return req.future

    def start(self):
        if self._thread is None:
            self._running = True
            self._thread = threading.Thread(target=self._loop, name="swdb-serve", daemon=True)
            self._thread.start()
        return self

    def stop(self, drain: bool = True, timeout: Optional[float] = None):
        with self._cv:
            if not drain:
                while self._pending:
                    r = self._pending.popleft()
                    r.future.cancel()
            self._running = False
            self._cv.notify()
        if self._thread is not None:
            self._thread.join(timeout)
            self._thread = None

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop(drain=True)

    def stats_by_length(self, edges: Sequence[int]) -> List[dict]:
        """p50 / p99 latency per query-length class: lengths below edges[0],
        between consecutive edges, and from edges[-1] up."""
        bounds = [0] + [int(e) for e in edges] + [1 << 62]
        out = []
        for lo, hi in zip(bounds[:-1], bounds[1:]):
            lat = [x for m, x in self.by_qlen if lo <= m < hi]
            p50, p99 = percentiles(lat)
            out.append({"qlen_lo": lo, "qlen_hi": hi if hi < (1 << 62) else None, "requests": len(lat),
                        "p50_s": p50, "p99_s": p99})
        return out

    def stats(self) -> dict:
        p50, p99 = percentiles(self.latencies)
        span = (self.last_completion - self.first_arrival) if self.completed else None
        return {"completed": self.completed, "p50_s": p50, "p99_s": p99,
                "sustained_gcups": (self.cells_done / span / 1e9) if span else None,
                "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else None,
                "max_batch": max(self.batch_sizes) if self.batch_sizes else 0,
                "max_bytes_in_use": self.max_in_use, "errors": len(self.errors)}

    # ------------------------------------------------------------------ scheduler

    def _complete(self):
        done = []
        for entry in self._inflight:
            slot, h, reqs, nbytes, t_launch = entry
            if self.backend.poll(h):
                done.append(entry)
        stepped = set(self._stepped)
        for entry in done:
            slot, h, reqs, nbytes, t_launch = entry
            self._inflight.remove(entry)
            self._stepped.discard(id(h))
            try:
                rows = self.backend.results(h)
                err = None
            except Exception as e:           # a failed batch fails its own requests only
                rows, err = None, e
            t = self.clock()
            for k, r in enumerate(reqs):
                if err is not None:
                    r.future.set_exception(err)
                    self.errors.append(err)
                    continue
                r.future.latency = t - r.arrival
                self.latencies.append(r.future.latency)
                self.by_qlen.append((r.qlen, r.future.latency))
                self.completed += 1
                r.future.set_result(rows[k])
            if err is None:
                cells = self.backend.cells([r.qlen for r in reqs])
                self.cells_done += cells
                self.last_completion = t
                if t > t_launch and cells > 0 and len(self._inflight) == 0 and id(h) not in stepped:
                    # rate of a batch that ran alone at the end, all its launches
                    # enqueued at once (a stepped batch's time includes the
                    # launches held back for others): an estimate of the device rate
                    self.rate = 0.7 * self.rate + 0.3 * cells / (t - t_launch)
            with self._cv:
                self._in_use -= nbytes
                self._free_slots.append(slot)
        return bool(done)

    def _admit(self):
        launched = False
        while True:
            with self._cv:
                if not self._free_slots or not self._pending:
                    return launched
                batch, lens = [], []
                if self.policy == "edf" and len(self._pending) > 1:
                    self._pending = collections.deque(sorted(self._pending, key=lambda r: (r.deadline, r.id)))
                while self._pending and self._pending[0].future.cancelled():
                    self._pending.popleft()
                if not self._pending:
                    return launched
                head = self._pending[0]
                head_cells = max(self.backend.cells([head.qlen]), 1)
                if (self.max_inflight >= 2 and self._is_long(head.qlen)
                        and self._long_inflight() >= self.max_inflight - 1):
                    # the last free slot stays for a request that is not long
                    short = next((r for r in self._pending if not self._is_long(r.qlen)
                                  and not r.future.cancelled()), None)
                    if short is None:
                        return launched
                    head, head_cells = short, max(self.backend.cells([short.qlen]), 1)
                keep = collections.deque()
                for r in list(self._pending):
                    if len(batch) >= self.max_batch or r.future.cancelled():
                        if not r.future.cancelled():
                            keep.append(r)
                        continue
                    c = self.backend.cells([r.qlen])
                    similar = r is head or self.size_ratio <= 0 or (
                        head_cells / self.size_ratio <= c <= head_cells * self.size_ratio
                        and (not self._is_long(r.qlen) or self._is_long(head.qlen)))
                    need = self.backend.need_bytes(lens + [r.qlen])
                    if (not batch and r is not head) or not similar or self._in_use + need > self.mem_budget:
                        keep.append(r)
                        continue
                    batch.append(r)
                    lens.append(r.qlen)
                if not batch:
                    return launched
                self._pending = keep
                nbytes = self.backend.need_bytes(lens)
                slot = self._free_slots.pop()
                self._in_use += nbytes
                self.max_in_use = max(self.max_in_use, self._in_use)
            live = []
            for r in batch:
                if r.future.set_running_or_notify_cancel():     # False: cancelled meanwhile
                    r.started = True
                    live.append(r)
            if len(live) != len(batch):
                with self._cv:
                    self._in_use -= nbytes
                    if not live:
                        self._free_slots.append(slot)
                        continue
                    nbytes = self.backend.need_bytes([r.qlen for r in live])
                    self._in_use += nbytes
                batch = live
            stepped = self.stepping and any(self._is_long(r.qlen) for r in batch)
            try:
                if stepped:
                    h = self.backend.launch(slot, [r.query for r in batch], stepped=True)
                else:
                    h = self.backend.launch(slot, [r.query for r in batch])
            except Exception as e:
                for r in batch:
                    r.future.set_exception(e)
                self.errors.append(e)
                with self._cv:
                    self._in_use -= nbytes
                    self._free_slots.append(slot)
                continue
            self.batch_sizes.append(len(batch))
            self._inflight.append((slot, h, batch, nbytes, self.clock()))
            if stepped:
                self._stepped.add(id(h))
            launched = True

    def _advance(self) -> bool:
        """Enqueue launches of stepped batches: none while a batch that is
        not stepped is in flight, else up to long_depth outstanding, earliest
        deadline first."""
        if not self._stepped:
            return False
        stepped = [e for e in self._inflight if id(e[1]) in self._stepped]
        if len(stepped) < len(self._inflight):
            return False
        outstanding = sum(self.backend.queued(e[1]) for e in stepped)
        moved = False
        for e in sorted(stepped, key=lambda e: min(r.deadline for r in e[2])):
            h = e[1]
            while outstanding < self.long_depth and self.backend.remaining(h) > 0:
                try:
                    self.backend.advance(h)
                except Exception as err:          # a failed launch fails its own batch only
                    self._drop(e, err)
                    break
                outstanding += 1
                moved = True
        return moved

    def _drop(self, entry, err):
        """Fail an in-flight batch whose launch could not be enqueued and
        give back its slot and memory."""
        slot, h, reqs, nbytes, _ = entry
        if entry in self._inflight:
            self._inflight.remove(entry)
        self._stepped.discard(id(h))
        self.errors.append(err)
        for r in reqs:
            if not r.future.done():
                r.future.set_exception(err)
        with self._cv:
            self._in_use -= nbytes
            self._free_slots.append(slot)

    def _is_long(self, qlen: int) -> bool:
        # by the nominal rate: a class that does not drift with the estimate
        return self.backend.cells([qlen]) / self.nominal_rate > self.long_s

    def _long_inflight(self) -> int:
        return sum(1 for _, _, reqs, _, _ in self._inflight if any(self._is_long(r.qlen) for r in reqs))

    def _loop(self):
        try:
            while True:
                progressed = self._complete()
                progressed |= self._admit()
                progressed |= self._advance()
                with self._cv:
                    if not self._running and not self._pending and not self._inflight:
                        return
                    if not progressed:
                        if self._inflight:
                            self._cv.wait(self.poll_interval)
                        else:
                            self._cv.wait(0.05)
        except BaseException as e:          # e.g. an asynchronous device error raised by poll()
            self._fail_all(e)

    def _fail_all(self, err):
        """The scheduler cannot go on: fail every pending and in-flight request
        with ``err`` and stop accepting work."""
        self.errors.append(err)
        with self._cv:
            self._failed = err
            self._running = False
            reqs = [r for _, _, batch, _, _ in self._inflight for r in batch] + list(self._pending)
            self._inflight = []
            self._stepped.clear()
            self._pending.clear()
        for r in reqs:
            if not r.future.done():
                if not r.started and not r.future.set_running_or_notify_cancel():
                    continue
                r.future.set_exception(err)
