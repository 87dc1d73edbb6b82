"""Continuous-batching EMST server on one GPU.

Requests (point clouds) arrive over time.  Each of `workers` threads owns
one EMST context, one HIP stream and a fixed share of the HBM budget.  A
free worker immediately admits every queued request that fits its budget
(oldest first, at least one) and solves them together with
``emst_build_batched``; requests that arrive meanwhile wait for the next free
worker.  Several batches are therefore in flight on the device at once,
and a worker whose batch ends takes new requests right away (admission by
memory footprint, at batch granularity).  Every request's result is exactly
the EMST of its cloud alone: a batch only groups independent clouds.

Latency of a request = completion on the host - arrival.  The server
reports p50/p99 latency and Mpoints/s over the run.

``SolverServer`` is the round-granular form on the native solver: requests
join between any two steps (one Boruvka round of every running cohort)
instead of between batches.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from typing import Callable, List, Optional

import numpy as np

from . import Context, workspace_bytes_batched


@dataclasses.dataclass
class Request:
    rid: int
    points: np.ndarray          # [n, dim] float32 (host)
    arrival: float = 0.0        # seconds on the server clock
    start: float = 0.0
    done: float = 0.0
    edges: Optional[np.ndarray] = None
    weights: Optional[np.ndarray] = None
    d2: Optional[np.ndarray] = None
    error: Optional[str] = None
    batch: int = -1

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """`budget_bytes` is the device memory all workers together may use for
    inputs, outputs and workspaces; each worker gets an equal share."""

    def __init__(self, workers: int = 4, budget_bytes: int = 8 << 30, max_batch: int = 256,
                 device: int = 0):
        import torch
        self.device = device
        self.workers = workers
        self.share = budget_bytes // workers
        self.max_batch = max_batch
        self._queue: collections.deque = collections.deque()
        self._cv = threading.Condition()
        self._closed = False
        self._threads: List[threading.Thread] = []
        self._ctx = [Context(device) for _ in range(workers)]
        self._streams = [torch.cuda.Stream(device=device) for _ in range(workers)]
        self._batches = 0
        self.t0 = time.perf_counter()

    # ---- footprint of one request inside a batch
    @staticmethod
    def footprint(n: int, dim: int) -> int:
        # points + outputs + this request's share of the batched workspace
        return n * dim * 4 + max(n - 1, 0) * 16 + workspace_bytes_batched(max(n, 2), 1)

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> None:
        n, dim = req.points.shape
        if self.footprint(n, dim) > self.share:
            req.error = "EMST_ENOMEM: request larger than a worker's memory share"
            req.done = self.now()
            return
        with self._cv:
            req.arrival = self.now() if req.arrival == 0.0 else req.arrival
            self._queue.append(req)
            self._cv.notify()

    def start(self) -> None:
        for w in range(self.workers):
            t = threading.Thread(target=self._run, args=(w,), daemon=True)
            t.start()
            self._threads.append(t)

    def close(self) -> None:
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()

    def _admit(self) -> List[Request]:
        batch, used = [], 0
        while self._queue and len(batch) < self.max_batch:
            r = self._queue[0]
            f = self.footprint(*r.points.shape)
            if batch and used + f > self.share:
                break
            batch.append(self._queue.popleft())
            used += f
        return batch

    def _run(self, w: int) -> None:
        import torch
        ctx, stream = self._ctx[w], self._streams[w]
        while True:
            with self._cv:
                while not self._queue and not self._closed:
                    self._cv.wait()
                if not self._queue and self._closed:
                    return
                batch = self._admit()
                bid = self._batches
                self._batches += 1
            t = self.now()
            for r in batch:
                r.start, r.batch = t, bid
            try:
                with torch.cuda.stream(stream):
                    dev = [torch.from_numpy(r.points).to(f"cuda:{self.device}", non_blocking=False)
                           for r in batch]
                    out = ctx.build_batched(dev, stream=stream)
                    res = [(e.cpu().numpy(), wt.cpu().numpy(), d.cpu().numpy()) for e, wt, d in out]
                stream.synchronize()
                t_done = self.now()
                for r, (e, wt, d) in zip(batch, res):
                    r.edges, r.weights, r.d2 = e, wt, d
                    r.done = t_done
            except Exception as exc:  # a failing batch fails its own requests only
                t_done = self.now()
                for r in batch:
                    r.error = str(exc)
                    r.done = t_done


class FifoServer:
    """The one-request-per-launch baseline: one worker thread solves the
    queued requests one at a time, oldest first, each with its own
    ``emst_build`` on one stream."""

    def __init__(self, device: int = 0):
        import torch
        self.device = device
        self._ctx = Context(device)
        self._stream = torch.cuda.Stream(device=device)
        self._queue: collections.deque = collections.deque()
        self._cv = threading.Condition()
        self._closed = False
        self._thread: Optional[threading.Thread] = None
        self._served = 0
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> None:
        with self._cv:
            req.arrival = self.now() if req.arrival == 0.0 else req.arrival
            self._queue.append(req)
            self._cv.notify()

    def start(self) -> None:
        self._thread = threading.Thread(target=self._run, daemon=True)
        self._thread.start()

    def close(self) -> None:
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        if self._thread:
            self._thread.join()

    def _run(self) -> None:
        import torch
        while True:
            with self._cv:
                while not self._queue and not self._closed:
                    self._cv.wait()
                if not self._queue and self._closed:
                    return
                r = self._queue.popleft()
            r.start, r.batch = self.now(), self._served
            self._served += 1
            try:
                with torch.cuda.stream(self._stream):
                    pts = torch.from_numpy(r.points).to(f"cuda:{self.device}")
                    e, w, d = self._ctx.build(pts, stream=self._stream)
                    r.edges, r.weights, r.d2 = e.cpu().numpy(), w.cpu().numpy(), d.cpu().numpy()
                self._stream.synchronize()
            except Exception as exc:  # a failing request fails alone
                r.error = str(exc)
            r.done = self.now()


class SolverServer:
    """Round-granular continuous batching on the native solver
    (``emst_solver_*``): one driver thread admits every uploaded request
    that finds a slot and budget, steps the solver (the requests admitted
    since the last step start as one cohort, every cohort whose phase
    completed moves on by one phase: tree, one Boruvka round, edge order)
    and takes finished results.  A request arriving while others run joins
    the next cohort.  `copy_workers` threads, each with its own stream, copy
    the points of arriving requests to the device and finished results back,
    so that the driver thread only drives the solver."""

    def __init__(self, budget_bytes: int = 8 << 30, max_slots: int = 64, device: int = 0,
                 copy_workers: int = 4):
        import torch
        from . import Context, Solver
        self.device = device
        self._ctx = Context(device)
        self._solver = Solver(self._ctx, budget_bytes, max_slots)
        self._stream = torch.cuda.Stream(device=device)
        self.budget = budget_bytes
        self.copy_workers = max(1, copy_workers)
        self._ready: collections.deque = collections.deque()   # (request, device points)
        self._uploading = 0
        self._jobs: "queue.Queue" = queue.Queue()
        self._cv = threading.Condition()
        self._closed = False
        self._thread: Optional[threading.Thread] = None
        self._copiers: List[threading.Thread] = []
        self._steps = 0
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> None:
        n, dim = req.points.shape
        if self._solver.slot_bytes(n, dim) > self.budget:
            req.error = "EMST_ENOMEM: request larger than the solver budget"
            req.done = self.now()
            return
        with self._cv:
            req.arrival = self.now() if req.arrival == 0.0 else req.arrival
            self._uploading += 1
        self._jobs.put(("up", req))

    def start(self) -> None:
        for _ in range(self.copy_workers):
            t = threading.Thread(target=self._copy, daemon=True)
            t.start()
            self._copiers.append(t)
        self._thread = threading.Thread(target=self._run, daemon=True)
        self._thread.start()

    def close(self) -> None:
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        if self._thread:
            self._thread.join()
        for _ in self._copiers:
            self._jobs.put(None)
        for t in self._copiers:
            t.join()
        self._solver.close()

    def _copy(self) -> None:
        import torch
        stream = torch.cuda.Stream(device=self.device)
        while True:
            job = self._jobs.get()
            if job is None:
                return
            with torch.cuda.stream(stream):
                if job[0] == "up":
                    r = job[1]
                    try:
                        pts = torch.from_numpy(r.points).to(f"cuda:{self.device}")
                        stream.synchronize()
                    except Exception as exc:
                        r.error, r.done = str(exc), self.now()
                        pts = None
                    with self._cv:
                        if pts is not None:
                            self._ready.append((r, pts))
                        self._uploading -= 1
                        self._cv.notify_all()
                else:
                    _, ev, reqs, e, w, d, offs = job
                    stream.wait_event(ev)   # the solver's copies into e, w, d
                    edges, weights, d2 = e.cpu().numpy(), w.cpu().numpy(), d.cpu().numpy()
                    t = self.now()
                    for i, r in enumerate(reqs):
                        a, b = offs[i], offs[i + 1]
                        r.edges, r.weights, r.d2 = edges[a:b], weights[a:b], d2[a:b]
                        r.done = t

    def _run(self) -> None:
        import torch
        running = {}   # slot -> request
        while True:
            with self._cv:
                while not self._ready and not running and not (self._closed and not self._uploading):
                    self._cv.wait()
                if not self._ready and not running and self._closed and not self._uploading:
                    return
                ready = list(self._ready)
            with torch.cuda.stream(self._stream):
                for r, pts in ready:
                    slot = self._solver.admit(pts, tag=r.rid, stream=self._stream)
                    if slot is None:
                        break
                    pts.record_stream(self._stream)   # the solver copies it on this stream
                    with self._cv:
                        self._ready.popleft()
                    r.start = self.now()
                    r.batch = self._steps
                    running[slot] = r
                if not running:
                    continue
                self._solver.step(stream=self._stream)
                self._steps += 1
                ok = []
                for slot in self._solver.ready():
                    if self._solver.poll(slot)[0] == 2:
                        ok.append(slot)
                        continue
                    r = running.pop(slot)   # a failed request fails alone
                    try:
                        self._solver.take(slot, stream=self._stream)
                    except Exception as exc:
                        r.error = str(exc)
                    r.done = self.now()
                if ok:
                    e, w, d, offs = self._solver.take_many(ok, stream=self._stream)
                    ev = torch.cuda.Event()
                    ev.record(self._stream)
                    self._jobs.put(("down", ev, [running.pop(s) for s in ok], e, w, d, offs))


def replay(server, requests: List[Request], arrivals: List[float],
           on_submit: Optional[Callable[[Request], None]] = None) -> float:
    """Submit `requests` at the given arrival times (seconds from now) and
    wait for all of them; returns the makespan in seconds."""
    server.start()
    t_begin = server.now()
    for r, a in zip(requests, arrivals):
        target = t_begin + a
        while True:
            dt = target - server.now()
            if dt <= 0:
                break
            time.sleep(min(dt, 0.002))
        r.arrival = server.now()
        server.submit(r)
        if on_submit:
            on_submit(r)
    server.close()
    return max(r.done for r in requests) - t_begin


def summary(requests: List[Request], makespan: float) -> dict:
    ok = [r for r in requests if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    pts = sum(r.points.shape[0] for r in ok)
    return {
        "requests": len(requests), "failed": len(requests) - len(ok),
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3), "mpoints_per_s": pts / makespan / 1e6 if makespan > 0 else 0.0,
        "makespan_s": makespan, "batches": len({r.batch for r in ok}),
    }
