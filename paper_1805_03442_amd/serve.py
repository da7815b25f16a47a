"""Continuous-batching server for MUSCL solves of different sizes and gases.

Requests (1D or 2D grid, gas parameters, initial state, end time) arrive over
time.  The server keeps one batch (``ng_batch_*``) resident on the GPU and, at
every tick:
  1. admits waiting requests, in arrival order, whenever a batch slot and
     enough of the device arena (the HBM budget) are free -- a small request
     may pass a large one that is still waiting for memory; a request's
     initial state is prepared only once it fits, or ahead of time on host
     threads for the first ``prefetch`` requests of the queue;
  2. advances every admitted, unfinished solve by ``tick_steps`` steps, each
     with its own dt (eq. (16)) and end time, in one step kernel per
     dimension -- enqueued before the admissions of step 1, so that the host
     work of admitting overlaps the steps on the GPU;
  3. collects the solves that reached their end time, releases their slots
     and arena space, and records their latency (finish - arrival).
A solve's arithmetic does not depend on what else is in the batch, so each
result is the one it would have alone.

The backend is any object with the methods of ``GpuBackend``; tests drive the
bookkeeping with a CPU stand-in.
"""
from __future__ import annotations

import collections
import math
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    id: int
    arrival: float          # seconds from the start of the trace
    nx: int
    ny: int
    gas: dict
    t_end: float
    W: object = None        # primitive initial state, or a callable producing it
    admitted: float = math.nan
    finished: float = math.nan
    steps: int = 0
    failed: bool = False    # a step was rejected (non-physical state), or the request was refused
    slot: int = -1
    result: object = None

    _future: object = field(default=None, repr=False)

    def prefetch(self, pool):
        """Start preparing the initial state on a host thread."""
        if self._future is None and callable(self.W):
            self._future = pool.submit(self.W)

    def state(self):
        if self._future is not None:
            f, self._future = self._future, None
            return f.result()
        return self.W() if callable(self.W) else self.W


@dataclass
class Stats:
    completed: list = field(default_factory=list)
    wall: float = 0.0
    ticks: int = 0
    queued_max: int = 0
    resident_max: int = 0
    cell_updates: float = 0.0          # work of the completed solves
    cell_updates_all: float = 0.0      # work of every solve, finished or not
    admit_s: float = 0.0               # host time spent admitting
    step_s: float = 0.0                # time spent in run + poll

    def summary(self, pending: int, waiting: int, unsubmitted: int) -> dict:
        lat = np.array([r.finished - r.arrival for r in self.completed])
        qd = np.array([r.admitted - r.arrival for r in self.completed])
        out = dict(completed=len(self.completed),
                   failed=sum(1 for r in self.completed if r.failed),
                   wall_s=self.wall, ticks=self.ticks,
                   solves_per_s=len(self.completed) / self.wall if self.wall > 0 else 0.0,
                   cell_updates_per_s=self.cell_updates / self.wall if self.wall > 0 else 0.0,
                   cell_updates_per_s_all=(self.cell_updates_all / self.wall
                                           if self.wall > 0 else 0.0),
                   admit_s=self.admit_s, step_s=self.step_s,
                   resident_max=self.resident_max, queued_max=self.queued_max,
                   still_running=pending, still_queued=waiting, not_yet_arrived=unsubmitted)
        if len(lat):
            out.update(p50_latency_s=float(np.percentile(lat, 50)),
                       p99_latency_s=float(np.percentile(lat, 99)),
                       mean_queue_s=float(qd.mean()))
        return out


class GpuBackend:
    """One FP32 (or FP64) batch in a device arena of ``budget_bytes``."""

    def __init__(self, capacity: int, budget_bytes: int, precision=None, keep_results=False):
        from . import ng
        self.ng = ng
        self.precision = ng.NG_FP32 if precision is None else precision
        self.batch = ng.Batch(capacity, int(budget_bytes), precision=self.precision)
        self.keep_results = keep_results
        self.state_s = 0.0      # host time waiting for initial states
        self.add_s = 0.0        # host time in ng_batch_add (conversion, upload)

    def solve_bytes(self, nx, ny):
        return self.ng.Batch.solve_bytes(nx, ny, self.precision)

    def fits(self, nx, ny):
        return self.batch.fits(nx, ny)

    def add(self, req: Request):
        """The slot, None when there is no room yet; ValueError for a request
        the library refuses (invalid parameters or initial state)."""
        t0 = time.perf_counter()
        W = req.state()
        t1 = time.perf_counter()
        try:
            slot = self.batch.add(req.gas, req.nx, req.ny, W, t_end=req.t_end)
        except self.ng.NgError as e:
            if e.code == self.ng.NG_EINVAL:
                raise ValueError(str(e)) from e
            raise
        finally:
            self.state_s += t1 - t0
            self.add_s += time.perf_counter() - t1
        return slot

    def run(self, nsteps: int):
        self.batch.run(nsteps)

    def poll(self):
        return self.batch.poll()

    def steps(self, slot):
        return self.batch.diagnostics(slot)["steps"]

    def failed(self, slot):
        return self.batch.diagnostics(slot)["status"] != 0

    def result(self, slot):
        return self.batch.conserved(slot) if self.keep_results else None

    def remove(self, slot):
        self.batch.remove(slot)

    def close(self):
        self.batch.close()


class Server:
    def __init__(self, backend, capacity: int, tick_steps: int = 32, clock=time.perf_counter,
                 sleep=time.sleep, prefetch: int = 0, prefetch_threads: int = 4):
        self.backend = backend
        self.prefetch = prefetch
        self._pool = ThreadPoolExecutor(max_workers=prefetch_threads) if prefetch > 0 else None
        self.capacity = capacity
        self.tick_steps = tick_steps
        self.clock = clock
        self.sleep = sleep
        self.queue: collections.deque = collections.deque()
        self.running: dict = {}     # slot -> Request
        self.rejected: list = []
        self.stats = Stats()
        self.t0 = None

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request):
        self.queue.append(req)
        self.stats.queued_max = max(self.stats.queued_max, len(self.queue))

    def _admit(self):
        if not self.queue or len(self.running) >= self.capacity:
            return
        keep = collections.deque()
        while self.queue:
            req = self.queue.popleft()
            if len(self.running) >= self.capacity or not self.backend.fits(req.nx, req.ny):
                keep.append(req)    # no slot or arena space yet: keep waiting
                continue
            try:
                slot = self.backend.add(req)
            except ValueError:
                req.failed = True       # refused by the library: never admitted
                self.rejected.append(req)
                continue
            if slot is None:
                keep.append(req)
                continue
            req.slot = slot
            req.admitted = self.now()
            self.running[slot] = req
        if not self.running:
            # nothing resident and still not admitted: larger than the arena
            self.rejected.extend(keep)
            keep = collections.deque()
        self.queue = keep
        if self._pool is not None:
            for req in list(self.queue)[:self.prefetch]:
                req.prefetch(self._pool)
        self.stats.resident_max = max(self.stats.resident_max, len(self.running))

    def tick(self):
        # the steps of the resident solves are enqueued first, so that the
        # admission work on the host (state preparation, conversion, upload)
        # overlaps them; solves admitted now join at the next tick
        t0 = self.clock()
        if self.running:
            self.backend.run(self.tick_steps)
        t1 = self.clock()
        self._admit()
        t2 = self.clock()
        self.stats.admit_s += t2 - t1
        if self.running:
            done = self.backend.poll()
            self.stats.step_s += (t1 - t0) + (self.clock() - t2)
            for slot in done:
                req = self.running.pop(slot)
                req.finished = self.now()
                req.steps = self.backend.steps(slot)
                req.failed = self.backend.failed(slot)
                req.result = self.backend.result(slot)
                self.backend.remove(slot)
                self.stats.completed.append(req)
                self.stats.cell_updates += float(req.nx) * req.ny * req.steps
        self.stats.ticks += 1

    def run_trace(self, trace, max_wall: float = 60.0, drain: bool = True,
                  lookahead: float = 0.0) -> dict:
        """Replay ``trace`` (requests sorted by arrival) in real time; stop at
        ``max_wall`` seconds, or when every request has finished.  With a
        prefetch pool, the states of requests arriving within ``lookahead``
        seconds are prepared before they arrive (a client that has its data
        ready when it submits)."""
        self.t0 = self.clock()
        pending = list(trace)
        i = 0
        ahead = 0
        while True:
            now = self.now()
            if self._pool is not None:
                while ahead < len(pending) and pending[ahead].arrival <= now + lookahead:
                    pending[ahead].prefetch(self._pool)
                    ahead += 1
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            if self.running or self.queue:
                self.tick()
            elif i < len(pending):
                # idle until the next arrival
                wait = pending[i].arrival - self.now()
                if wait > 0:
                    self.sleep(min(wait, 0.01))
            else:
                break
            if self.now() > max_wall:
                break
            if not drain and i >= len(pending):
                break
        self.stats.wall = self.now()
        self.stats.cell_updates_all = self.stats.cell_updates + sum(
            float(r.nx) * r.ny * self.backend.steps(slot) for slot, r in self.running.items())
        if self._pool is not None:
            self._pool.shutdown(wait=False, cancel_futures=True)
        out = self.stats.summary(len(self.running), len(self.queue), len(pending) - i)
        out["rejected"] = len(self.rejected)
        return out


def requests_from_trace(trace_dicts, state_fn):
    """Request objects from serve_trace() records; states drawn lazily."""
    out = []
    for r in trace_dicts:
        out.append(Request(id=r["id"], arrival=r["arrival"], nx=r["nx"], ny=r["ny"],
                           gas=r["gas"], t_end=r["t_end"], W=(lambda rr=r: state_fn(rr))))
    return out
