"""Serving loop: continuous batching of small shifted randomized ST-HOSVDs.

Requests (an FP32 order-3 tensor resident on the device, its ranks and seed)
arrive over time. The loop admits waiting requests into the next batch while
the batch fits the capacity and the workspace budget, writes the batch plan
(host only) and replays a graph captured once per slot: the library's
persistent batched kernels run every phase of Algorithm 3 for all requests
of the batch in one launch each. Two slots alternate, so the next batch is
planned while the previous one runs; a request's latency runs from its
arrival to the moment its batch's completion event is seen.

The one-at-a-time reference solves the same requests in arrival order with
one tucker_rsthosvd call each on a preallocated workspace.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import time
from typing import List, Optional, Sequence

import torch

from . import _lib as T


@dataclasses.dataclass
class Job:
    rid: int
    A: torch.Tensor
    ranks: tuple
    seed: int
    arrival: float
    G: Optional[torch.Tensor] = None
    U: Optional[List[torch.Tensor]] = None
    done: float = -1.0


def _alloc_outputs(job: Job, device) -> None:
    job.G = torch.empty(job.ranks, dtype=torch.float32, device=device)
    job.U = [torch.empty((n, r), dtype=torch.float32, device=device) for n, r in zip(job.A.shape, job.ranks)]


class _Slot:
    def __init__(self, capacity, q, p, lclass, ws_bytes, shift, device):
        self.solver = T.BatchSolver(capacity, 3, q, p, lclass, ws_bytes, shift, device)
        self.graph = None
        self.event = None
        self.jobs: List[Job] = []

    def capture(self):
        """Capture one step (on an empty plan) into a graph; replays run later plans."""
        self.solver.plan([])
        s = torch.cuda.Stream(device=self.solver.device)
        s.wait_stream(torch.cuda.current_stream(self.solver.device))
        with torch.cuda.stream(s):
            self.solver.step()  # warm the launch path outside capture
        torch.cuda.current_stream(self.solver.device).wait_stream(s)
        torch.cuda.synchronize(self.solver.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.solver.step()
        torch.cuda.synchronize(self.solver.device)


class BatchServer:
    """Continuous batching over two graph-replayed slots."""

    def __init__(self, capacity=256, q=1, p=8, lclass=48, ws_bytes=8 << 30, shift="adaptive", device="cuda",
                 use_graphs=True):
        self.device = torch.device(device)
        self.p, self.q = p, q
        self.slots = [_Slot(capacity, q, p, lclass, ws_bytes, shift, self.device) for _ in range(2)]
        self.capacity = capacity
        self.use_graphs = use_graphs
        if use_graphs:
            for s in self.slots:
                s.capture()
        self.budget = self.slots[0].solver.ws.numel() - self.slots[0].solver.table_bytes

    def _launch(self, slot: _Slot, jobs: List[Job]):
        items = [T.BatchSolver.item(j.A, j.G, j.U, j.ranks, j.seed) for j in jobs]
        slot.solver.plan(items)
        if self.use_graphs:
            slot.graph.replay()
        else:
            slot.solver.step()
        slot.event = torch.cuda.Event()
        slot.event.record()
        slot.jobs = jobs

    def run(self, jobs: Sequence[Job], t0: Optional[float] = None) -> List[Job]:
        """Serve `jobs` (arrival seconds relative to t0); returns them with .done set."""
        pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
        waiting: collections.deque = collections.deque()
        t0 = time.perf_counter() if t0 is None else t0
        sizer = self.slots[0].solver
        while pending or waiting or any(s.jobs for s in self.slots):
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            for s in self.slots:
                if s.jobs and s.event.query():
                    t = time.perf_counter() - t0
                    for j in s.jobs:
                        j.done = t
                    s.jobs = []
            free = [s for s in self.slots if not s.jobs]
            if free and waiting:
                batch, used = [], 0
                while waiting and len(batch) < self.capacity:
                    j = waiting[0]
                    if j.G is None:
                        _alloc_outputs(j, self.device)
                    need = sizer.item_bytes(T.BatchSolver.item(j.A, j.G, j.U, j.ranks, j.seed))
                    if batch and used + need > self.budget:
                        break
                    batch.append(waiting.popleft())
                    used += need
                self._launch(free[0], batch)
                continue
            if not pending and not waiting:
                time.sleep(20e-6)
            elif pending and not waiting:
                time.sleep(min(200e-6, max(0.0, pending[0].arrival - now)))
            else:
                time.sleep(20e-6)
        return list(jobs)


class SingleServer:
    """One request at a time: tucker_rsthosvd per request, in arrival order."""

    def __init__(self, p=8, q=1, shift="adaptive", ws_bytes=256 << 20, device="cuda"):
        self.device = torch.device(device)
        self.p, self.q, self.shift = p, q, T._SHIFT[shift]
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)

    def _solve(self, j: Job):
        s = T._shape(j.A.shape)
        r = (ctypes.c_int64 * 3)(*j.ranks)
        u = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in j.U])
        T._check(T.lib.tucker_rsthosvd(ctypes.byref(s), ctypes.c_void_p(j.A.data_ptr()), r, self.p, self.q,
                                       self.shift, ctypes.c_uint64(j.seed), T.FP32,
                                       ctypes.c_void_p(j.G.data_ptr()), u, None,
                                       ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_size_t(self.ws.numel()),
                                       T._stream(self.device)))

    def run(self, jobs: Sequence[Job], t0: Optional[float] = None) -> List[Job]:
        order = sorted(jobs, key=lambda j: j.arrival)
        t0 = time.perf_counter() if t0 is None else t0
        inflight = collections.deque()
        for j in order:
            while time.perf_counter() - t0 < j.arrival:
                while inflight and inflight[0][1].query():
                    jj, _ = inflight.popleft()
                    jj.done = time.perf_counter() - t0
                time.sleep(20e-6)
            if j.G is None:
                _alloc_outputs(j, self.device)
            self._solve(j)
            ev = torch.cuda.Event()
            ev.record()
            inflight.append((j, ev))
            while inflight and inflight[0][1].query():
                jj, _ = inflight.popleft()
                jj.done = time.perf_counter() - t0
        while inflight:
            jj, ev = inflight.popleft()
            ev.synchronize()
            jj.done = time.perf_counter() - t0
        return list(order)


def latency_stats(jobs: Sequence[Job]) -> dict:
    lat = sorted(j.done - j.arrival for j in jobs)
    if not lat:
        return {}
    pick = lambda f: lat[min(len(lat) - 1, int(f * len(lat)))]
    span = max(j.done for j in jobs) - min(j.arrival for j in jobs)
    return {"count": len(lat), "p50_ms": 1e3 * pick(0.5), "p99_ms": 1e3 * pick(0.99), "max_ms": 1e3 * lat[-1],
            "span_s": span, "approx_per_s": len(lat) / span if span > 0 else float("inf")}
