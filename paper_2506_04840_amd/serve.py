"""Serving loop: continuous batching of small shifted randomized ST-HOSVDs.

Requests (an FP32 tensor resident on the device, its Tucker ranks and seed)
arrive over time. The loop admits waiting requests into the next batch while
the batch fits the capacity and the workspace budget, writes the batch plan
(host only) and replays a graph captured once per slot: the library's
persistent batched kernels run every phase of Algorithm 3 for all requests of
the batch in one launch each. Requests of different orders go to different
slot pairs (a plan holds one order). Each slot has its own stream and
workspace, so two batches run on the device at once: the latency-bound small
SVD and orthonormalisation phases of one overlap the bandwidth-bound mode
products of the other, and a batch is admitted and planned as soon as a slot
is free. A request's latency runs from its arrival to the moment its batch's
completion event is seen by the loop.

A request's descriptor (shape, ranks, seed and device pointers of A, G and the
U_k) is built once when the request is made (Job.prepare), as a client would
hand over its buffers; admission reads only its workspace size.

The one-at-a-time reference solves the same requests in arrival order with
one tucker_rsthosvd call each (FP32, same p, q, shift and seed) on a
preallocated workspace.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

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
    item: Optional[T.BatchItem] = None
    ws_bytes: int = 0
    done: float = -1.0

    def prepare(self, p: int, q: int) -> "Job":
        """Allocate G and the U_k on A's device and build the request's descriptor."""
        if self.A.dtype != torch.float32:
            raise ValueError("served requests are FP32")
        dev = self.A.device
        self.G = torch.empty(self.ranks, dtype=torch.float32, device=dev)
        self.U = [torch.empty((n, r), dtype=torch.float32, device=dev) for n, r in zip(self.A.shape, self.ranks)]
        self.item = T.BatchSolver.item(self.A, self.G, self.U, self.ranks, self.seed)
        nb = T.lib.tucker_batch_item_bytes(ctypes.byref(self.item), p, q)
        if nb == 0:
            raise ValueError("request %d: invalid shape or ranks" % self.rid)
        self.ws_bytes = int(nb)
        return self


class _Slot:
    def __init__(self, capacity, order, q, p, lclass, ws_bytes, shift, device):
        self.solver = T.BatchSolver(capacity, order, q, p, lclass, ws_bytes, shift, device)
        self.stream = torch.cuda.Stream(device=self.solver.device)  # default priority
        self.graph = None
        self.event = None
        self.jobs: List[Job] = []

    def capture(self):
        """Capture one step (on an empty plan) into a graph; replays run later plans."""
        dev = self.solver.device
        self.solver.plan([])
        s = torch.cuda.Stream(device=dev)
        s.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(s):
            self.solver.step()  # warm the launch path outside capture
        torch.cuda.current_stream(dev).wait_stream(s)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.solver.step()
        torch.cuda.synchronize(dev)


class BatchServer:
    """Continuous batching over two graph-replayed slots per tensor order."""

    def __init__(self, capacity=256, q=1, p=8, lclass=48, ws_bytes=8 << 30, shift="adaptive", device="cuda",
                 use_graphs=True, orders=(3,), overlap=True):
        """overlap=False runs every batch on the caller's current stream (one
        batch on the device at a time), e.g. to time each phase alone."""
        self.device = torch.device(device)
        self.overlap = overlap
        self.p, self.q, self.lclass, self.shift = p, q, lclass, shift
        self.capacity, self.ws_bytes = capacity, ws_bytes
        self.use_graphs = use_graphs
        self.slots: Dict[int, List[_Slot]] = {}
        for d in orders:
            self._slots_for(d)
        self.batch_sizes: List[int] = []  # requests per launched batch
        self.inflight: List[int] = []     # requests on the device right after each launch

    def _slots_for(self, d: int) -> List[_Slot]:
        if d not in self.slots:
            pair = [_Slot(self.capacity, d, self.q, self.p, self.lclass, self.ws_bytes, self.shift, self.device)
                    for _ in range(2)]
            if self.use_graphs:
                for s in pair:
                    s.capture()
            self.slots[d] = pair
        return self.slots[d]

    def budget(self, d: int) -> int:
        s = self._slots_for(d)[0].solver
        return s.ws.numel() - s.table_bytes

    def _launch(self, slot: _Slot, jobs: List[Job]):
        # the plan buffer is free: the slot's previous step has completed
        slot.solver.plan([j.item for j in jobs])
        stream = slot.stream if self.overlap else torch.cuda.current_stream(self.device)
        stream.wait_stream(torch.cuda.current_stream(self.device))  # inputs written on the caller's stream
        with torch.cuda.stream(stream):
            if self.use_graphs:
                slot.graph.replay()
            else:
                slot.solver.step()
            slot.event = torch.cuda.Event()
            slot.event.record()
        slot.jobs = jobs
        self.batch_sizes.append(len(jobs))

    def _admit(self, waiting: collections.deque, d: int) -> List[Job]:
        """FIFO among waiting requests of order d, while capacity and budget allow."""
        batch, used, keep = [], 0, collections.deque()
        budget = self.budget(d)
        while waiting and len(batch) < self.capacity:
            j = waiting.popleft()
            if j.A.dim() != d:
                keep.append(j)
                continue
            if j.ws_bytes > budget:
                raise ValueError("request %d needs %d workspace bytes, budget %d" % (j.rid, j.ws_bytes, budget))
            if used + j.ws_bytes > budget:
                keep.append(j)
                break
            batch.append(j)
            used += j.ws_bytes
        keep.extend(waiting)
        waiting.clear()
        waiting.extend(keep)
        return batch

    def run(self, jobs: Sequence[Job], t0: Optional[float] = None) -> List[Job]:
        """Serve prepared `jobs` (arrival seconds relative to t0); returns them with .done set.
        The results are complete on the device when run returns (every slot's
        completion event has been seen)."""
        for j in jobs:
            if j.item is None:
                j.prepare(self.p, self.q)
        for d in sorted({j.A.dim() for j in jobs}):
            self._slots_for(d)
        pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
        waiting: collections.deque = collections.deque()
        busy: List[_Slot] = []
        t0 = time.perf_counter() if t0 is None else t0
        while pending or waiting or busy:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            for s in list(busy):
                if s.event.query():
                    t = time.perf_counter() - t0
                    for j in s.jobs:
                        j.done = t
                    s.jobs = []
                    busy.remove(s)
            if waiting:
                d = waiting[0].A.dim()
                free = [s for s in self.slots[d] if not s.jobs]
                if free:
                    batch = self._admit(waiting, d)
                    self._launch(free[0], batch)
                    busy.append(free[0])
                    self.inflight.append(sum(len(s.jobs) for s in busy))
                    continue
            if pending and not waiting and not busy:
                time.sleep(min(200e-6, max(0.0, pending[0].arrival - now)))
            else:
                time.sleep(10e-6)
        return list(jobs)


class SingleServer:
    """One request at a time: tucker_rsthosvd per request, in arrival order."""

    def __init__(self, p=8, q=1, shift="adaptive", ws_bytes=256 << 20, device="cuda"):
        self.device = torch.device(device)
        self.p, self.q, self.shift = p, q, T._SHIFT[shift]
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)

    def _solve(self, j: Job, stream):
        it = j.item
        T._check(T.lib.tucker_rsthosvd(ctypes.byref(it.shape), it.A, it.ranks, self.p, self.q, self.shift,
                                       ctypes.c_uint64(it.seed), T.FP32, it.G, it.U, None,
                                       ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_size_t(self.ws.numel()),
                                       stream))

    def run(self, jobs: Sequence[Job], t0: Optional[float] = None) -> List[Job]:
        for j in jobs:
            if j.item is None:
                j.prepare(self.p, self.q)
        order = sorted(jobs, key=lambda j: j.arrival)
        stream = T._stream(self.device)
        t0 = time.perf_counter() if t0 is None else t0
        inflight = collections.deque()

        def retire():
            while inflight and inflight[0][1].query():
                jj, _ = inflight.popleft()
                jj.done = time.perf_counter() - t0

        for j in order:
            while time.perf_counter() - t0 < j.arrival:
                retire()
                time.sleep(10e-6)
            self._solve(j, stream)
            ev = torch.cuda.Event()
            ev.record()
            inflight.append((j, ev))
            retire()
        while inflight:
            jj, ev = inflight.popleft()
            ev.synchronize()
            jj.done = time.perf_counter() - t0
        return list(order)


def latency_stats(jobs: Sequence[Job]) -> dict:
    """p50 / p99 / max latency (arrival to completion seen), span and throughput."""
    lat = sorted(j.done - j.arrival for j in jobs)
    if not lat:
        return {}
    pick = lambda f: lat[min(len(lat) - 1, int(f * len(lat)))]
    span = max(j.done for j in jobs) - min(j.arrival for j in jobs)
    return {"count": len(lat), "p50_ms": 1e3 * pick(0.5), "p99_ms": 1e3 * pick(0.99), "max_ms": 1e3 * lat[-1],
            "span_s": span, "approx_per_s": len(lat) / span if span > 0 else float("inf")}
