"""Serving loop: continuous batching of small shifted randomized ST-HOSVDs.

Requests (an FP32 tensor resident on the device, its Tucker ranks and seed)
arrive over time. The loop admits waiting requests into the next batch while
the batch fits the capacity and the workspace budget, writes the batch plan
(host only) and replays a graph captured once per slot: the library's
persistent batched kernels run every phase of Algorithm 3 for all requests of
the batch in one launch each. Requests of different orders go to different
slot pairs (a plan holds one order), and so, with lclass="auto", do requests
of different width classes: a request goes to the smallest class (16, 32, 48,
64) that holds its sketch widths, since the batched kernels' tiles, registers
and small SVDs are sized by the class. Each slot has its own stream and
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
    key: tuple = ()   # (order, width class) of the slots that serve it

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
    """Continuous batching over two graph-replayed slots per (order, width class)."""

    CLASSES = (16, 32, 48, 64)

    def __init__(self, capacity=256, q=1, p=8, lclass=48, ws_bytes=8 << 30, shift="adaptive", device="cuda",
                 use_graphs=True, orders=(), overlap=True, spill=False, max_inflight=2, poll_s=10e-6):
        """lclass: the width class of every slot, or "auto" (each request to the
        smallest class that holds its sketch widths; with spill, a batch whose
        own class has no free slot may run in a free slot of a wider class).
        max_inflight bounds the batches on the device at once, over all slots.
        overlap=False runs every batch on the caller's current stream (one
        batch on the device at a time), e.g. to time each phase alone. Slot
        pairs are made for `orders` now (with the widest class for "auto"),
        for the keys of a job list by ensure_slots(), and for other keys when
        run() first sees them."""
        self.device = torch.device(device)
        self.overlap = overlap
        self.p, self.q, self.shift = p, q, shift
        self.classes = self.CLASSES if lclass == "auto" else (int(lclass),)
        self.capacity, self.ws_bytes = capacity, ws_bytes
        self.use_graphs = use_graphs
        self.spill = spill
        self.max_inflight = max_inflight
        self.poll_s = poll_s  # sleep between polls while batches run (0: spin)
        self.slots: Dict[tuple, List[_Slot]] = {}
        for d in orders:
            self._slots_for((d, self.classes[-1]))
        self.batch_sizes: List[int] = []  # requests per launched batch
        self.inflight: List[int] = []     # requests on the device right after each launch

    def key_of(self, j: Job) -> tuple:
        """(order, smallest class >= every sketch width min(r_k + p, n_k) of the request)."""
        if not j.key:
            need = max(min(r + self.p, n) for r, n in zip(j.ranks, j.A.shape))
            fit = [c for c in self.classes if need <= c]
            if not fit:
                raise ValueError("request %d: sketch width %d exceeds the classes %s" % (j.rid, need, self.classes))
            j.key = (j.A.dim(), fit[0])
        return j.key

    def ensure_slots(self, jobs: Sequence[Job]) -> None:
        """Make (and capture) the slot pairs every key of `jobs` needs, e.g. before a timed run."""
        for j in jobs:
            self._slots_for(self.key_of(j))

    def _slots_for(self, key: tuple) -> List[_Slot]:
        if key not in self.slots:
            d, lclass = key
            pair = [_Slot(self.capacity, d, self.q, self.p, lclass, self.ws_bytes, self.shift, self.device)
                    for _ in range(2)]
            if self.use_graphs:
                for s in pair:
                    s.capture()
            self.slots[key] = pair
        return self.slots[key]

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

    def _admit(self, queue: collections.deque, slot: _Slot) -> List[Job]:
        """FIFO from one key's queue while capacity and the slot's budget allow."""
        batch, used = [], 0
        budget = slot.solver.ws.numel() - slot.solver.table_bytes
        while queue and len(batch) < self.capacity:
            j = queue[0]
            if j.ws_bytes > budget:
                raise ValueError("request %d needs %d workspace bytes, budget %d" % (j.rid, j.ws_bytes, budget))
            if used + j.ws_bytes > budget:
                break
            batch.append(queue.popleft())
            used += j.ws_bytes
        return batch

    def run(self, jobs: Sequence[Job], t0: Optional[float] = None) -> List[Job]:
        """Serve prepared `jobs` (arrival seconds relative to t0); returns them with .done set.
        The results are complete on the device when run returns (every slot's
        completion event has been seen). Waiting requests queue per (order,
        class) key. The key whose oldest waiting request arrived first launches
        next, in a free slot of its own class, else (spill) of the narrowest
        wider class of its order that has one."""
        for j in jobs:
            if j.item is None:
                j.prepare(self.p, self.q)
            j.key = ()
            self.key_of(j)
        keys = sorted({j.key for j in jobs})
        for key in keys:
            self._slots_for(key)
        pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
        waiting: Dict[tuple, collections.deque] = {k: collections.deque() for k in keys}
        busy: List[_Slot] = []
        t0 = time.perf_counter() if t0 is None else t0
        nwait = 0
        while pending or nwait or busy:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                j = pending.popleft()
                waiting[j.key].append(j)
                nwait += 1
            for s in list(busy):
                if s.event.query():
                    t = time.perf_counter() - t0
                    for j in s.jobs:
                        j.done = t
                    s.jobs = []
                    busy.remove(s)
            slot, key = None, None
            for k in [] if len(busy) >= self.max_inflight else sorted((k for k in keys if waiting[k]), key=lambda k: waiting[k][0].arrival):
                homes = [k2 for k2 in sorted(self.slots) if k2 == k or
                         (self.spill and k2[0] == k[0] and k2[1] > k[1])]
                slot = next((s for k2 in homes for s in self.slots[k2] if not s.jobs), None)
                if slot is not None:
                    key = k
                    break
            if slot is not None:
                batch = self._admit(waiting[key], slot)
                nwait -= len(batch)
                self._launch(slot, batch)
                busy.append(slot)
                self.inflight.append(sum(len(s.jobs) for s in busy))
                continue
            if pending and not nwait and not busy:
                time.sleep(min(200e-6, max(0.0, pending[0].arrival - now)))
            elif self.poll_s > 0:
                time.sleep(self.poll_s)
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
