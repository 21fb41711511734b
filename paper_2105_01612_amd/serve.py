"""Continuous-batching request loop for equilibrium projections on one GPU.

Requests (one stress field each, any supported grid size) arrive over time.  The
server keeps *slots* per size class: a slot is a libeq plan with a captured
hipGraph, plus device input/output buffers.  A request is admitted as soon as a
slot of its class is free, or a new slot fits the HBM budget (eq_plan_footprint +
buffers), evicting idle slots of other classes if needed.  Admitted work runs
asynchronously on its slot's stream; the backend keeps a small pool of streams (as
many as the device has hardware queues) and gives each size class the stream of
its rank among the sizes, so a small request never waits in a stream behind a large
one, while requests on different streams overlap on the device.  Completions are
found by polling events, and every completion frees a slot for the next waiting
request (no head-of-line blocking across classes).  By default the smallest waiting
field is admitted first and at most eight requests run at once.  Inputs are taken from pools,
device-resident as if produced by an upstream GPU stage, or in pinned host memory (the copy into the
slot is then the request's transfer over PCIe); the copy into the slot is part of the request's
service.

The executor is a backend object, so the admission and bookkeeping logic also runs
on the CPU against a fake backend in the tests.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional

import numpy as np

__all__ = ["Request", "Server", "GpuBackend", "latency_summary"]


@dataclasses.dataclass
class Request:
    rid: int
    n: int                  # grid edge (n^3 field)
    arrival: float          # seconds after the run starts
    field: int = 0          # index into the size class's input pool
    admitted: float = math.nan
    done: float = math.nan

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Slot:
    def __init__(self, n: int, nbytes: int, handle):
        self.n = n
        self.nbytes = nbytes
        self.handle = handle        # backend object
        self.req: Optional[Request] = None
        self.last_used = 0.0


def stream_of_size(n: int, sizes, streams: int) -> int:
    """Stream index of size class n: its rank among `sizes`, scaled onto `streams` streams
    (smallest sizes on stream 0, the largest alone on the last one when there are enough)."""
    order = sorted(set(int(x) for x in sizes))
    if n not in order:
        order = sorted(set(order) | {int(n)})
    return min(streams - 1, order.index(int(n)) * streams // len(order))


class GpuBackend:
    """libeq executor: one plan (graph capture) and two buffers per slot; slots share a pool of
    `streams` streams by size class (see stream_of_size)."""

    def __init__(self, pools: Dict[int, "object"], prec: str = "fp32", op: str = "ddo", h: float = 1.0,
                 streams: int = 4, tune_cache: Optional[str] = None, graphs: bool = True):
        import torch

        import paper_2105_01612_amd as eq

        self.torch, self.eq = torch, eq
        self.tune_cache = tune_cache  # autotune results file: a slot's plan takes its class's entry
        self.graphs = graphs          # replay a captured hipGraph per slot, else launch the passes
        self.pools = pools            # n -> device tensor (k, 6, n, n, n)
        self.prec, self.op, self.h = prec, op, h
        self.dtype = torch.float32 if prec == "fp32" else torch.float64
        self.streams = [torch.cuda.Stream() for _ in range(max(1, int(streams)))]
        self.sizes = sorted(int(n) for n in pools)

    def slot_bytes(self, n: int) -> int:
        field = 6 * n ** 3 * (4 if self.prec == "fp32" else 8)
        return self.eq.footprint(n, n, n, 1, self.op, self.prec, self.h) + 2 * field

    def create(self, n: int):
        torch = self.torch
        stream = self.streams[stream_of_size(n, self.sizes, len(self.streams))]
        plan = self.eq.plan(n, op=self.op, prec=self.prec, h=self.h, flags=["capture_graph"] if self.graphs else [],
                            stream=stream)
        if self.tune_cache:
            from .autotune import apply_cached

            apply_cached(plan, self.tune_cache)
        with torch.cuda.stream(stream):
            inp = torch.empty((6, n, n, n), dtype=self.dtype, device="cuda")
            out = torch.empty_like(inp)
        return {"plan": plan, "stream": stream, "inp": inp, "out": out, "ev": torch.cuda.Event()}

    def submit(self, h, req: Request) -> None:
        torch = self.torch
        with torch.cuda.stream(h["stream"]):
            h["inp"].copy_(self.pools[req.n][req.field], non_blocking=True)
            h["plan"].project(h["inp"], h["out"])
            h["ev"].record(h["stream"])

    def done(self, h) -> bool:
        return h["ev"].query()

    def result(self, h):
        return h["out"]

    def destroy(self, h) -> None:
        h["stream"].synchronize()
        h["plan"].destroy()
        del h["inp"], h["out"]
        # return the slot's buffers to the device, so that the budget's count of the HBM in use
        # matches what the next plan allocation finds free
        self.torch.cuda.empty_cache()


class Server:
    """max_inflight caps the requests running at once (None: as many as slots allow); with a
    cap, requests queue on the host, which bounds how long a small request shares the GPU with
    large ones.  order: "fifo" admits in arrival order, "sjf" (the default) admits the smallest
    waiting field first."""

    def __init__(self, backend, budget_bytes: int, max_slots_per_class: int = 8,
                 max_inflight: Optional[int] = 8, order: str = "sjf"):
        if order not in ("fifo", "sjf"):
            raise ValueError("order must be 'fifo' or 'sjf'")
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_slots = max_slots_per_class
        self.max_inflight = max_inflight
        self.order = order
        self.slots: Dict[int, List[Slot]] = collections.defaultdict(list)
        self.used = 0
        self.peak_used = 0
        self._slot_bytes: Dict[int, int] = {}

    # -- slots -------------------------------------------------------------
    def _bytes(self, n: int) -> int:
        if n not in self._slot_bytes:
            self._slot_bytes[n] = self.backend.slot_bytes(n)
        return self._slot_bytes[n]

    def _free_slot(self, n: int) -> Optional[Slot]:
        for s in self.slots[n]:
            if s.req is None:
                return s
        return None

    def _evict_idle(self, need: int, keep: int) -> bool:
        """Destroy idle slots of other classes (least recently used first) until `need` fits."""
        idle = sorted((s for n, ss in self.slots.items() if n != keep for s in ss if s.req is None),
                      key=lambda s: s.last_used)
        for s in idle:
            if self.used + need <= self.budget:
                break
            self.backend.destroy(s.handle)
            self.slots[s.n].remove(s)
            self.used -= s.nbytes
        return self.used + need <= self.budget

    def _acquire(self, n: int) -> Optional[Slot]:
        s = self._free_slot(n)
        if s is not None:
            return s
        if len(self.slots[n]) >= self.max_slots:
            return None
        need = self._bytes(n)
        if need > self.budget:
            raise ValueError(f"a {n}^3 slot needs {need} B, more than the budget {self.budget} B")
        if self.used + need > self.budget and not self._evict_idle(need, n):
            return None
        s = Slot(n, need, self.backend.create(n))
        self.slots[n].append(s)
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        return s

    def warm(self, sizes) -> None:
        """Create one slot per size and run it once (plans, tables and graphs exist before timing)."""
        for i, n in enumerate(sizes):
            s = self._acquire(n)
            if s is None:
                continue
            r = Request(-1 - i, n, 0.0, 0)
            self.backend.submit(s.handle, r)
            while not self.backend.done(s.handle):
                pass

    def close(self) -> None:
        for ss in self.slots.values():
            for s in ss:
                self.backend.destroy(s.handle)
        self.slots.clear()
        self.used = 0

    # -- the loop ------------------------------------------------------------
    def run(self, requests: List[Request], clock: Callable[[], float] = time.perf_counter,
            on_complete: Optional[Callable[[Request, object], None]] = None) -> dict:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: List[Request] = []
        busy: List[Slot] = []
        finished: List[Request] = []
        t0 = clock()
        while pending or queue or busy:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            # completions free slots first
            for s in list(busy):
                if self.backend.done(s.handle):
                    r = s.req
                    r.done = clock() - t0
                    if on_complete is not None:
                        on_complete(r, self.backend.result(s.handle))
                    s.req = None
                    s.last_used = r.done
                    busy.remove(s)
                    finished.append(r)
                    progressed = True
            # admissions (arrival order, or smallest first); a request that cannot be placed does not
            # block other classes
            blocked = set()
            waiting = sorted(queue, key=lambda q: (q.n, q.arrival, q.rid)) if self.order == "sjf" else list(queue)
            for r in waiting:
                if self.max_inflight is not None and len(busy) >= self.max_inflight:
                    break
                if r.n in blocked:
                    continue
                s = self._acquire(r.n)
                if s is None:
                    blocked.add(r.n)
                    continue
                r.admitted = clock() - t0
                s.req = r
                self.backend.submit(s.handle, r)
                busy.append(s)
                queue.remove(r)
                progressed = True
            if not progressed and not busy and queue and not pending:
                raise RuntimeError("requests cannot be admitted: no slot fits the budget")
        return summarize(finished, self)


def latency_summary(lat_s: List[float]) -> dict:
    a = np.asarray(lat_s) * 1e3
    return {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean()), "max_ms": float(a.max())}


def summarize(finished: List[Request], server: Server) -> dict:
    if not finished:
        return {"completed": 0}
    first = min(r.arrival for r in finished)
    last = max(r.done for r in finished)
    vox = sum(r.n ** 3 for r in finished)
    out = {"completed": len(finished), "span_s": last - first,
           "requests_per_s": len(finished) / (last - first) if last > first else float("inf"),
           "voxels_per_s": vox / (last - first) if last > first else float("inf"),
           "peak_bytes": server.peak_used, "budget_bytes": server.budget,
           "queue_wait_p99_ms": float(np.percentile([(r.admitted - r.arrival) * 1e3 for r in finished], 99))}
    out.update(latency_summary([r.latency for r in finished]))
    per = collections.defaultdict(list)
    for r in finished:
        per[r.n].append(r.latency)
    out["per_size"] = {str(n): latency_summary(v) for n, v in sorted(per.items())}
    return out
