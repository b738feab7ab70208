"""Serving loop: continuous batching of TT transport solves on one GPU.

Requests (a problem and a step count) arrive over time.  The loop admits
them in arrival order while their device workspace fits a memory budget and
a slot is free (`tt_transport_workspace_bytes` gives the bytes from the rank
caps), keeps every admitted request's cores on the device until it has run
all its steps, and frees its memory when it completes.  Admitted requests
advance together: each loop iteration enqueues a chunk of steps for every
request that has fewer than two chunks in flight, each request on its own
stream, so the kernels of different requests overlap on the device while new
requests join as others leave.  Completion is observed through HIP events;
latency is completion time minus arrival time, both on the GPU's clock
relative to a start event.

The scheduling decisions (`Admission`) are plain host logic and are tested
without a GPU; `Server` runs them against the library.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    prob: object
    arrival: float          # seconds after the start of the run
    steps: int
    nbytes: int = 0         # device workspace the request needs


class Admission:
    """First-come first-served admission by memory and slots.  The head of the
    queue is admitted once it has arrived, its workspace fits the free part of
    the budget and fewer than `max_active` requests are running; requests
    behind it never overtake it (no starvation of large requests)."""

    def __init__(self, budget_bytes: int, max_active: int):
        if budget_bytes <= 0 or max_active <= 0:
            raise ValueError("budget and slots must be positive")
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.in_use = 0
        self.active = 0

    def check(self, req: Request):
        if req.nbytes > self.budget:
            raise ValueError(f"request {req.rid} needs {req.nbytes} bytes, above the whole budget {self.budget}")

    def take(self, queue: "collections.deque[Request]", now: float) -> List[Request]:
        out = []
        while queue and queue[0].arrival <= now and self.active < self.max_active \
                and self.in_use + queue[0].nbytes <= self.budget:
            r = queue.popleft()
            self.in_use += r.nbytes
            self.active += 1
            out.append(r)
        return out

    def release(self, req: Request):
        self.in_use -= req.nbytes
        self.active -= 1
        assert self.in_use >= 0 and self.active >= 0


@dataclasses.dataclass
class _Slot:
    req: Request
    solver: object
    stream: object
    done: int = 0
    inflight: "collections.deque" = dataclasses.field(default_factory=collections.deque)
    final: object = None


class Server:
    """Runs requests through the library with continuous batching (see the
    module docstring).  `n_streams` streams are shared round robin by the
    running requests; `chunk` steps are enqueued per request per iteration."""

    def __init__(self, device="cuda:0", budget_bytes: int = 64 << 30, max_active: int = 32, n_streams: int = 16,
                 chunk: int = 4, keep_results: bool = False):
        import torch

        from . import Solver, workspace_bytes  # noqa: F401  (binding loads the library)

        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, n_streams))]
        self.chunk = max(1, int(chunk))
        self.keep_results = keep_results
        self.results: Dict[int, tuple] = {}

    def run(self, reqs: Sequence[Request], on_complete: Optional[Callable] = None) -> dict:
        from . import Solver, step_batch, workspace_bytes

        torch = self.torch
        adm = Admission(self.budget, self.max_active)
        for r in reqs:
            if not r.nbytes:
                r.nbytes = workspace_bytes(r.prob) + 256
            adm.check(r)
        queue = collections.deque(sorted(reqs, key=lambda r: (r.arrival, r.rid)))
        active: List[_Slot] = []
        lat: Dict[int, float] = {}
        finish: Dict[int, float] = {}
        start = torch.cuda.Event(enable_timing=True)
        start.record(torch.cuda.current_stream(self.device))
        t0 = time.perf_counter()
        rr = 0
        max_active_seen = 0
        peak_bytes = 0
        while queue or active:
            now = time.perf_counter() - t0
            for r in adm.take(queue, now):
                st = self.streams[rr % len(self.streams)]
                rr += 1
                sv = Solver(r.prob, device=self.device, stream=st)
                active.append(_Slot(r, sv, st))
            max_active_seen = max(max_active_seen, len(active))
            peak_bytes = max(peak_bytes, adm.in_use)
            # retire completed chunks; enqueue the next chunk where fewer than two are in flight
            ready = []
            for sl in active:
                while sl.inflight and sl.inflight[0].query():
                    sl.inflight.popleft()
                if sl.done < sl.req.steps and len(sl.inflight) < 2:
                    ready.append(sl)
            if ready:
                n = min(min(sl.req.steps - sl.done for sl in ready), self.chunk)
                for _ in range(n):
                    step_batch([sl.solver for sl in ready], [sl.stream for sl in ready])
                for sl in ready:
                    sl.done += n
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(sl.stream)
                    sl.inflight.append(ev)
                    if sl.done == sl.req.steps:
                        sl.final = ev
            # completed requests leave and free their memory
            still = []
            for sl in active:
                if sl.final is not None and sl.final.query():
                    t_done = start.elapsed_time(sl.final) * 1e-3
                    finish[sl.req.rid] = t_done
                    lat[sl.req.rid] = t_done - sl.req.arrival
                    if self.keep_results:
                        self.results[sl.req.rid] = sl.solver.get_cores()
                    if on_complete:
                        on_complete(sl)
                    sl.solver.destroy()
                    adm.release(sl.req)
                else:
                    still.append(sl)
            active = still
            if not active and queue:
                # idle until the next arrival
                time.sleep(max(0.0, min(queue[0].arrival - (time.perf_counter() - t0), 0.01)))
            elif not ready:
                time.sleep(2e-5)
        torch.cuda.synchronize(self.device)
        lats = np.array([lat[r.rid] for r in reqs]) * 1e3
        makespan = max(finish.values()) - min(r.arrival for r in reqs)
        return {
            "requests": len(reqs),
            "p50_ms": float(np.percentile(lats, 50)),
            "p99_ms": float(np.percentile(lats, 99)),
            "mean_ms": float(lats.mean()),
            "throughput_rps": len(reqs) / makespan if makespan > 0 else float("inf"),
            "makespan_s": makespan,
            "max_active": max_active_seen,
            "peak_workspace_bytes": peak_bytes,
            "budget_bytes": self.budget,
            "latency_ms": {r.rid: float(lat[r.rid] * 1e3) for r in reqs},
        }


def make_requests(problems, arrivals=None, steps: Optional[int] = None) -> List[Request]:
    """Requests from problems (tt_inputs.Problem) with arrival times (seconds;
    default all at 0) and step counts (default each problem's n_steps)."""
    out = []
    for i, p in enumerate(problems):
        a = 0.0 if arrivals is None else float(arrivals[i])
        out.append(Request(rid=i, prob=p, arrival=a, steps=int(steps if steps is not None else p.n_steps)))
    return out
