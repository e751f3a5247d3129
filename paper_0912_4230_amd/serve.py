"""Serving loop: continuous batching of lattice Boltzmann solve requests on one GPU.

Requests (domain size, medium, physics, number of steps) arrive over time.
The scheduler admits them in arrival order while their workspaces fit in
an HBM budget, keeps every admitted lattice resident on the device, and
advances all active lattices together in ticks: one batched launch per
step for all lattices of the same physics and storage (lbm_step_batch), so
requests that arrive while others run join the next tick and their work
overlaps on the device.  A lattice that reaches its step count is retired
once its tick has completed (moments copied out, workspace freed), which
frees budget for the queue.  Latency = completion - arrival on the host clock.

The host keeps one tick queued ahead of the device: tick n+1 is issued
before the host waits for tick n, and new lattices are set up (and finished
ones read back) on a second stream while the ticks run, so the device does
not idle while the host admits or retires requests.

The scheduler talks to an executor (GpuExecutor here, a mock in the CPU
tests), so admission, budget and retirement logic run without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import json
import math
import time
from typing import Callable, Dict, List, Optional, TextIO

from . import inputs as I


@dataclasses.dataclass
class Job:
    req: I.Request
    handle: object
    nbytes: int
    remaining: int
    admitted: float


@dataclasses.dataclass
class Outcome:
    rid: int
    arrival: float
    admitted: float
    completed: float
    latency: float
    cells: int
    steps: int
    status: str             # "ok", "unstable", "rejected", "error: ..."
    result: object = None


class GpuExecutor:
    """Runs lattices through the C ABI.  The ticks of all active lattices run
    on one stream (the current stream of the device); set-up and read-back
    run on a second stream of default priority, so they overlap the ticks."""

    def __init__(self, storage="f32", device="cuda:0", keep_results=False, problems=None):
        import torch
        from . import binding as B
        self.B = B
        self.torch = torch
        self.storage = B.STORAGE_NAMES[storage] if isinstance(storage, str) else storage
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.side = torch.cuda.Stream(device=self.device)
        self.keep_results = keep_results
        self.problems = problems or {}
        self.busy_s = 0.0           # device time of the completed ticks

    def problem(self, req: I.Request):
        p = self.problems.get(req.rid)
        return p if p is not None else I.request_problem(req)

    def workspace_bytes(self, req: I.Request) -> int:
        from .sim import make_desc
        return self.B.lbm_workspace_bytes(make_desc(self.problem(req), self.storage))

    def admit(self, req: I.Request):
        """Set the lattice up on the side stream (lbm_set_medium synchronises
        that stream only), then hand it to the tick stream."""
        from .sim import Simulation
        sim = Simulation(self.problem(req), storage=self.storage, device=self.device, stream=self.side)
        return sim.set_stream(self.stream)

    def run_tick(self, handles, nsteps):
        """Issue one tick (asynchronous); returns its token."""
        from .sim import step_batch
        t0 = self.torch.cuda.Event(enable_timing=True)
        t1 = self.torch.cuda.Event(enable_timing=True)
        t0.record(self.stream)
        step_batch(handles, nsteps)
        t1.record(self.stream)
        return (t0, t1)

    def wait(self, token):
        """Block until the tick of `token` has completed on the device."""
        t0, t1 = token
        t1.synchronize()
        self.busy_s += t0.elapsed_time(t1) / 1e3

    def finish(self, sim):
        """Moments of the last step (its tick has completed); status 'ok' or
        'unstable'.  Read back on the side stream."""
        sim.set_stream(self.side)
        rho, vel, conc, diag = sim.moments(check=False)
        status = "ok" if diag[7] == 0 else "unstable"
        res = (rho, vel, conc, diag) if self.keep_results else diag
        return status, res

    def release(self, sim):
        sim.close()
        sim.ws = None

    def busy_seconds(self) -> float:
        return self.busy_s


def nearest_rank(values: List[float], p: float) -> float:
    """p-th percentile by nearest rank (with n samples, p99 of n <= 100 is the max)."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, math.ceil(p / 100.0 * len(v)))
    return v[k - 1]


def record(o: Outcome) -> Dict:
    """The JSON record of one request: times on the serving clock (s since the
    loop started), latency, size, status and the request's own rate while it
    was resident (cell updates / (completed - admitted), MLUPS; null when it
    never ran)."""
    resident = o.completed - o.admitted
    ran = o.status in ("ok", "unstable") and resident > 0
    return {"rid": o.rid, "arrival_s": round(o.arrival, 6), "admitted_s": round(o.admitted, 6),
            "completed_s": round(o.completed, 6), "latency_s": round(o.latency, 6), "cells": o.cells,
            "steps": o.steps, "status": o.status,
            "mlups_resident": round(o.cells * o.steps / resident / 1e6, 3) if ran else None}


def serve(requests: List[I.Request], executor, budget_bytes: int, tick_steps: int = 50,
          clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
          log: Optional[Callable[[str], None]] = None, jsonl: Optional[TextIO] = None) -> Dict:
    """Run the request stream to completion; returns per-request outcomes and
    aggregate statistics.  With `jsonl` (a text stream) every request's
    record() is written as one JSON line as soon as its outcome is known."""
    pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
    active: List[Job] = []
    used = 0
    outcomes: Dict[int, Outcome] = {}
    ticks = 0
    max_active = 0
    t0 = clock()

    def now():
        return clock() - t0

    def settle(o: Outcome):
        outcomes[o.rid] = o
        if jsonl is not None:
            jsonl.write(json.dumps(record(o)) + "\n")

    def admit_ready():
        nonlocal used
        while pending and pending[0].arrival <= now():
            req = pending[0]
            try:
                nb = executor.workspace_bytes(req)
            except Exception as e:  # invalid request description
                pending.popleft()
                settle(Outcome(req.rid, req.arrival, now(), now(), now() - req.arrival,
                               req.edge ** 3, req.steps, f"error: {e}"))
                continue
            if nb <= 0 or nb > budget_bytes:
                pending.popleft()
                settle(Outcome(req.rid, req.arrival, now(), now(), now() - req.arrival,
                               req.edge ** 3, req.steps, "rejected"))
                continue
            if used + nb > budget_bytes:
                break          # FIFO: wait for memory to free up
            pending.popleft()
            try:
                h = executor.admit(req)
            except Exception as e:
                settle(Outcome(req.rid, req.arrival, now(), now(), now() - req.arrival,
                               req.edge ** 3, req.steps, f"error: {e}"))
                continue
            used += nb
            active.append(Job(req, h, nb, req.steps, now()))

    def retire(jobs):
        nonlocal used
        for j in jobs:
            status, res = executor.finish(j.handle)
            t = now()
            settle(Outcome(j.req.rid, j.req.arrival, j.admitted, t, t - j.req.arrival,
                           j.req.edge ** 3, j.req.steps, status, res))
            executor.release(j.handle)
            used -= j.nbytes
            if log:
                log(f"serve: request {j.req.rid} ({j.req.edge}^3 x {j.req.steps}) done in {t - j.req.arrival:.2f} s")

    # the tick issued last and the lattices that finish with it
    inflight = None
    while pending or active or inflight is not None:
        admit_ready()
        token, finishing = None, []
        if active:
            nsteps = [min(tick_steps, j.remaining) for j in active]
            token = executor.run_tick([j.handle for j in active], nsteps)
            ticks += 1
            max_active = max(max_active, len(active))
            still = []
            for j, n in zip(active, nsteps):
                j.remaining -= n
                (still if j.remaining > 0 else finishing).append(j)
            active = still
        # the device runs the tick just issued while the host waits for the
        # previous one and retires what finished with it
        if inflight is not None:
            executor.wait(inflight[0])
            retire(inflight[1])
            inflight = None
        if token is not None:
            inflight = (token, finishing)
        elif pending:
            wait = pending[0].arrival - now()
            if wait > 0:
                sleep(wait)

    done = [o for o in outcomes.values() if o.status in ("ok", "unstable")]
    lat = [o.latency for o in done]
    lups = sum(o.cells * o.steps for o in done)
    span = (max(o.completed for o in done) - min(o.arrival for o in done)) if done else float("nan")
    busy = executor.busy_seconds() if hasattr(executor, "busy_seconds") else float("nan")
    return {
        "outcomes": outcomes,
        "busy_s": busy,
        "busy_fraction": busy / span if done and span > 0 else float("nan"),
        "p50_s": nearest_rank(lat, 50),
        "p99_s": nearest_rank(lat, 99),
        "mean_s": sum(lat) / len(lat) if lat else float("nan"),
        "aggregate_mlups": lups / span / 1e6 if done else float("nan"),
        "completed": len(done),
        "failed": len(outcomes) - len(done),
        "ticks": ticks,
        "max_active": max_active,
        "span_s": span,
    }
