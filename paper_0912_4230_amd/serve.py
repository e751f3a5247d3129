"""Serving loop: continuous batching of lattice Boltzmann solve requests on one GPU.

Requests (domain size, medium, physics, number of steps) arrive over time.
The scheduler admits them in arrival order while their workspaces fit in
an HBM budget, keeps every admitted lattice resident on the device, and
advances all active lattices together in ticks: one batched launch per
step for all lattices of the same physics and storage (lbm_step_batch), so
requests that arrive while others run join the next tick and their work
overlaps on the device.  A lattice that reaches its step count is retired
at the end of its tick (moments copied out, workspace freed), which frees
budget for the queue.  Latency = completion - arrival on the host clock.

The scheduler talks to an executor (GpuExecutor here, a mock in the CPU
tests), so admission, budget and retirement logic run without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional

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
    """Runs lattices through the C ABI; all lattices share one stream."""

    def __init__(self, storage="f32", device="cuda:0", keep_results=False, problems=None):
        import torch
        from . import binding as B
        self.B = B
        self.torch = torch
        self.storage = B.STORAGE_NAMES[storage] if isinstance(storage, str) else storage
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.keep_results = keep_results
        self.problems = problems or {}

    def problem(self, req: I.Request):
        p = self.problems.get(req.rid)
        return p if p is not None else I.request_problem(req)

    def workspace_bytes(self, req: I.Request) -> int:
        from .sim import make_desc
        return self.B.lbm_workspace_bytes(make_desc(self.problem(req), self.storage))

    def admit(self, req: I.Request):
        from .sim import Simulation
        return Simulation(self.problem(req), storage=self.storage, device=self.device, stream=self.stream)

    def run_tick(self, handles, nsteps):
        from .sim import step_batch
        step_batch(handles, nsteps)

    def sync(self):
        self.torch.cuda.synchronize(self.device)

    def finish(self, sim):
        """Moments of the last step; status 'ok' or 'unstable'."""
        rho, vel, conc, diag = sim.moments(check=False)
        status = "ok" if diag[7] == 0 else "unstable"
        res = (rho, vel, conc, diag) if self.keep_results else diag
        return status, res

    def release(self, sim):
        sim.close()
        sim.ws = None


def nearest_rank(values: List[float], p: float) -> float:
    """p-th percentile by nearest rank (with n samples, p99 of n <= 100 is the max)."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, math.ceil(p / 100.0 * len(v)))
    return v[k - 1]


def serve(requests: List[I.Request], executor, budget_bytes: int, tick_steps: int = 50,
          clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
          log: Optional[Callable[[str], None]] = None) -> Dict:
    """Run the request stream to completion; returns per-request outcomes and
    aggregate statistics."""
    pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
    active: List[Job] = []
    used = 0
    outcomes: Dict[int, Outcome] = {}
    ticks = 0
    max_active = 0
    t0 = clock()

    def now():
        return clock() - t0

    def admit_ready():
        nonlocal used
        while pending and pending[0].arrival <= now():
            req = pending[0]
            try:
                nb = executor.workspace_bytes(req)
            except Exception as e:  # invalid request description
                pending.popleft()
                outcomes[req.rid] = Outcome(req.rid, req.arrival, now(), now(), now() - req.arrival,
                                            req.edge ** 3, req.steps, f"error: {e}")
                continue
            if nb <= 0 or nb > budget_bytes:
                pending.popleft()
                outcomes[req.rid] = Outcome(req.rid, req.arrival, now(), now(), now() - req.arrival,
                                            req.edge ** 3, req.steps, "rejected")
                continue
            if used + nb > budget_bytes:
                break          # FIFO: wait for memory to free up
            pending.popleft()
            try:
                h = executor.admit(req)
            except Exception as e:
                outcomes[req.rid] = Outcome(req.rid, req.arrival, now(), now(), now() - req.arrival,
                                            req.edge ** 3, req.steps, f"error: {e}")
                continue
            used += nb
            active.append(Job(req, h, nb, req.steps, now()))

    while pending or active:
        admit_ready()
        if not active:
            if pending:
                wait = pending[0].arrival - now()
                if wait > 0:
                    sleep(wait)
            continue
        nsteps = [min(tick_steps, j.remaining) for j in active]
        executor.run_tick([j.handle for j in active], nsteps)
        executor.sync()
        ticks += 1
        max_active = max(max_active, len(active))
        still = []
        for j, n in zip(active, nsteps):
            j.remaining -= n
            if j.remaining > 0:
                still.append(j)
                continue
            status, res = executor.finish(j.handle)
            t = now()
            outcomes[j.req.rid] = Outcome(j.req.rid, j.req.arrival, j.admitted, t, t - j.req.arrival,
                                          j.req.edge ** 3, j.req.steps, status, res)
            executor.release(j.handle)
            used -= j.nbytes
            if log:
                log(f"serve: request {j.req.rid} ({j.req.edge}^3 x {j.req.steps}) done in {t - j.req.arrival:.2f} s")
        active = still

    done = [o for o in outcomes.values() if o.status in ("ok", "unstable")]
    lat = [o.latency for o in done]
    lups = sum(o.cells * o.steps for o in done)
    span = (max(o.completed for o in done) - min(o.arrival for o in done)) if done else float("nan")
    return {
        "outcomes": outcomes,
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
