"""Serving scheduler on the CPU with a mock executor: admission in arrival
order under the HBM budget, continuous batching across ticks, retirement,
rejection of oversized requests and isolation of a failing request."""
import pytest

from paper_0912_4230_amd import inputs as I
from paper_0912_4230_amd.serve import nearest_rank, serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class MockExecutor:
    """Fake lattices: bytes = 100 per cell, cost = cells * steps / rate seconds
    of a fake device that runs the issued ticks one after the other while the
    host goes on (run_tick returns the time the tick completes, wait advances
    the host clock to it)."""

    def __init__(self, clock, rate=1e9, unstable=()):
        self.clock = clock
        self.rate = rate
        self.unstable = set(unstable)
        self.used = 0
        self.peak = 0
        self.batches = []
        self.free_at = 0.0
        self.busy = 0.0

    def workspace_bytes(self, req):
        return 100 * req.edge ** 3

    def admit(self, req):
        self.used += self.workspace_bytes(req)
        self.peak = max(self.peak, self.used)
        return {"req": req}

    def run_tick(self, handles, nsteps):
        self.batches.append([h["req"].rid for h in handles])
        cost = sum(h["req"].edge ** 3 * n for h, n in zip(handles, nsteps)) / self.rate
        start = max(self.clock.t, self.free_at)
        self.free_at = start + cost
        self.busy += cost
        return self.free_at

    def wait(self, token):
        self.clock.t = max(self.clock.t, token)

    def busy_seconds(self):
        return self.busy

    def finish(self, h):
        return ("unstable" if h["req"].rid in self.unstable else "ok"), None

    def release(self, h):
        self.used -= self.workspace_bytes(h["req"])


def _reqs(n=20, seed=1):
    return I.request_stream(n=n, rate=4.0, edge_lo=16, edge_hi=64, steps_lo=50, steps_hi=400,
                            arrival_seed=seed, param_seed=seed + 1)


def test_all_complete_and_budget_respected():
    clk = Clock()
    ex = MockExecutor(clk, rate=2e7)
    reqs = _reqs()
    budget = 100 * 64 ** 3 * 3
    st = serve(reqs, ex, budget, tick_steps=25, clock=clk, sleep=clk.sleep)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert ex.peak <= budget
    assert ex.used == 0
    for r in reqs:
        o = st["outcomes"][r.rid]
        assert o.admitted >= r.arrival - 1e-12
        assert o.completed >= o.admitted
        assert o.latency >= r.edge ** 3 * r.steps / ex.rate * (1 - 1e-9)


def test_continuous_batching_joins_running_ticks():
    clk = Clock()
    ex = MockExecutor(clk, rate=5e6)
    reqs = _reqs()
    st = serve(reqs, ex, 1 << 60, tick_steps=20, clock=clk, sleep=clk.sleep)
    # some tick runs several requests at once, and the set of requests changes
    # between consecutive ticks while earlier ones are still running
    assert max(len(b) for b in ex.batches) >= 3
    joined = any(set(a) < set(b) or (set(a) & set(b) and set(b) - set(a))
                 for a, b in zip(ex.batches, ex.batches[1:]))
    assert joined
    assert st["max_active"] >= 3


def test_fifo_admission_under_tight_budget():
    clk = Clock()
    ex = MockExecutor(clk, rate=1e7)
    reqs = _reqs(12)
    budget = max(100 * r.edge ** 3 for r in reqs)      # one of the largest at a time
    st = serve(reqs, ex, budget, tick_steps=50, clock=clk, sleep=clk.sleep)
    order = sorted(reqs, key=lambda r: r.arrival)
    adm = [st["outcomes"][r.rid].admitted for r in order]
    assert adm == sorted(adm)
    assert ex.peak <= budget


def test_oversized_request_rejected_others_served():
    clk = Clock()
    ex = MockExecutor(clk, rate=1e8)
    reqs = _reqs(8)
    big = max(reqs, key=lambda r: r.edge)
    budget = 100 * big.edge ** 3 - 1
    st = serve(reqs, ex, budget, tick_steps=50, clock=clk, sleep=clk.sleep)
    assert st["outcomes"][big.rid].status == "rejected"
    assert all(st["outcomes"][r.rid].status == "ok" for r in reqs if r.edge ** 3 * 100 <= budget)


def test_unstable_request_is_isolated():
    clk = Clock()
    reqs = _reqs(10)
    ex = MockExecutor(clk, rate=1e8, unstable={reqs[3].rid})
    st = serve(reqs, ex, 1 << 60, tick_steps=50, clock=clk, sleep=clk.sleep)
    assert st["outcomes"][reqs[3].rid].status == "unstable"
    assert sum(o.status == "ok" for o in st["outcomes"].values()) == len(reqs) - 1


def test_next_tick_issued_before_waiting():
    """The host issues tick n+1 before it waits for tick n: while requests keep
    the device busy it never idles between ticks, and the busy fraction is the
    device time over the span."""
    clk = Clock()
    ex = MockExecutor(clk, rate=1e7)
    waits = []
    wait0 = ex.wait

    def wait(token):
        # at every wait, a later tick is already issued (unless the stream drained)
        waits.append((token, ex.free_at))
        wait0(token)
    ex.wait = wait
    reqs = _reqs(16)
    st = serve(reqs, ex, 1 << 60, tick_steps=25, clock=clk, sleep=clk.sleep)
    assert st["completed"] == len(reqs)
    # a wait without a later tick issued happens only where the active set
    # drains (the device then has nothing to run anyway)
    ahead = sum(1 for tok, free in waits if free > tok)
    assert ahead > len(waits) // 2
    assert 0.0 < st["busy_fraction"] <= 1.0 + 1e-12
    assert abs(st["busy_s"] - ex.busy) < 1e-12


def test_jsonl_records_every_request():
    """One JSON line per request as its outcome is known: the statuses and
    times of the returned outcomes, latency = completion - arrival, and a
    resident rate for the requests that ran."""
    import io
    import json
    clk = Clock()
    reqs = _reqs(12)
    big = max(reqs, key=lambda r: r.edge)
    ex = MockExecutor(clk, rate=1e8, unstable={reqs[2].rid})
    out = io.StringIO()
    st = serve(reqs, ex, 100 * big.edge ** 3 - 1, tick_steps=50, clock=clk, sleep=clk.sleep, jsonl=out)
    lines = [json.loads(x) for x in out.getvalue().splitlines()]
    assert sorted(r["rid"] for r in lines) == sorted(r.rid for r in reqs)
    for r in lines:
        o = st["outcomes"][r["rid"]]
        assert r["status"] == o.status
        assert abs(r["latency_s"] - (r["completed_s"] - r["arrival_s"])) < 1e-5
        assert r["admitted_s"] >= r["arrival_s"] - 1e-9 and r["completed_s"] >= r["admitted_s"]
        if o.status in ("ok", "unstable"):
            assert r["mlups_resident"] > 0
            assert abs(r["mlups_resident"] - o.cells * o.steps / (o.completed - o.admitted) / 1e6) < 1e-3
        else:
            assert r["mlups_resident"] is None
    assert {r["status"] for r in lines} >= {"ok", "unstable", "rejected"}
    # records appear in completion order
    done = [r["completed_s"] for r in lines]
    assert done == sorted(done)


def test_nearest_rank():
    v = list(range(1, 65))
    assert nearest_rank(v, 50) == 32
    assert nearest_rank(v, 99) == 64
    assert nearest_rank([5.0], 99) == 5.0
    with pytest.raises(Exception):
        nearest_rank(None, 50)
