"""Serving on the GPU: requests that run together in batched launches give
bitwise the same fields as each request run alone."""
import numpy as np
import pytest

from gpu_util import ensure_built, need_gpu
from paper_0912_4230_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    ensure_built()


def _stream():
    # arrivals within microseconds of each other: the requests are admitted
    # together and overlap on the GPU however fast each one runs
    reqs = I.request_stream(n=7, rate=1e6, edge_lo=18, edge_hi=40, steps_lo=30, steps_hi=140,
                            arrival_seed=11, param_seed=12, medium_seed0=500)
    # make sure both physics appear
    reqs[0].physics = I.IMMISCIBLE
    reqs[1].physics = I.MISCIBLE
    return reqs


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_alone_equals_mix(storage):
    import torch
    from paper_0912_4230_amd.serve import GpuExecutor, serve
    from paper_0912_4230_amd.sim import Simulation
    reqs = _stream()
    probs = {r.rid: I.request_problem(r) for r in reqs}
    ex = GpuExecutor(storage=storage, keep_results=True, problems=probs)
    st = serve(reqs, ex, budget_bytes=1 << 40, tick_steps=16)
    print(f"[serving] {storage}: max_active={st['max_active']} ticks={st['ticks']} "
          f"p50={st['p50_s']:.3f}s p99={st['p99_s']:.3f}s", flush=True)
    assert st["completed"] == len(reqs)
    assert st["max_active"] >= 2
    for r in reqs:
        o = st["outcomes"][r.rid]
        assert o.status == "ok"
        rho_m, vel_m, conc_m, diag_m = o.result
        sim = Simulation(probs[r.rid], storage=storage)
        sim.step(r.steps)
        rho_a, vel_a, conc_a, diag_a = sim.moments()
        assert torch.equal(rho_m, rho_a) and torch.equal(vel_m, vel_a) and torch.equal(conc_m, conc_a), r.rid
        # every diagnostic except the residual (which refers to the previous
        # snapshot, taken at tick ends in the mix)
        keep = [0, 1, 2, 3, 4, 6, 7]
        assert np.array_equal(diag_m[keep], diag_a[keep]), r.rid
        sim.close()


def test_batch_of_different_shapes_matches_single_steps():
    """lbm_step_batch on lattices of different sizes, physics and step counts
    equals lbm_step on each."""
    import torch
    from paper_0912_4230_amd.sim import Simulation, step_batch
    obst = I.miscible(shape=(21, 15, 12), seed=8)
    obst.solid = I.sphere_obstacles(obst.shape, seed=9, solid_fraction=0.1, radius=(1.5, 2.5))
    probs = [I.miscible(shape=(20, 17, 13), seed=5), I.drop(shape=(24, 22, 20), radius=5.0),
             I.miscible(shape=(33, 9, 11), seed=6), I.drop(shape=(16, 16, 16), radius=4.0), obst]
    steps = [25, 40, 7, 33, 19]
    a = [Simulation(p, storage="f32") for p in probs]
    step_batch(a, steps)
    for p, n, s in zip(probs, steps, a):
        b = Simulation(p, storage="f32")
        b.step(n)
        ra, va, ca, _ = s.moments()
        rb, vb, cb, _ = b.moments()
        assert torch.equal(ra, rb) and torch.equal(va, vb) and torch.equal(ca, cb)
        assert torch.equal(s.populations(0), b.populations(0))
        assert s.steps_done == n
        b.close()
    for s in a:
        s.close()


def test_batch_covers_every_storage_and_tensor_form():
    """lbm_step_batch steps lattices of every storage mode and of both
    permeability forms (each group its own launch) exactly like lbm_step."""
    import torch
    from paper_0912_4230_amd.sim import Simulation, step_batch
    probs, storages = [], []
    for i, st in enumerate(("f64", "f32", "bf16", "f16", "bf16s", "f16s")):
        probs.append(I.miscible(shape=(17, 11, 9), seed=20 + i))
        storages.append(st)
    probs.append(I.miscible(shape=(15, 13, 10), seed=30, ring_angle=45.0))
    storages.append("f32")
    probs.append(I.miscible(shape=(15, 13, 10), seed=31, ring_angle=30.0))
    storages.append("bf16s")
    steps = [9, 12, 7, 5, 11, 8, 10, 6]
    a = [Simulation(p, storage=st) for p, st in zip(probs, storages)]
    step_batch(a, steps)
    for p, st, n, s in zip(probs, storages, steps, a):
        b = Simulation(p, storage=st)
        b.step(n)
        assert s.steps_done == n
        ra, va, ca, _ = s.moments()
        rb, vb, cb, _ = b.moments()
        assert torch.equal(ra, rb) and torch.equal(va, vb) and torch.equal(ca, cb), st
        b.close()
    for s in a:
        s.close()
