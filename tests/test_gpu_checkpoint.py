"""Checkpoint and resume through the C ABI (lbm_state_bytes, lbm_save_state,
lbm_load_state): n steps, a checkpoint, a fresh lattice of the same problem
(another workspace) loaded from it and n more steps give bitwise the state of
2n uninterrupted steps, for every physics and a range of storage forms; a
checkpoint that does not fit a lattice is rejected before anything is
written."""
import numpy as np
import pytest

from gpu_util import ensure_built, need_gpu

from paper_0912_4230_amd import binding as B
from paper_0912_4230_amd import inputs as I

pytestmark = pytest.mark.gpu

N = 13   # odd: the checkpoint is taken with the second population copy current


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    ensure_built()


def _problem(case):
    if case.startswith("miscible"):
        return I.miscible(shape=(37, 29, 23), seed=0)
    if case.startswith("species"):
        from test_gpu_species import _three_solutes
        return _three_solutes()
    if case.startswith("two-fluid"):
        return I.drop(shape=(33, 31, 29), radius=8.0, speed=0.05)
    if case.startswith("tensor"):
        p = I.miscible(shape=(30, 26, 22), seed=2, ring_angle=45.0)
        p.solid = I.sphere_obstacles(p.shape, seed=5, solid_fraction=0.08, radius=(1.5, 3.0))
        return p
    if case.startswith("freesurface"):
        return I.penetration(shape=(40, 36, 34), seed=1)
    raise ValueError(case)


def _state(sim, two, fs):
    rho, vel, conc, dg = sim.moments(check=False)
    out = [rho.cpu().numpy(), vel.cpu().numpy(), conc.cpu().numpy(), dg, sim.populations(0).cpu().numpy()]
    if two:
        out.append(sim.populations(1).cpu().numpy())
    if fs:
        cls, mass, lam, lost = sim.free_surface(fill=True)
        out += [cls.cpu().numpy(), mass.cpu().numpy(), lam.cpu().numpy(), np.array([lost])]
    return out


@pytest.mark.parametrize("case,storage", [("miscible", "f32"), ("miscible", "f16s"), ("miscible", "bf16"),
                                          ("species", "bf16s"), ("two-fluid", "bf16"), ("tensor", "f64"),
                                          ("freesurface", "f32"), ("freesurface", "bf16"),
                                          ("freesurface", "f16s"), ("two-fluid", "bf16s"), ("two-fluid", "f16")])
def test_resume_is_bitwise(case, storage):
    from paper_0912_4230_amd.sim import Simulation
    p = _problem(case)
    two = p.physics in (I.MISCIBLE, I.IMMISCIBLE)
    fs = p.physics == I.FREESURF
    a = Simulation(p, storage=storage, diag_every=5)
    a.step(N)
    a.step(N)
    ref = _state(a, two, fs)
    a.close()
    b = Simulation(p, storage=storage, diag_every=5)
    b.step(N)
    buf = b.save_state()
    assert buf.nbytes == B.lbm_state_bytes(b.h) and buf.nbytes <= b.nbytes + 4096
    b.close()
    c = Simulation(p, storage=storage, diag_every=5)
    c.step(3)                       # state that the load replaces
    c.load_state(buf)
    assert c.steps_done == N
    c.step(N)
    got = _state(c, two, fs)
    c.close()
    print(f"[checkpoint] {case} {storage}: {buf.nbytes} bytes, resumed after {N} steps", flush=True)
    for k, (x, y) in enumerate(zip(got, ref)):
        assert np.array_equal(x, y, equal_nan=True), (case, storage, k)


def test_resume_into_the_static_workspace():
    """A checkpoint of a lattice in a caller's workspace loads into the
    library's static workspace (another device address) and continues
    bitwise."""
    from paper_0912_4230_amd.sim import Simulation
    p = I.miscible(shape=(24, 20, 18), seed=4)
    a = Simulation(p, storage="f32", diag_every=5)
    a.step(2 * N)
    ref = _state(a, True, False)
    a.close()
    b = Simulation(p, storage="f32", diag_every=5)
    b.step(N)
    buf = b.save_state()
    b.close()
    c = Simulation(p, storage="f32", diag_every=5, static_workspace=True)
    try:
        c.load_state(buf).step(N)
        got = _state(c, True, False)
    finally:
        c.close()
    for k, (x, y) in enumerate(zip(got, ref)):
        assert np.array_equal(x, y), k


def test_checkpoint_that_does_not_fit_is_rejected():
    import torch
    from paper_0912_4230_amd.sim import Simulation, make_desc
    p = I.miscible(shape=(24, 20, 18), seed=4)
    p.eps = np.full(p.eps.shape, 0.45)      # uniform: held as one value unless asked otherwise
    a = Simulation(p, storage="f32", diag_every=5)
    a.step(4)
    buf = a.save_state()
    # a short host buffer for the save, and a truncated checkpoint for the load
    with pytest.raises(B.LbmError) as e:
        B.lbm_save_state(a.h, np.empty(buf.nbytes - 1, dtype=np.uint8))
    assert e.value.status == B.LBM_EINVAL
    with pytest.raises(B.LbmError) as e:
        B.lbm_load_state(a.h, buf[:-1])
    assert e.value.status == B.LBM_EINVAL
    ref = _state(a, True, False)
    # another storage, another size, a per-cell medium where it was uniform,
    # and bytes that are not a checkpoint: rejected, the lattice unchanged
    others = [Simulation(p, storage="f16s"), Simulation(I.miscible(shape=(24, 20, 17), seed=4), storage="f32"),
              Simulation(p, storage="f32", uniform_medium=False)]
    for o in others:
        before = _state(o, True, False)
        with pytest.raises(B.LbmError) as e:
            o.load_state(buf)
        assert e.value.status == B.LBM_EINVAL
        after = _state(o, True, False)
        assert all(np.array_equal(x, y) for x, y in zip(before, after))
        o.close()
    junk = buf.copy()
    junk[:8] = 0
    with pytest.raises(B.LbmError) as e:
        a.load_state(junk)
    assert e.value.status == B.LBM_EINVAL
    assert all(np.array_equal(x, y) for x, y in zip(_state(a, True, False), ref))
    a.close()
    # a lattice without a medium: LBM_ESTATE for both calls
    d = make_desc(p.fill_defaults(), B.LBM_F32)
    nbytes = B.lbm_workspace_bytes(d)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    h = B.lbm_create(d, ws.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    try:
        for call in (lambda: B.lbm_save_state(h, np.empty(buf.nbytes, dtype=np.uint8)),
                     lambda: B.lbm_load_state(h, buf)):
            with pytest.raises(B.LbmError) as e:
                call()
            assert e.value.status == B.LBM_ESTATE
    finally:
        B.lbm_destroy(h)
