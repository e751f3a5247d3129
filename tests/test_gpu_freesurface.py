"""Free-surface mode (Sec. 3) on the GPU through the C ABI, against the FP64
oracle.

FP64: the cell classes agree exactly at every checkpoint (the conversion
decisions are taken in double on both sides), masses, rho, V' and the fill
fraction within 1e-10 relative L2, the total liquid mass of the diagnostics
within 1e-12.  FP32 and 16-bit storage: the classes may part where a mass
sits at a threshold, so those runs are held to conservation of the total
liquid mass and to the ballistic fall.  The mass of a liquid cell is the
sum of its stored populations, so it is conserved only to their rounding:
1e-6 in FP32 over 1200 steps; in the 16-bit formats, where the drop falls at
up to 0.08 (the velocity part of the populations is rounded to 8 or 11
bits), 2e-3.  The paper's droplet (Sec. 5.3,
140x140x1, R = 8, tau = 0.7, G = 1e-6) checks its two printed facts: mass
error below 1% and the impact near 10600 steps.
"""
import numpy as np
import pytest

from gpu_util import ensure_built, need_gpu, rel_l2
from paper_0912_4230_amd import inputs as I

pytestmark = pytest.mark.gpu

LIQ, IF, GAS = 2, 1, 0


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    ensure_built()


def _gpu_state(sim):
    rho, vel, lam, dg = sim.moments()
    cls, mass, lost = sim.free_surface()
    return (rho.double().cpu().numpy(), vel.double().cpu().numpy(), lam.double().cpu().numpy(),
            cls.cpu().numpy(), mass.cpu().numpy(), lost, dg)


def _compare(p, checkpoints, storage="f64", diag_every=0, tol=1e-10, name=""):
    from oracle import oracle as O
    from paper_0912_4230_amd.sim import Simulation
    sim = Simulation(p, storage=storage, diag_every=diag_every)
    o = O.Oracle(p)
    fluid = o.cell_types() == 0
    t = 0
    worst = 0.0
    for tc in checkpoints:
        sim.step(tc - t)
        o.step(tc - t)
        t = tc
        rho, vel, lam, cls, mass, lost, dg = _gpu_state(sim)
        ocls, omass, olost = o.fs_state()
        r, v, l = o.moments()
        od = o.diag()
        assert (cls[~fluid] == 3).all()
        mism = int((cls[fluid] != ocls[fluid]).sum())
        assert mism == 0, f"{name} step {tc}: {mism} cells of another class"
        e = {"mass": rel_l2(mass, omass, fluid), "rho": rel_l2(rho, r, fluid),
             "vel": rel_l2(vel, v, fluid), "lam": rel_l2(lam, l, fluid)}
        print(f"[parity] free surface {name} {storage} step {tc}: "
              + ", ".join(f"{k}={x:.2e}" for k, x in e.items())
              + f", IF cells {int((cls == IF).sum())}, total mass {dg[4]:.12g}", flush=True)
        assert all(x < tol for x in e.values()), e
        assert abs(dg[4] - od[4]) <= 1e-12 * od[4]
        assert abs(dg[0] - od[0]) <= 1e-12 * od[0]
        assert lost == olost == 0.0
        worst = max(worst, *e.values())
    sim.close()
    o.close()
    return worst


def test_drop_fall_and_impact_f64():
    p = I.falling_drop(shape=(40, 60, 1), radius=5.0, centre=(20.0, 40.0, 0.0), G=1e-4, tau=0.7)
    _compare(p, [1, 50, 300, 700, 900, 1200], diag_every=50, name="2D drop 40x60")


def test_porous_3d_drop_with_obstacles_f64():
    shape = (14, 12, 18)
    p = I.falling_drop(shape=shape, radius=4.2, centre=(7.0, 6.0, 11.5), G=3e-4, tau=0.8, axis=2)
    eps, kinv = I.spruce_medium(shape, seed=5, ratio=20.0)
    p.eps, p.kinv = eps, kinv * 1e-2
    p.forchheimer = True
    solid = I.block_obstacles(shape, seed=2, solid_fraction=0.08, free_x=0)
    solid[:, :, :] = solid & (np.arange(shape[2])[:, None, None] < 5)   # obstacles in the floor region
    p.solid = solid
    _compare(p, [1, 60, 150, 240], diag_every=7, name="3D porous drop with obstacles 14x12x18")


def test_ragged_box_f64():
    """A box whose cell count is not a multiple of the 16-cell tiles of the
    class passes (13 x 11 x 17 = 2431 cells) nor of the 256-cell blocks."""
    shape = (13, 11, 17)
    p = I.falling_drop(shape=shape, radius=3.6, centre=(6.3, 5.4, 10.2), G=5e-4, tau=0.75, axis=2)
    assert (13 * 11 * 17) % 16 != 0
    _compare(p, [30, 90, 200], diag_every=13, name="ragged drop 13x11x17")


def test_surface_tension_drop_f64():
    """Surface tension at the free surface (Sec. 5.4): a 2D drop relaxing from
    a square and a 3D drop falling into a porous medium with A != 0."""
    n = 40
    p = I.falling_drop(shape=(n, n, 1), radius=0.0, G=0.0, tau=0.7, wall=False)
    z, y, x = np.meshgrid(np.arange(1), np.arange(n), np.arange(n), indexing="ij")
    p.c0 = ((np.abs(x - 19.5) < 7) & (np.abs(y - 19.5) < 7)).astype(float)
    p.A = 0.003
    _compare(p, [1, 100, 400, 900], diag_every=50, name="square with surface tension 40x40")
    shape = (14, 12, 18)
    q = I.falling_drop(shape=shape, radius=4.2, centre=(7.0, 6.0, 11.5), G=3e-4, tau=0.8, axis=2)
    eps, kinv = I.spruce_medium(shape, seed=5, ratio=20.0)
    q.eps, q.kinv = eps, kinv * 1e-2
    q.A = 0.002
    _compare(q, [60, 200], name="3D drop with surface tension 14x12x18")


def test_interface_rows_beyond_the_launch_prefix_f64():
    """The stream/collide pass takes the rows (256 cells) listed as holding
    interface cells first, in a prefix of 1/32 of the rows and at least 64;
    listed rows beyond the prefix are processed by their own row blocks.  A
    wavy surface puts interface cells in most of the 480 rows of this box, so
    both paths run; the result is the oracle's, class for class."""
    from paper_0912_4230_amd.sim import Simulation
    shape = (64, 40, 48)
    p = I.falling_drop(shape=shape, radius=0.0, G=2e-4, tau=0.8, axis=1)
    z, y, x = np.meshgrid(np.arange(shape[2]), np.arange(shape[1]), np.arange(shape[0]), indexing="ij")
    h = 20.0 + 6.0 * np.sin(2 * np.pi * x / 16.0) * np.cos(2 * np.pi * z / 12.0)
    p.c0 = np.clip(h - y, 0.0, 1.0)
    sim = Simulation(p, storage="f64")
    sim.step(1)
    cls = sim.free_surface()[0].cpu().numpy().reshape(-1)
    rows_with_if = int((cls.reshape(-1, 256) == IF).any(axis=1).sum())
    sim.close()
    assert rows_with_if > 64, rows_with_if
    _compare(p, [1, 25, 80], diag_every=11, name=f"wavy surface 64x40x48 ({rows_with_if} of 480 rows)")


def test_full_tensor_medium_f64():
    shape = (16, 13, 15)
    p = I.falling_drop(shape=shape, radius=4.0, centre=(8.0, 6.5, 9.0), G=4e-4, tau=0.9, axis=2)
    eps, kinv = I.inclined_spruce_medium(shape, seed=4, ratio=10.0, angle_deg=35.0)
    p.eps, p.kinv = eps, kinv * 3e-3
    _compare(p, [40, 160], name="inclined medium 16x13x15")


@pytest.mark.parametrize("speed", [0.05, -0.04])
def test_slab_translates_f64(speed):
    p = I.slab(shape=(48, 4, 3), lo=18, hi=30, speed=speed)
    _compare(p, [40, 200], name=f"slab u={speed}")


def test_all_liquid_is_the_single_fluid_step():
    """With no gas the free-surface step is the single-fluid step, bit for bit."""
    from paper_0912_4230_amd.sim import Simulation
    shape = (20, 17, 9)
    eps, kinv = I.spruce_medium(shape, seed=3)
    faces = [I.Face() for _ in range(6)]
    faces[4] = I.Face(kind=I.WALL)
    faces[5] = I.Face(kind=I.WALL)
    out = []
    for phys, c0 in ((I.SINGLE, None), (I.FREESURF, np.ones((9, 17, 20)))):
        p = I.Problem(shape=shape, physics=phys, G=(2e-4, -1e-4, 5e-5), forchheimer=True, faces=faces,
                      eps=eps, kinv=kinv, c0=c0).fill_defaults()
        sim = Simulation(p, storage="f32")
        sim.step(30)
        rho, vel, conc, dg = sim.moments()
        out.append((rho.cpu().numpy(), vel.cpu().numpy(), sim.populations(0).cpu().numpy(), dg))
        sim.close()
    a, b = out
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert a[3][0] == b[3][0] and b[3][4] == b[3][0]


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16", "bf16s", "f16s"])
def test_reduced_precision_conserves_mass_and_falls(storage):
    from paper_0912_4230_amd.sim import Simulation
    G = 1e-4
    p = I.falling_drop(shape=(40, 60, 1), radius=5.0, centre=(20.0, 40.0, 0.0), G=G, tau=0.7)
    sim = Simulation(p, storage=storage)
    M0 = sim.diag()[4]
    y = np.arange(60)[None, :, None]
    m = sim.free_surface()[1].cpu().numpy()
    y0 = (m * y).sum() / m.sum()
    tol = 1e-6 if storage == "f32" else 2e-3
    for t in (200, 400, 600, 800, 1200):
        sim.step(t - sim.steps_done)
        rho, vel, lam, cls, mass, lost, dg = _gpu_state(sim)
        assert lost == 0.0
        assert abs(dg[4] / M0 - 1.0) < tol, (t, dg[4], M0)
        assert abs(mass.sum() / M0 - 1.0) < tol
        if t <= 800:
            yc = (mass * y).sum() / mass.sum()
            assert abs((y0 - yc) / (0.5 * G * t * t) - 1.0) < (0.02 if storage == "f32" else 0.06), (t, y0 - yc)
    print(f"[physics] free-surface drop {storage}: mass drift {dg[4] / M0 - 1.0:.2e} after 1200 steps", flush=True)
    sim.close()


def test_batched_free_surface_equals_single_calls():
    from paper_0912_4230_amd.sim import Simulation, step_batch
    probs = [I.falling_drop(shape=(40, 60, 1), radius=5.0, centre=(20.0, 40.0, 0.0), G=1e-4),
             I.falling_drop(shape=(23, 19, 17), radius=4.0, centre=(11.0, 9.0, 9.0), G=2e-4, axis=2),
             I.miscible(shape=(20, 16, 12), seed=1)]
    steps = [150, 90, 120]
    ref = []
    for p, n in zip(probs, steps):
        s = Simulation(p, storage="f32")
        s.step(n)
        ref.append(s)
    sims = [Simulation(p, storage="f32") for p in probs]
    step_batch(sims, steps)
    for a, b in zip(ref, sims):
        ra, rb = a.moments(), b.moments()
        for x, y in zip(ra[:3], rb[:3]):
            assert torch_equal(x, y)
        if a.problem.physics == I.FREESURF:
            fa, fb = a.free_surface(), b.free_surface()
            assert torch_equal(fa[0], fb[0]) and torch_equal(fa[1], fb[1])
        a.close()
        b.close()


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


def test_all_gas_and_rejections():
    import ctypes as C
    import torch
    from paper_0912_4230_amd import binding as B
    from paper_0912_4230_amd.sim import Simulation, make_desc
    p = I.falling_drop(shape=(9, 8, 7), radius=0.0, G=1e-4, axis=2)
    assert not p.c0.any()
    sim = Simulation(p, storage="f64")
    sim.step(5)
    rho, vel, lam, cls, mass, lost, dg = _gpu_state(sim)
    assert not rho.any() and not vel.any() and not lam.any() and not mass.any()
    assert dg[0] == 0.0 and dg[4] == 0.0 and dg[7] == 0
    sim.close()
    # reservoir faces are rejected before any GPU call; so is lbm_free_surface
    # on a handle of another physics
    q = I.slab()
    q.faces[0] = I.Face(kind=I.RESERVOIR)
    q.faces[1] = I.Face(kind=I.RESERVOIR)
    assert B.lbm_workspace_bytes(make_desc(q, B.LBM_F32)) == 0
    s2 = Simulation(I.miscible(shape=(8, 8, 8), seed=0), storage="f32")
    lost = C.c_double(0.0)
    assert B.lib().lbm_free_surface(s2.h, None, None, None, C.byref(lost)) == B.LBM_EINVAL
    s2.close()


def test_paper_droplet_mass_and_impact():
    """Sec. 5.3: 140x140x1, R = 8, rho = 1, tau = 0.7, G = 1e-6 toward the wall at
    y = 0.  The paper reports a mass error below 1% over 20000 steps and the
    impact after about 10600 steps, which for a drop released at rest is a fall
    of G t^2 / 2 = 56 cells: the drop is placed that high (its height is not
    printed).  Impact is taken as the step at which the centre-of-mass velocity
    of the liquid first falls 10% behind the free-fall velocity G t."""
    from paper_0912_4230_amd.sim import Simulation
    G, R = 1e-6, 8.0
    yc = 0.5 + R + 0.5 * G * 10600.0 ** 2
    p = I.falling_drop(shape=(140, 140, 1), radius=R, centre=(70.0, yc, 0.0), G=G, tau=0.7)
    sim = Simulation(p, storage="f64")
    M0 = sim.diag()[4]
    t_hit = None
    worst = 0.0
    for t in range(200, 20001, 200):
        sim.step(200)
        rho, vel, lam, cls, mass, lost, dg = _gpu_state(sim)
        worst = max(worst, abs(dg[4] / M0 - 1.0))
        vy = (mass * vel[1]).sum() / mass.sum()
        if t_hit is None and -vy < 0.9 * G * t:
            t_hit = t
    print(f"[physics] paper droplet: mass error {worst:.2e} over 20000 steps, impact at {t_hit} "
          f"(free fall from {yc - R - 0.5:.1f} cells: {np.sqrt(2 * (yc - R - 0.5) / G):.0f})", flush=True)
    assert worst < 1e-10
    assert t_hit is not None and abs(t_hit / 10600.0 - 1.0) < 0.05
    sim.close()


def test_paper_surface_smoothing():
    """Sec. 5.4 as the paper ran it: a 20 x 20 square of liquid in a 100 x 100 x 1
    box with the free surface, rho = 1, tau = 0.7, A = 0.001, no force, 10000
    steps: the square becomes round (radius RMS / mean 0.104 -> below 0.015)
    and keeps its mass; without the term it stays a square."""
    from paper_0912_4230_amd.sim import Simulation
    n = 100
    p = I.falling_drop(shape=(n, n, 1), radius=0.0, G=0.0, tau=0.7, wall=False)
    z, y, x = np.meshgrid(np.arange(1), np.arange(n), np.arange(n), indexing="ij")
    p.c0 = ((np.abs(x - 49.5) < 10) & (np.abs(y - 49.5) < 10)).astype(float)
    out = {}
    for A in (0.001, 0.0):
        p.A = A
        sim = Simulation(p, storage="f32")
        M0 = sim.diag()[4]
        lam0 = sim.moments()[2].double().cpu().numpy()
        sim.step(10000)
        rho, vel, lam, dg = sim.moments()
        out[A] = (_roundness(lam0), _roundness(lam.double().cpu().numpy()), dg[4] / M0 - 1.0)
        sim.close()
    print(f"[physics] paper surface smoothing 100x100x1 x10000: A=0.001 roundness {out[0.001][0]:.3f} -> "
          f"{out[0.001][1]:.4f} (mass drift {out[0.001][2]:.1e}); A=0 {out[0.0][0]:.3f} -> {out[0.0][1]:.3f}",
          flush=True)
    assert out[0.001][0] > 0.09 and out[0.001][1] < 0.015
    assert abs(out[0.0][1] - out[0.0][0]) < 1e-3
    assert abs(out[0.001][2]) < 1e-5


def _roundness(lam):
    c = lam[0]
    n = c.shape[0]
    cx = (c * np.arange(c.shape[1])[None, :]).sum() / c.sum()
    cy = (c * np.arange(n)[:, None]).sum() / c.sum()
    pts = []
    for ang in np.linspace(0, 2 * np.pi, 180, endpoint=False):
        r = np.arange(0, n / 2 - 2, 0.05)
        px, py = cx + r * np.cos(ang), cy + r * np.sin(ang)
        ix, iy = np.floor(px).astype(int), np.floor(py).astype(int)
        fx, fy = px - ix, py - iy
        v = ((1 - fx) * (1 - fy) * c[iy, ix] + fx * (1 - fy) * c[iy, ix + 1]
             + (1 - fx) * fy * c[iy + 1, ix] + fx * fy * c[iy + 1, ix + 1])
        pts.append(r[np.nonzero(v < 0.5)[0][0]])
    pts = np.array(pts)
    return pts.std() / pts.mean()
