"""Physics of the two-fluid model at 3D sizes on the GPU (FP32), where the
FP64 oracle is too slow to run: the properties its quasi-2D pins fix.

- Laplace law (surface-tension term of Eqs. equilc1/2; p = rho c_s^2 / eps,
  Sec. 2): a static 3D drop has Delta p = 2 sigma / R, so Delta p R is the same
  for every radius, and Delta p R / 2 equals the tension measured on a
  quasi-2D drop (Delta p = sigma / R) by the same kernels.
- Contact angle from the wall colour C_w = (1 + cos theta)/2: a sessile 3D
  drop settles to the wall's angle (sphere fit of the C = 1/2 surface).
"""
import numpy as np
import pytest

from gpu_util import ensure_built, need_gpu
from paper_0912_4230_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    ensure_built()


def _run(p, steps):
    from paper_0912_4230_amd.sim import Simulation
    sim = Simulation(p, storage="f32")
    sim.step(steps)
    rho, vel, conc, dg = sim.moments()
    out = rho.double().cpu().numpy(), conc.double().cpu().numpy(), dg
    sim.close()
    return out


def _pressure_jump(rho, c, centre, R):
    nz, ny, nx = rho.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = [np.abs(a - ca) for a, ca in zip((x, y, z), centre)]
    d = [np.minimum(da, n - da) for da, n in zip(d, (nx, ny, nz))]
    dist = np.sqrt(sum(da ** 2 for da in d))
    return (rho[dist < R - 3].mean() - rho[dist > R + 3].mean()) / 3.0


def test_laplace_law_3d_and_consistency_with_2d():
    N, steps = 56, 2500
    vals = []
    for R in (8, 11, 14):
        p = I.drop(shape=(N, N, N), radius=R, speed=0.0, walls=False)
        rho, c, dg = _run(p, steps)
        assert dg[7] == 0
        Reff = (3.0 * (c > 0.5).sum() / (4.0 * np.pi)) ** (1.0 / 3.0)
        dp = _pressure_jump(rho, c, (N // 2,) * 3, R)
        assert dp > 0
        vals.append(dp * Reff)
    vals = np.array(vals)
    print(f"[physics] 3D Laplace: dp R = {vals}", flush=True)
    assert (vals.max() - vals.min()) / vals.mean() < 0.05, vals
    # quasi-2D cylinder with the same kernels: dp R = sigma
    R = 12
    p = I.drop(shape=(N, N, 1), radius=R, speed=0.0, walls=False, centre=(N // 2, N // 2, 0))
    rho, c, dg = _run(p, steps)
    Reff = np.sqrt((c[0] > 0.5).sum() / np.pi)
    sigma = _pressure_jump(rho, c, (N // 2, N // 2, 0), R) * Reff
    print(f"[physics] quasi-2D sigma = {sigma:.5f}, 3D dp R / 2 = {vals.mean() / 2:.5f}", flush=True)
    assert abs(vals.mean() / 2 / sigma - 1.0) < 0.1


def _sphere_fit(P):
    A = np.concatenate([P, np.ones((len(P), 1))], 1)
    b = -(P ** 2).sum(1)
    sol = np.linalg.lstsq(A, b, rcond=None)[0]
    c = -sol[:3] / 2
    return c, np.sqrt((c ** 2).sum() - sol[3])


@pytest.mark.parametrize("angle", [60.0, 120.0])
def test_contact_angle_3d(angle):
    NX, NZ = 64, 40
    p = I.drop(shape=(NX, NX, NZ), radius=12, speed=0.0, centre=(NX // 2, NX // 2, 1),
               bottom_angle=angle, top_angle=90.0)
    rho, c, dg = _run(p, 5000)
    assert dg[7] == 0
    pts = []
    # C = 1/2 crossings along z columns and along x rows, away from the walls
    for k in range(3, NZ - 3):
        for j in range(NX):
            row = c[k, j, :]
            s = np.nonzero((row[:-1] - 0.5) * (row[1:] - 0.5) < 0)[0]
            for i in s:
                pts.append((i + (row[i] - 0.5) / (row[i] - row[i + 1]), j, k - 0.5))
    for j in range(NX):
        for i in range(NX):
            col = c[:, j, i]
            for k in range(3, NZ - 3):
                if (col[k] - 0.5) * (col[k + 1] - 0.5) < 0:
                    pts.append((i, j, k + (col[k] - 0.5) / (col[k] - col[k + 1]) - 0.5))
    ctr, R = _sphere_fit(np.array(pts, float))
    # the wall plane is z = 0 in these coordinates (cell k sits at k - 0.5)
    theta = np.degrees(np.arccos(np.clip(-ctr[2] / R, -1, 1)))
    print(f"[physics] sessile drop on a {angle:.0f}-degree wall: {theta:.1f} degrees (R = {R:.1f})", flush=True)
    assert abs(theta - angle) < 10.0, theta


def test_square_relaxes_to_a_circle():
    """Sec. 5.4 (surface smoothing, its figure only): a 20 x 20 square of fluid 1
    in a 100 x 100 x 1 box, tau = 0.7, A = 0.001, 10000 steps, becomes round.
    The radius of the C = 1/2 contour about the centre of mass varies by 10%
    (RMS over angle) for the square and must end below 1%; the fluid-1 mass
    is conserved (FP64 storage: to rounding)."""
    from paper_0912_4230_amd.sim import Simulation
    p = I.square()
    sim = Simulation(p, storage="f64")
    c0 = sim.moments()[2].double().cpu().numpy()[0]

    def roundness(c):
        ys, xs = np.nonzero(c > 0.5)
        cx, cy = xs.mean(), ys.mean()
        pts = []
        for ang in np.linspace(0, 2 * np.pi, 180, endpoint=False):
            d = np.array([np.cos(ang), np.sin(ang)])
            r = np.arange(0, 40, 0.05)
            px, py = cx + r * d[0], cy + r * d[1]
            ix, iy = np.floor(px).astype(int), np.floor(py).astype(int)
            fx, fy = px - ix, py - iy
            v = ((1 - fx) * (1 - fy) * c[iy, ix] + fx * (1 - fy) * c[iy, ix + 1]
                 + (1 - fx) * fy * c[iy + 1, ix] + fx * fy * c[iy + 1, ix + 1])
            k = np.nonzero(v < 0.5)[0][0]
            pts.append(r[k])
        pts = np.array(pts)
        return pts.std() / pts.mean(), pts.mean()

    s0, r0 = roundness(c0)
    m0 = sim.diag()[4]
    sim.step(10000)
    rho, vel, c, dg = sim.moments()
    s1, r1 = roundness(c.double().cpu().numpy()[0])
    print(f"[physics] square -> circle: contour radius RMS/mean {s0:.3f} -> {s1:.4f}, mean radius {r0:.2f} -> {r1:.2f}",
          flush=True)
    assert dg[7] == 0
    assert s0 > 0.05 and s1 < 0.01
    assert abs(dg[4] / m0 - 1.0) < 1e-12
    sim.close()
