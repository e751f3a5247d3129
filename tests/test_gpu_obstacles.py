"""Obstacle cells (per-cell solid mask) on the GPU, through the C ABI, against
the FP64 oracle: relative L2 over fluid cells, FP64 1e-10, FP32 1e-5 for
rho and C (V' of the porous workloads per case, as in the other parity
tests)."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import ensure_built, errors, need_gpu, report, run_pair
from paper_0912_4230_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    need_gpu()
    ensure_built()


def test_duct_fp64_matches_oracle_and_closed_form():
    from test_oracle_obstacles import duct_closed_form
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    p = I.duct(shape=(3, 20, 20), G=1e-6, tau=tau)
    g, r, mask, dg, od = run_pair(p, 4000, "f64", chunks=[1000, 3000])
    e = errors(g, r, mask)
    report("duct 3x20x20 x4000 f64", e)
    assert e["rho"] < 1e-10 and e["vel"] < 1e-10
    s = np.arange(1, 19) - 9.5
    Y, Z = np.meshgrid(s, s, indexing="xy")
    exact = duct_closed_form(Y, Z, 18.0, 18.0, 1e-6, (tau - 0.5) / 3.0)
    num = g[1][0, 1:19, 1:19, 1]
    assert np.linalg.norm(num - exact) / np.linalg.norm(exact) < 1e-3
    # obstacles read 0
    assert np.all(g[0][~mask] == 0.0) and np.all(g[1][:, ~mask] == 0.0)


def _miscible_obstacles(shape, seed=0):
    p = I.miscible(shape=shape, seed=seed)
    p.solid = I.sphere_obstacles(shape, seed=seed + 7, solid_fraction=0.12, radius=(1.5, 3.5))
    return p


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_miscible_obstacles_ragged(storage, tol):
    """Miscible workload physics with spherical obstacles between the
    reservoirs, on a ragged grid of several blocks."""
    p = _miscible_obstacles((37, 29, 23))
    g, r, mask, dg, od = run_pair(p, 120, storage, chunks=[60, 60])
    assert mask.sum() < 0.9 * mask.size
    e = errors(g, r, mask)
    report(f"miscible+obstacles 37x29x23 x120 {storage}", e)
    assert e["rho"] < tol and e["conc"] < tol
    assert e["vel"] < (tol if storage == "f64" else 3e-5)   # measured FP32: 1.02e-5
    assert abs(dg[4] - od[4]) < 10 * tol * od[4]


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_miscible_obstacles_longitudinal(storage, tol):
    """Flow along the permeable axis past obstacles: V' ~ 1e-4."""
    shape = (20, 40, 18)
    p = I.miscible(shape=shape, seed=3, reservoirs=False)
    p.faces[2] = I.Face(kind=I.RESERVOIR, rho=1.02, conc=1.0)
    p.faces[3] = I.Face(kind=I.RESERVOIR, rho=1.0, conc=0.0)
    solid = I.sphere_obstacles(shape, seed=11, solid_fraction=0.1, radius=(1.5, 3.0), keep_planes=())
    solid[:, [0, 1, -2, -1], :] = 0      # keep the y reservoir layers free
    p.solid = solid
    g, r, mask, dg, od = run_pair(p, 150, storage)
    e = errors(g, r, mask)
    report(f"miscible+obstacles longitudinal 20x40x18 x150 {storage}", e)
    assert e["rho"] < tol and e["conc"] < tol and e["vel"] < tol   # measured FP32 V': 3.2e-7


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_two_fluid_obstacles(storage, tol):
    """Two-fluid drop among obstacles of contact angle 60 degrees, walls of
    120 / 90 degrees on z."""
    shape = (33, 31, 29)
    p = I.drop(shape=shape, radius=7.0, speed=0.05)
    solid = I.sphere_obstacles(shape, seed=5, solid_fraction=0.08, radius=(1.5, 3.0), keep_planes=())
    solid[p.c0 > 0] = 0
    p.solid = solid
    p.solid_angle = 60.0
    g, r, mask, dg, od = run_pair(p, 120, storage, chunks=[40, 80])
    e = errors(g, r, mask)
    report(f"two-fluid+obstacles 33x31x29 x120 {storage}", e)
    assert e["rho"] < tol and e["conc"] < tol and e["vel"] < tol   # measured FP32 V': 2.7e-6
    assert abs(dg[4] - od[4]) < 10 * tol * od[4]


def test_obstacles_split_storage():
    """FP16 split storage with obstacles: the bounds of the obstacle-free
    FP16-split case."""
    p = _miscible_obstacles((37, 29, 23), seed=1)
    p.faces[2] = I.Face(kind=I.RESERVOIR, rho=1.02, conc=1.0)
    p.faces[3] = I.Face(kind=I.RESERVOIR, rho=1.0, conc=0.0)
    p.faces[0] = I.Face()
    p.faces[1] = I.Face()
    g, r, mask, dg, od = run_pair(p, 120, "f16s")
    e = errors(g, r, mask)
    report("miscible+obstacles 37x29x23 x120 f16s", e)
    # measured: rho 3.1e-7, drho 8.1e-5, V' 2.9e-4, C 3.4e-6
    assert e["rho"] < 6.2e-7 and e["drho"] < 1.6e-4 and e["vel"] < 5.8e-4 and e["conc"] < 6.9e-6


def test_all_solid_and_single_fluid_cell():
    """Degenerate masks: every cell an obstacle (no fluid at all), and one
    fluid cell enclosed by obstacles (every link bounces back)."""
    p = I.poiseuille(shape=(8, 6, 5), G=1e-4)
    p.faces = [I.Face() for _ in range(6)]
    p.solid = np.ones(p.eps.shape, dtype=np.uint8)
    g, r, mask, dg, od = run_pair(p, 10, "f64")
    assert mask.sum() == 0
    assert np.all(g[0] == 0.0) and np.all(g[1] == 0.0) and np.all(dg[:7] == 0.0)
    p.solid[2, 3, 4] = 0
    p.rho0 = np.full(p.eps.shape, 1.03)
    g, r, mask, dg, od = run_pair(p, 25, "f64")
    assert mask.sum() == 1
    e = errors(g, r, mask)
    report("one enclosed fluid cell f64", e)
    assert e["rho"] < 1e-12 and abs(g[0][2, 3, 4] - 1.03) < 1e-12
    assert abs(g[1][0, 2, 3, 4] - r[1][0, 2, 3, 4]) < 1e-14


def test_solid_without_mask_flag_rejected():
    import torch
    from paper_0912_4230_amd import binding as B
    from paper_0912_4230_amd.sim import make_desc
    p = I.poiseuille(shape=(8, 6, 5))
    d = make_desc(p, B.LBM_F32)
    assert d.solid_mask == 0
    nbytes = B.lbm_workspace_bytes(d)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    h = B.lbm_create(d, ws.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    solid = torch.zeros(8 * 6 * 5, dtype=torch.uint8, device="cuda")
    m = B.lbm_medium()
    m.eps_uniform = 0.5
    m.solid = solid.data_ptr()
    st = B.lib().lbm_set_medium(h, C.byref(m))
    assert st == B.LBM_EINVAL
    B.lbm_destroy(h)
