"""Full permeability tensor on the GPU (eigenframe form), through the C ABI,
against the FP64 oracle (lab-frame form): relative L2 over fluid cells,
FP64 1e-10, FP32 1e-5 for rho and C; V' stated per case."""
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


def _uniform(k6, eps, G, forch, shape=(6, 5, 7)):
    p = I.Problem(shape=shape, physics=I.SINGLE, G=G, forchheimer=forch, nu0=0.1)
    p.fill_defaults()
    p.eps[:] = eps
    p.kinv = np.empty((6,) + p.eps.shape)
    for c in range(6):
        p.kinv[c] = k6[c]
    return p


def _rot(seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return q * np.sign(np.linalg.det(q))


def _packed(M):
    return np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_uniform_darcy_tensor_steady_state(storage, tol):
    Q = _rot(4)
    K = Q @ np.diag([2.0, 0.2, 0.05]) @ Q.T
    G = (1e-4, -3e-5, 5e-5)
    p = _uniform(_packed(np.linalg.inv(K)), 0.6, G, False)
    g, r, mask, dg, od = run_pair(p, 1500, storage)
    e = errors(g, r, mask)
    report(f"uniform Darcy tensor x1500 {storage}", e)
    assert e["rho"] < tol and e["vel"] < tol
    ref = K @ np.array(G) / 0.1
    assert np.abs(g[1][:, 3, 2, 3] - ref).max() < (1e-12 if storage == "f64" else 1e-5) * np.abs(ref).max()


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_uniform_forchheimer_tensor(storage, tol):
    Q = _rot(5)
    K = Q @ np.diag([3.0, 0.8, 0.3]) @ Q.T
    p = _uniform(_packed(np.linalg.inv(K)), 0.5, (1.2e-3, -4e-4, 6e-4), True)
    g, r, mask, dg, od = run_pair(p, 600, storage)
    e = errors(g, r, mask)
    report(f"uniform Forchheimer tensor x600 {storage}", e)
    assert e["rho"] < tol and e["vel"] < tol


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_inclined_rings_miscible_ragged(storage, tol):
    """Miscible workload physics in the medium with 45-degree rings (full
    K^-1 per cell), reservoirs on x, ragged grid."""
    p = I.miscible(shape=(37, 29, 23), seed=0, ring_angle=45.0)
    g, r, mask, dg, od = run_pair(p, 120, storage, chunks=[60, 60])
    e = errors(g, r, mask)
    report(f"inclined rings 37x29x23 x120 {storage}", e)
    assert e["rho"] < tol and e["conc"] < tol
    assert e["vel"] < tol   # measured FP32: 9.6e-7 (inclined rings), 3.1e-7 (wood)
    assert abs(dg[4] - od[4]) < 10 * tol * od[4]


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_paper_wood_medium_ragged(storage, tol):
    """The spruce medium of Sec. 5.5 from the paper's laws (density law,
    porosity, Eq. Ktensor with 45-degree rings; K^-1 up to 2.5e9), adhesive
    driven along the grain between reservoirs, the hardening law of Eq. nuall
    with the paper's constants; ragged grid."""
    p = I.wood(shape=(37, 29, 23), origin=(5, 3, 0))
    g, r, mask, dg, od = run_pair(p, 120, storage, chunks=[50, 70])
    e = errors(g, r, mask)
    report(f"paper wood medium 37x29x23 x120 {storage}", e)
    assert e["rho"] < tol and e["conc"] < tol
    assert e["vel"] < tol   # measured FP32: 9.6e-7 (inclined rings), 3.1e-7 (wood)


def test_inclined_rings_two_fluid_with_obstacles():
    """A drop in the inclined medium among obstacles: full tensor, obstacle
    mask and the two-fluid model together (FP64)."""
    shape = (30, 28, 26)
    p = I.drop(shape=shape, radius=6.0, speed=0.03)
    eps, kinv = I.inclined_spruce_medium(shape, seed=9, ratio=30.0, angle_deg=30.0)
    p.eps, p.kinv = eps, kinv
    solid = I.block_obstacles(shape, seed=3, solid_fraction=0.05, free_x=0)
    solid[p.c0 > 0] = 0
    p.solid = solid
    g, r, mask, dg, od = run_pair(p, 80, "f64", chunks=[30, 50])
    e = errors(g, r, mask)
    report("two-fluid, inclined rings, obstacles 30x28x26 x80 f64", e)
    assert e["rho"] < 1e-10 and e["conc"] < 1e-10 and e["vel"] < 1e-10


def test_inclined_rings_split_storage():
    p = I.miscible(shape=(37, 29, 23), seed=1, ring_angle=45.0)
    g, r, mask, dg, od = run_pair(p, 120, "f16s")
    e = errors(g, r, mask)
    report("inclined rings 37x29x23 x120 f16s", e)
    # measured: rho 2.4e-7, drho 1.2e-5, V' 6.1e-5, C 3.5e-6
    assert e["rho"] < 4.8e-7 and e["drho"] < 2.4e-5 and e["vel"] < 1.25e-4 and e["conc"] < 7.1e-6


def test_non_psd_tensor_rejected():
    import torch
    from paper_0912_4230_amd import binding as B
    from paper_0912_4230_amd.sim import make_desc
    p = _uniform(np.array([1.0, 1.0, 1.0, 2.0, 0.0, 0.0]), 0.5, (0.0, 0.0, 0.0), False, shape=(5, 4, 3))
    d = make_desc(p, B.LBM_F32)
    assert d.full_tensor == 1
    nbytes = B.lbm_workspace_bytes(d)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    h = B.lbm_create(d, ws.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    k = torch.from_numpy(np.ascontiguousarray(p.kinv, dtype=np.float32)).cuda()
    m = B.lbm_medium()
    m.eps_uniform = 0.5
    m.kinv = k.data_ptr()
    assert B.lib().lbm_set_medium(h, C.byref(m)) == B.LBM_EINVAL
    # the same tensor made positive definite is accepted
    p.kinv[3] = 0.5
    k = torch.from_numpy(np.ascontiguousarray(p.kinv, dtype=np.float32)).cuda()
    m.kinv = k.data_ptr()
    assert B.lib().lbm_set_medium(h, C.byref(m)) == B.LBM_OK
    B.lbm_destroy(h)


def test_rejected_medium_leaves_the_lattice_as_it_was():
    """A set-medium call rejected on the host (an out-of-range uniform
    porosity; an obstacle mask on a lattice without one) returns LBM_EINVAL
    and leaves a ready full-tensor lattice as it was: it steps on bitwise like
    a twin that never saw the call.  A medium rejected on the device (a tensor
    that is not positive semi-definite in one cell) leaves the lattice not
    ready: lbm_step returns LBM_ESTATE instead of stepping a half-set medium."""
    import torch
    from paper_0912_4230_amd import binding as B
    from paper_0912_4230_amd.sim import Simulation
    p = I.miscible(shape=(21, 19, 17), seed=4, ring_angle=45.0)
    a = Simulation(p, storage="f32", uniform_medium=False)
    b = Simulation(p, storage="f32", uniform_medium=False)
    assert a.desc.full_tensor == 1
    a.step(10)
    m = B.lbm_medium()
    m.eps_uniform = -1.0
    m.kinv_uniform = (C.c_double * 3)(0.0, 0.0, 0.0)
    assert B.lib().lbm_set_medium(a.h, C.byref(m)) == B.LBM_EINVAL
    mask = torch.zeros(p.shape[::-1], dtype=torch.uint8, device="cuda")
    m.eps_uniform = 0.5
    m.solid = mask.data_ptr()
    assert B.lib().lbm_set_medium(a.h, C.byref(m)) == B.LBM_EINVAL
    a.step(10)
    b.step(20)
    ra, va, ca, _ = a.moments()
    rb, vb, cb, _ = b.moments()
    assert torch.equal(ra, rb) and torch.equal(va, vb) and torch.equal(ca, cb)
    # a medium the device rejects: K^-1 with a large off-diagonal term in one cell
    k = np.array(p.kinv, dtype=np.float32, copy=True)
    k[3, 5, 6, 7] = 10.0 * float(np.max(np.abs(k[:3, 5, 6, 7]))) + 1.0
    kt = torch.from_numpy(np.ascontiguousarray(k)).cuda()
    et = torch.from_numpy(np.ascontiguousarray(p.eps, dtype=np.float32)).cuda()
    m = B.lbm_medium()
    m.eps = et.data_ptr()
    m.kinv = kt.data_ptr()
    assert B.lib().lbm_set_medium(a.h, C.byref(m)) == B.LBM_EINVAL
    assert B.lib().lbm_step(a.h, 1) == B.LBM_ESTATE
    a.close()
    b.close()
