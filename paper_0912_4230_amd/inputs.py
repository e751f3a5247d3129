"""Seeded synthetic inputs: problem descriptions and media shaped like the
workloads of the paper (Poiseuille channels of Sec. 5.1-5.2, the drop of
Sec. 5.3, the spruce-like ring medium of Sec. 5.5).

This module describes *inputs* only.  It holds none of the update's
arithmetic and is the one module that both the FP64 oracle (tests) and the
GPU library (product) are fed from.  Arrays use C order with shape
(nz, ny, nx), so the flat index is x + nx * (y + ny * z); vector fields carry
a leading axis of 3.

Random numbers come from a counter-based generator: SplitMix64 (Steele, Lea
and Flood, OOPSLA 2014) applied to the global cell coordinates and a seed,
so that a crop of a large medium equals the medium generated for the crop.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

PERIODIC, WALL, RESERVOIR = 0, 1, 2
SINGLE, MISCIBLE, IMMISCIBLE, FREESURF = 0, 1, 2, 3
PHYSICS_NAMES = {"single": SINGLE, "miscible": MISCIBLE, "immiscible": IMMISCIBLE,
                 "freesurface": FREESURF}


@dataclasses.dataclass
class Face:
    kind: int = PERIODIC
    rho: float = 1.0        # reservoir density
    conc: float = 0.0       # reservoir concentration
    angle: float = 90.0     # wall contact angle in degrees (two-fluid model)
    conc_x: Tuple[float, ...] = ()   # reservoir concentrations of solutes 2, 3, ...


@dataclasses.dataclass
class Problem:
    """Everything needed to set up one lattice: sizes, physics, parameters,
    boundary faces (-x,+x,-y,+y,-z,+z) and the initial / medium fields."""
    shape: Tuple[int, int, int]                 # (nx, ny, nz)
    physics: int = SINGLE
    G: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    forchheimer: bool = False
    eps_grad: bool = True
    # viscosity law nu = nu0 * min(a0 + a1 exp(alpha t), cap) * exp(k1 C + k0)
    nu0: float = 0.1
    a0: float = 1.0
    a1: float = 0.0
    alpha: float = 0.0
    cap: float = 1e30
    k1: float = 0.0
    k0: float = 0.0
    tau1: float = 0.7       # two-fluid: fluid 1 (the one carried by the second lattice)
    tau2: float = 1.0       # two-fluid: fluid 2
    tau_d: float = 0.65     # solute relaxation time
    A: float = 0.0          # surface-tension strength
    beta: float = 0.7       # recolouring strength
    faces: List[Face] = dataclasses.field(default_factory=lambda: [Face() for _ in range(6)])
    eps: Optional[np.ndarray] = None    # (nz,ny,nx)
    kinv: Optional[np.ndarray] = None   # (3,nz,ny,nx) diagonal, or (6,nz,ny,nx) full {xx,yy,zz,xy,xz,yz}
    rho0: Optional[np.ndarray] = None   # (nz,ny,nx)
    vel0: Optional[np.ndarray] = None   # (3,nz,ny,nx)
    c0: Optional[np.ndarray] = None     # (nz,ny,nx); free surface: initial fill fraction
    solid: Optional[np.ndarray] = None  # (nz,ny,nx) nonzero = obstacle cell (no state, bounce-back)
    solid_angle: float = 90.0           # contact angle of the obstacle surfaces (two-fluid model)
    species_tau_d: Tuple[float, ...] = ()   # miscible: relaxation times of solutes 2, 3, ... (c0 then
                                            # holds one plane per solute: (nspecies, nz, ny, nx))

    @property
    def ncell(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def fill_defaults(self) -> "Problem":
        nx, ny, nz = self.shape
        if self.eps is None:
            self.eps = np.ones((nz, ny, nx))
        if self.kinv is None:
            self.kinv = np.zeros((3, nz, ny, nx))
        if self.rho0 is None:
            self.rho0 = np.ones((nz, ny, nx))
        if self.vel0 is None:
            self.vel0 = np.zeros((3, nz, ny, nx))
        if self.c0 is None:
            self.c0 = np.zeros((nz, ny, nx)) if self.nspecies == 1 else np.zeros((self.nspecies, nz, ny, nx))
        return self

    def uniform_medium(self) -> bool:
        e = self.eps
        k = self.kinv
        return bool(np.all(e == e.flat[0]) and all(np.all(k[a] == k[a].flat[0]) for a in range(k.shape[0])))

    @property
    def nspecies(self) -> int:
        return 1 + len(self.species_tau_d)

    @property
    def full_tensor(self) -> bool:
        return self.kinv is not None and np.asarray(self.kinv).shape[0] == 6


# --------------------------------------------------------------------------
# counter-based random numbers

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied to uint64 counters (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = (x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def cell_uniform(seed: int, x: np.ndarray, y: np.ndarray, z: np.ndarray, stream: int) -> np.ndarray:
    """Uniform variate in (0,1) for global cell (x,y,z), a seed and a stream id."""
    c = (x.astype(np.uint64) | (y.astype(np.uint64) << np.uint64(20))
         | (z.astype(np.uint64) << np.uint64(40)) | (np.uint64(stream & 0xF) << np.uint64(60)))
    k = splitmix64(np.asarray([seed], dtype=np.uint64))[0]
    h = splitmix64(splitmix64(c) ^ k)
    return ((h >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def cell_normal(seed: int, x, y, z) -> np.ndarray:
    """Standard normal variate per global cell (Box-Muller on two streams)."""
    u1 = cell_uniform(seed, x, y, z, 0)
    u2 = cell_uniform(seed, x, y, z, 1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


# --------------------------------------------------------------------------
# media

def kappa(eps):
    """Porosity dependence of the wood permeability tensor: with
    rho/rho_max = 1 - eps the prefactor (rho_max/rho)^2 eps^(11/3) of Eq. Ktensor
    becomes eps^(11/3) / (1 - eps)^2."""
    return eps ** (11.0 / 3.0) / (1.0 - eps) ** 2


def spruce_medium(shape, seed: int = 0, ratio: float = 100.0, origin=(0, 0, 0),
                  eps_lo: float = 0.4, eps_hi: float = 0.8, period: float = 32.0,
                  k_ref: float = 1e-2, sigma: float = 0.3):
    """Spruce-like banded medium.  x is the radial (ring) axis, y longitudinal,
    z tangential (the (r, z, theta) frame of Eq. Ktensor).  Porosity varies
    sinusoidally between eps_lo and eps_hi along x with the ring period;
    the diagonal permeability is K_ref * kappa(eps)/kappa(eps_mid) *
    exp(sigma xi) * (1/ratio, 1, 1/ratio) with one seeded standard normal xi per
    cell.  `origin` is the global coordinate of the crop's first cell.
    Returns (eps (nz,ny,nx), kinv (3,nz,ny,nx)) in float64."""
    nx, ny, nz = shape
    ox, oy, oz = origin
    x = np.arange(nx, dtype=np.int64) + ox
    y = np.arange(ny, dtype=np.int64) + oy
    z = np.arange(nz, dtype=np.int64) + oz
    mid = 0.5 * (eps_lo + eps_hi)
    amp = 0.5 * (eps_hi - eps_lo)
    eps_x = mid + amp * np.sin(2.0 * math.pi * x / period)
    eps = np.broadcast_to(eps_x[None, None, :], (nz, ny, nx)).copy()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    xi = cell_normal(seed, X, Y, Z)
    kl = k_ref * kappa(eps) / kappa(mid) * np.exp(sigma * xi)
    kinv = np.empty((3, nz, ny, nx))
    kinv[0] = ratio / kl
    kinv[1] = 1.0 / kl
    kinv[2] = ratio / kl
    return eps, kinv


def inclined_spruce_medium(shape, seed: int = 0, ratio: float = 100.0, angle_deg: float = 45.0,
                           origin=(0, 0, 0), eps_lo: float = 0.4, eps_hi: float = 0.8,
                           period: float = 32.0, k_ref: float = 1e-2, sigma: float = 0.3):
    """The spruce-like medium with its annual rings inclined by `angle_deg` in
    the x-y plane (the rotated permeability of Eq. Ktensor): radial axis
    n = (cos a, sin a, 0), longitudinal axis l = (-sin a, cos a, 0),
    tangential axis z.  Porosity follows the ring coordinate r = n.x (global
    cell coordinates); K = K_L (n n^T / R + l l^T + z z^T / R) with
    K_L = K_ref kappa(eps)/kappa(eps_mid) exp(sigma xi), so
    K^-1 = (R n n^T + l l^T + R z z^T) / K_L.  At angle 0 this is
    `spruce_medium` written as a full tensor.  Returns (eps (nz,ny,nx),
    kinv (6,nz,ny,nx) = {xx, yy, zz, xy, xz, yz}) in float64."""
    nx, ny, nz = shape
    ox, oy, oz = origin
    a = math.radians(angle_deg)
    c, sn = math.cos(a), math.sin(a)
    Z, Y, X = np.meshgrid(np.arange(nz, dtype=np.int64) + oz, np.arange(ny, dtype=np.int64) + oy,
                          np.arange(nx, dtype=np.int64) + ox, indexing="ij")
    r = c * X + sn * Y
    mid = 0.5 * (eps_lo + eps_hi)
    amp = 0.5 * (eps_hi - eps_lo)
    eps = mid + amp * np.sin(2.0 * math.pi * r / period)
    xi = cell_normal(seed, X, Y, Z)
    kl = k_ref * kappa(eps) / kappa(mid) * np.exp(sigma * xi)
    ikl = 1.0 / kl
    kinv = np.empty((6, nz, ny, nx))
    kinv[0] = ratio * ikl * (c * c) + ikl * (sn * sn)
    kinv[1] = ratio * ikl * (sn * sn) + ikl * (c * c)
    kinv[2] = ratio * ikl
    kinv[3] = (ratio - 1.0) * ikl * (c * sn)
    kinv[4] = 0.0
    kinv[5] = 0.0
    return eps, kinv


# Spruce wood of Sec. 5.5 (wood-properties paragraph): density law of Eq.
# wooddensityfunc with rho_0 = 310 kg/m^3, a = 24/Delta, b = 0.8, c = 9.6/Delta,
# ring width Delta = 2.9 mm (positions in mm); permeabilities of Eq. Ktensor in
# mm^2 along the radial, longitudinal and tangential axes.  The cell-wall density
# rho_max is not printed: 1500 kg/m^3, the usual value for the wood substance.
SPRUCE_RHO0 = 310.0
SPRUCE_RING_MM = 2.9
SPRUCE_B = 0.8
SPRUCE_A = 24.0 / SPRUCE_RING_MM
SPRUCE_C = 9.6 / SPRUCE_RING_MM
WOOD_RHO_MAX = 1500.0
WOOD_K_MM2 = (8.2e-10, 51470e-10, 0.82e-10)   # radial, longitudinal, tangential


def wood_density(s_mm):
    """Eq. wooddensityfunc made periodic over the year rings: rho(s) = rho_0
    [1 + 2 a x^b exp(-c x)] with x = s mod Delta, the position in the ring (mm)."""
    x = np.mod(np.asarray(s_mm, dtype=np.float64), SPRUCE_RING_MM)
    return SPRUCE_RHO0 * (1.0 + 2.0 * SPRUCE_A * x ** SPRUCE_B * np.exp(-SPRUCE_C * x))


def wood_medium(shape, angle_deg: float = 45.0, ring_cells: float = 30.0, rho_max: float = WOOD_RHO_MAX,
                origin=(0, 0, 0)):
    """The spruce medium of Sec. 5.5 built from the paper's laws: the x-y plane is
    the wood cross-section (radial-tangential), the year rings inclined by
    `angle_deg` in it (radial axis n = (cos a, sin a, 0), tangential
    t = (-sin a, cos a, 0)), z the longitudinal (grain) axis; one ring is
    `ring_cells` cells wide (the ring distance of the penetration example), so a
    cell is Delta / ring_cells mm.  Per cell, at the ring coordinate
    s = n.(x, y, z) Delta / ring_cells: rho(s) by Eq. wooddensityfunc,
    eps = 1 - rho / rho_max (Eq. epsilonfunction), and the permeabilities of Eq.
    Ktensor, K_k = (rho_max / rho)^2 eps^(11/3) K_k^0 / dx^2 in lattice units, so
    K^-1 = n n^T / K_r + t t^T / K_t + z z^T / K_L.  Returns (eps (nz,ny,nx),
    kinv (6,nz,ny,nx) = {xx, yy, zz, xy, xz, yz}) in float64; crops agree with the
    full medium through `origin`."""
    nx, ny, nz = shape
    ox, oy, oz = origin
    a = math.radians(angle_deg)
    c, sn = math.cos(a), math.sin(a)
    Z, Y, X = np.meshgrid(np.arange(nz, dtype=np.int64) + oz, np.arange(ny, dtype=np.int64) + oy,
                          np.arange(nx, dtype=np.int64) + ox, indexing="ij")
    dx_mm = SPRUCE_RING_MM / ring_cells
    rho = wood_density((c * X + sn * Y) * dx_mm)
    eps = 1.0 - rho / rho_max
    pref = (rho_max / rho) ** 2 * eps ** (11.0 / 3.0) / (dx_mm * dx_mm)
    ikr = 1.0 / (pref * WOOD_K_MM2[0])
    ikl = 1.0 / (pref * WOOD_K_MM2[1])
    ikt = 1.0 / (pref * WOOD_K_MM2[2])
    kinv = np.empty((6, nz, ny, nx))
    kinv[0] = ikr * (c * c) + ikt * (sn * sn)
    kinv[1] = ikr * (sn * sn) + ikt * (c * c)
    kinv[2] = ikl
    kinv[3] = (ikr - ikt) * (c * sn)
    kinv[4] = 0.0
    kinv[5] = 0.0
    return eps, kinv


def wood_hardening_law(p: "Problem", alpha: float = 2e-3) -> "Problem":
    """Eq. nuall with the urea-formaldehyde constants of Sec. 5.5: nu_g = 0.15,
    a = 2.05e-9, beta = 1e-3; alpha is not printed: 2e-3 per step, so that the
    reaction term a exp(alpha t) reaches 1 (the viscosity doubles) after 1e4 steps."""
    beta = 1e-3
    p.nu0, p.a0, p.a1, p.alpha, p.cap, p.k1, p.k0 = 0.15, 1.0, 2.05e-9, alpha, 1e30, -beta, beta
    return p


# --------------------------------------------------------------------------
# problems shaped like the paper's workloads

def poiseuille(shape=(32, 32, 32), eps=0.7, K=1e-2, G=1e-6, tau=0.8, wall_axis=2,
               flow_axis=0, kdiag=None, forchheimer=False) -> Problem:
    """Body-force driven channel through a homogeneous porous medium between
    two no-slip walls (Sec. 5.1): solid planes at both ends of `wall_axis`,
    periodic elsewhere, constant viscosity nu = (tau - 1/2)/3."""
    nx, ny, nz = shape
    faces = [Face() for _ in range(6)]
    faces[2 * wall_axis] = Face(kind=WALL)
    faces[2 * wall_axis + 1] = Face(kind=WALL)
    g = [0.0, 0.0, 0.0]
    g[flow_axis] = G
    kd = kdiag if kdiag is not None else (K, K, K)
    kinv = np.empty((3, nz, ny, nx))
    for a in range(3):
        kinv[a] = 1.0 / kd[a]
    p = Problem(shape=tuple(shape), physics=SINGLE, G=tuple(g), forchheimer=forchheimer,
                nu0=(tau - 0.5) / 3.0, faces=faces,
                eps=np.full((nz, ny, nx), float(eps)), kinv=kinv)
    return p.fill_defaults()


def hardening_law(p: Problem) -> Problem:
    """nu = 0.1 exp(2 C) min(exp(1e-4 t), 10): the hardening law of the
    miscible workloads, a member of the Eq. nuall family."""
    p.nu0, p.a0, p.a1, p.alpha, p.cap, p.k1, p.k0 = 0.1, 0.0, 1.0, 1e-4, 10.0, 2.0, 0.0
    return p


P_EXT = 0.0441  # applied pressure of the penetration example, Sec. 5.5


def miscible(shape=(256, 256, 256), seed=0, ratio=100.0, origin=(0, 0, 0), D=0.05,
             p_ext=P_EXT, reservoirs=True, ring_angle=None) -> Problem:
    """Miscible mixture in the spruce-like medium: hydrodynamic lattice plus the
    solute lattice (diffusivity D), hardening viscosity, Darcy + Forchheimer
    drag, inlet reservoir at x = 0 with rho = 1 + 3 p_ext and C = 1, outlet
    reservoir at x = nx-1 with rho = 1 and C = 0, periodic in y and z.  With
    `ring_angle` (degrees) the rings are inclined and K^-1 is a full tensor."""
    nx, ny, nz = shape
    if ring_angle is None:
        eps, kinv = spruce_medium(shape, seed=seed, ratio=ratio, origin=origin)
    else:
        eps, kinv = inclined_spruce_medium(shape, seed=seed, ratio=ratio, angle_deg=ring_angle, origin=origin)
    faces = [Face() for _ in range(6)]
    if reservoirs:
        faces[0] = Face(kind=RESERVOIR, rho=1.0 + 3.0 * p_ext, conc=1.0)
        faces[1] = Face(kind=RESERVOIR, rho=1.0, conc=0.0)
    p = Problem(shape=tuple(shape), physics=MISCIBLE, forchheimer=True, tau_d=0.5 + 3.0 * D,
                faces=faces, eps=eps, kinv=kinv)
    hardening_law(p)
    return p.fill_defaults()


def miscible_parallel(n: int, seed: int = 0, slabs: int = 16, workers: int = 8) -> Problem:
    """The n^3 miscible workload (`miscible`) with its medium generated in
    z-slabs by a thread pool and held in float32: the counter-based generator
    makes every slab equal to the corresponding crop of the full medium, so
    the values are `miscible`'s rounded to float32 (what the FP32 and 16-bit
    storage modes take anyway).  For the 512^3 workloads, where the serial
    float64 generation takes half a minute and 10 GB."""
    from concurrent.futures import ThreadPoolExecutor
    p = miscible(shape=(n, n, 2), seed=seed)
    p.shape = (n, n, n)
    dz = (n + slabs - 1) // slabs
    parts = [(z0, min(dz, n - z0)) for z0 in range(0, n, dz)]
    eps = np.empty((n, n, n), dtype=np.float32)
    kinv = np.empty((3, n, n, n), dtype=np.float32)

    def gen(part):
        z0, nzp = part
        e, k = spruce_medium((n, n, nzp), seed=seed, ratio=100.0, origin=(0, 0, z0))
        eps[z0:z0 + nzp] = e
        kinv[:, z0:z0 + nzp] = k

    with ThreadPoolExecutor(workers) as pool:
        list(pool.map(gen, parts))
    p.eps, p.kinv = eps, kinv
    p.rho0 = np.ones((n, n, n), dtype=np.float32)
    p.vel0 = np.zeros((3, n, n, n), dtype=np.float32)
    p.c0 = np.zeros((n, n, n), dtype=np.float32)
    return p


def wood(shape=(256, 256, 256), angle_deg=45.0, D=0.05, p_ext=P_EXT, origin=(0, 0, 0)) -> Problem:
    """Miscible adhesive in the spruce medium of Sec. 5.5 (`wood_medium`, rings
    inclined by 45 degrees in the cross-section), driven along the grain: inlet
    reservoir at z = 0 with rho = 1 + 3 p_ext and C = 1, outlet at z = nz-1 with
    rho = 1 and C = 0, periodic in x and y; the hardening law of Eq. nuall with
    the paper's constants (`wood_hardening_law`), Darcy + Forchheimer drag."""
    eps, kinv = wood_medium(shape, angle_deg=angle_deg, origin=origin)
    faces = [Face() for _ in range(6)]
    faces[4] = Face(kind=RESERVOIR, rho=1.0 + 3.0 * p_ext, conc=1.0)
    faces[5] = Face(kind=RESERVOIR, rho=1.0, conc=0.0)
    p = Problem(shape=tuple(shape), physics=MISCIBLE, forchheimer=True, tau_d=0.5 + 3.0 * D,
                faces=faces, eps=eps, kinv=kinv)
    wood_hardening_law(p)
    return p.fill_defaults()


def drop(shape=(128, 128, 128), radius=20.0, centre=None, speed=0.05, tau1=0.7, tau2=1.0,
         A=0.01, beta=0.7, bottom_angle=120.0, top_angle=90.0, walls=True) -> Problem:
    """Two-fluid drop moving toward a hydrophobic plane (Sec. 5.3 set-up, two-fluid
    form): a sharp sphere of fluid 1 (C = 1) of the given radius, moving with
    velocity -speed along z, walls at z = 0 (bottom_angle) and z = nz-1
    (top_angle), periodic in x and y, no porous medium (eps = 1, K^-1 = 0)."""
    nx, ny, nz = shape
    if centre is None:
        centre = (nx // 2, ny // 2, nz // 2)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    inside = r2 <= radius * radius
    c0 = inside.astype(np.float64)
    vel0 = np.zeros((3, nz, ny, nx))
    vel0[2][inside] = -speed
    faces = [Face() for _ in range(6)]
    if walls:
        faces[4] = Face(kind=WALL, angle=bottom_angle)
        faces[5] = Face(kind=WALL, angle=top_angle)
    p = Problem(shape=tuple(shape), physics=IMMISCIBLE, tau1=tau1, tau2=tau2, A=A, beta=beta,
                faces=faces, c0=c0, vel0=vel0)
    return p.fill_defaults()


def falling_drop(shape=(140, 140, 1), radius=8.0, centre=None, G=1e-6, tau=0.7, axis=1,
                 wall=True, speed=0.0) -> Problem:
    """Free-surface drop falling onto an impermeable plane (Sec. 5.3): a liquid
    disc (quasi-2D when the third extent is 1) or sphere of the given radius
    in gas, gravity G toward -axis, a wall on the low face of that axis,
    every other face periodic; no porous medium (eps = 1, K^-1 = 0).  The
    fill fraction of a cell is its covered volume estimated on a 4^3
    subgrid, so the drop's initial liquid mass is close to pi R^2 (or
    4 pi R^3 / 3) for any centre.  The high face of the fall axis is a wall
    too (both faces of an axis are periodic or neither); the drop never
    reaches it."""
    nx, ny, nz = shape
    if centre is None:
        centre = [nx / 2.0, ny / 2.0, nz / 2.0]
        centre[axis] = shape[axis] / 2.0
        if shape[2] == 1:
            centre[2] = 0.0
    sub = (np.arange(4) + 0.5) / 4.0 - 0.5
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    frac = np.zeros((nz, ny, nx))
    flat = shape[2] == 1
    for a in sub:
        for b in sub:
            for c in ([0.0] if flat else sub):
                d2 = (x + a - centre[0]) ** 2 + (y + b - centre[1]) ** 2
                if not flat:
                    d2 = d2 + (z + c - centre[2]) ** 2
                frac += d2 <= radius * radius
    frac /= 16.0 if flat else 64.0
    g = [0.0, 0.0, 0.0]
    g[axis] = -G
    vel0 = np.zeros((3, nz, ny, nx))
    vel0[axis][frac > 0] = -speed
    faces = [Face() for _ in range(6)]
    if wall:
        faces[2 * axis] = Face(kind=WALL)
        faces[2 * axis + 1] = Face(kind=WALL)
    p = Problem(shape=tuple(shape), physics=FREESURF, G=tuple(g), nu0=(tau - 0.5) / 3.0,
                faces=faces, c0=frac, vel0=vel0)
    return p.fill_defaults()


def pool(shape=(6, 5, 40), depth=20.5, G=1e-4, tau=0.8) -> Problem:
    """Free-surface liquid pool at rest: liquid up to the height `depth`
    (the cell straddling it partly filled) above a wall at z = 0, gas above
    up to a wall at z = nz - 1, gravity G toward -z, periodic in x and y."""
    nx, ny, nz = shape
    zc = np.arange(nz, dtype=np.float64)[:, None, None] * np.ones((nz, ny, nx))
    # the wall cell z = 0 is solid; liquid fills from its face z = 0.5 upward
    c0 = np.clip(depth - (zc - 0.5), 0.0, 1.0)
    faces = [Face() for _ in range(6)]
    faces[4] = Face(kind=WALL)
    faces[5] = Face(kind=WALL)
    p = Problem(shape=tuple(shape), physics=FREESURF, G=(0.0, 0.0, -G), nu0=(tau - 0.5) / 3.0,
                faces=faces, c0=c0)
    return p.fill_defaults()


def penetration(shape=(256, 256, 256), seed=0, G=1e-4, k_ref=1.0, ratio=100.0, tau=0.8,
                ring_angle=None) -> Problem:
    """Liquid penetrating an unsaturated porous medium (the set-up of Sec. 5.5
    in 3D, without its unprinted parameters): the spruce-like medium fills
    the box, liquid fills the upper half y >= ny/2 and gas the pores below,
    gravity G toward -y (along the grain), walls on both y faces, periodic in
    x and z, Darcy + Forchheimer drag."""
    nx, ny, nz = shape
    if ring_angle is None:
        eps, kinv = spruce_medium(shape, seed=seed, ratio=ratio, k_ref=k_ref)
    else:
        eps, kinv = inclined_spruce_medium(shape, seed=seed, ratio=ratio, angle_deg=ring_angle, k_ref=k_ref)
    y = np.arange(ny)[None, :, None] * np.ones((nz, ny, nx))
    c0 = (y >= ny // 2).astype(np.float64)
    faces = [Face() for _ in range(6)]
    faces[2] = Face(kind=WALL)
    faces[3] = Face(kind=WALL)
    p = Problem(shape=tuple(shape), physics=FREESURF, G=(0.0, -G, 0.0), forchheimer=True,
                nu0=(tau - 0.5) / 3.0, faces=faces, eps=eps, kinv=kinv, c0=c0)
    return p.fill_defaults()


def slab(shape=(48, 4, 3), lo=8, hi=20, speed=0.05, tau=0.8) -> Problem:
    """Free-surface liquid slab lo <= x < hi moving with velocity `speed`
    along x through gas, periodic on every face, no force."""
    nx, ny, nz = shape
    x = np.arange(nx)[None, None, :] * np.ones((nz, ny, nx))
    c0 = ((x >= lo) & (x < hi)).astype(np.float64)
    vel0 = np.zeros((3, nz, ny, nx))
    vel0[0] = speed
    p = Problem(shape=tuple(shape), physics=FREESURF, nu0=(tau - 0.5) / 3.0, c0=c0, vel0=vel0)
    return p.fill_defaults()


def square(shape=(100, 100, 1), side=20, tau=0.7, A=0.001, beta=0.7) -> Problem:
    """The surface-smoothing set-up of Sec. 5.4 in the two-fluid model: a square
    (a cube when nz > 1) of fluid 1 with the given side at the box centre, both
    fluids at tau = 0.7 (the droplet's), surface-tension strength A, periodic
    box, no force and no porous medium."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inside = (np.abs(x - (nx - 1) / 2.0) < side / 2.0) & (np.abs(y - (ny - 1) / 2.0) < side / 2.0)
    if nz > 1:
        inside &= np.abs(z - (nz - 1) / 2.0) < side / 2.0
    p = Problem(shape=tuple(shape), physics=IMMISCIBLE, tau1=tau, tau2=tau, A=A, beta=beta,
                c0=inside.astype(np.float64))
    return p.fill_defaults()


def sphere_obstacles(shape, seed: int = 0, solid_fraction: float = 0.1, radius=(2.0, 4.0),
                     keep_planes=(0,)) -> np.ndarray:
    """Seeded obstacle mask: spheres with radii uniform in `radius` and centres
    uniform in the box (distances wrap on every axis), added until the solid
    fraction reaches `solid_fraction`.  The planes x = i for i in
    `keep_planes` (and x = nx-1-i) stay free so that reservoir faces on x keep
    a fluid layer next to them.  Returns uint8 (nz,ny,nx)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mask = np.zeros((nz, ny, nx), dtype=bool)
    ncell = nx * ny * nz
    while mask.sum() < solid_fraction * ncell:
        c = rng.random(3) * np.array([nx, ny, nz])
        r = rng.uniform(*radius)
        d = [np.abs(a - ca) for a, ca in zip((x, y, z), c)]
        d = [np.minimum(da, n - da) for da, n in zip(d, (nx, ny, nz))]
        mask |= d[0] ** 2 + d[1] ** 2 + d[2] ** 2 <= r * r
    for i in keep_planes:
        for xi in sorted({i, 1 + i, nx - 1 - i, nx - 2 - i}):
            if 0 <= xi < nx:
                mask[:, :, xi] = False
    return mask.astype(np.uint8)


def block_obstacles(shape, seed: int = 0, solid_fraction: float = 0.1, block: int = 4, origin=(0, 0, 0),
                    free_x=2) -> np.ndarray:
    """Seeded obstacle mask of solid cubes: the box is tiled by block^3
    cubes (in global coordinates) and each cube is solid with probability
    `solid_fraction`, from the counter-based generator on the cube's
    coordinates (so crops agree with the full mask).  The `free_x` planes at
    each end of x stay fluid (room for reservoir faces).  Returns uint8
    (nz,ny,nx)."""
    nx, ny, nz = shape
    ox, oy, oz = origin
    x = (np.arange(nx, dtype=np.int64) + ox) // block
    y = (np.arange(ny, dtype=np.int64) + oy) // block
    z = (np.arange(nz, dtype=np.int64) + oz) // block
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    mask = cell_uniform(seed, X, Y, Z, 2) < solid_fraction
    if free_x:
        mask[:, :, :free_x] = False
        mask[:, :, nx - free_x:] = False
    return mask.astype(np.uint8)


def duct(shape=(4, 20, 20), G=1e-6, tau=0.8) -> Problem:
    """Body-force driven flow along x through a square duct made of obstacle
    cells: the y and z edge layers of the box are solid, every face is
    periodic, free fluid inside (eps = 1, K^-1 = 0)."""
    nx, ny, nz = shape
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    solid[:, [0, ny - 1], :] = 1
    solid[[0, nz - 1], :, :] = 1
    p = Problem(shape=tuple(shape), physics=SINGLE, G=(G, 0.0, 0.0), nu0=(tau - 0.5) / 3.0,
                solid=solid)
    return p.fill_defaults()


# --------------------------------------------------------------------------
# serving workload: a stream of solve requests

@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    edge: int               # cubic domain edge
    physics: int
    steps: int
    ratio: float
    seed: int


def request_stream(n=64, rate=4.0, edge_lo=48, edge_hi=192, p_miscible=0.7,
                   steps_lo=500, steps_hi=5000, ratio_lo=10.0, ratio_hi=200.0,
                   arrival_seed=1, param_seed=2, medium_seed0=1000) -> List[Request]:
    """Poisson arrivals at `rate` per second; edge log-uniform in
    [edge_lo, edge_hi]; physics miscible with probability p_miscible, else
    two-fluid; steps uniform in [steps_lo, steps_hi]; anisotropy ratio uniform
    in [ratio_lo, ratio_hi]."""
    ra = np.random.default_rng(arrival_seed)
    rp = np.random.default_rng(param_seed)
    t = np.cumsum(ra.exponential(1.0 / rate, size=n))
    out = []
    for i in range(n):
        u = rp.random()
        edge = int(round(edge_lo * (edge_hi / edge_lo) ** u))
        phys = MISCIBLE if rp.random() < p_miscible else IMMISCIBLE
        steps = int(rp.integers(steps_lo, steps_hi + 1))
        ratio = float(rp.uniform(ratio_lo, ratio_hi))
        out.append(Request(rid=i, arrival=float(t[i]), edge=edge, physics=phys, steps=steps,
                           ratio=ratio, seed=medium_seed0 + i))
    return out


def request_problem(req: Request) -> Problem:
    """The lattice a serving request asks for: the miscible workload at its
    edge and anisotropy, or a drop of radius 20 N / 128 in that request's
    medium."""
    n = req.edge
    if req.physics == MISCIBLE:
        return miscible((n, n, n), seed=req.seed, ratio=req.ratio)
    p = drop((n, n, n), radius=round(20.0 * n / 128.0))
    eps, kinv = spruce_medium((n, n, n), seed=req.seed, ratio=req.ratio)
    p.eps, p.kinv = eps, kinv
    return p
