"""ctypes front end of the FP64 CPU oracle (oracle/lbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product package.  It
shares no code with the GPU library; both are fed the same `Problem`
description from the seeded input module.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")
NQ = 19

_lib = None


class OrcParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("physics", C.c_int), ("forchheimer", C.c_int), ("eps_grad", C.c_int),
        ("G", C.c_double * 3),
        ("nu0", C.c_double), ("a0", C.c_double), ("a1", C.c_double), ("alpha", C.c_double),
        ("cap", C.c_double), ("k1", C.c_double), ("k0", C.c_double),
        ("tau1", C.c_double), ("tau2", C.c_double), ("tau_d", C.c_double),
        ("A", C.c_double), ("beta", C.c_double),
        ("face_kind", C.c_int * 6),
        ("face_rho", C.c_double * 6), ("face_conc", C.c_double * 6), ("face_angle", C.c_double * 6),
        ("solid_angle", C.c_double),
        ("full_tensor", C.c_int),
        ("nspecies", C.c_int),
        ("tau_dx", C.c_double * 3),
        ("face_concx", (C.c_double * 6) * 3),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build_oracle
            build_oracle.build()
        _lib = _load(LIB_PATH)
    return _lib


@contextlib.contextmanager
def library(path: str):
    """Run the oracle from another build of lbm_oracle.c (for example a copy
    with a planted mistake, to show that a pin fails on it) inside the block."""
    global _lib
    saved = lib()
    _lib = _load(path)
    try:
        yield _lib
    finally:
        _lib = saved


def _load(path: str):
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.POINTER(OrcParams), dp, dp, dp, dp, dp, C.POINTER(C.c_ubyte)]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_step.argtypes = [C.c_void_p, C.c_int]
    L.orc_step.restype = C.c_int
    L.orc_steps_done.argtypes = [C.c_void_p]
    L.orc_steps_done.restype = C.c_long
    L.orc_moments.argtypes = [C.c_void_p, dp, dp, dp]
    L.orc_diag.argtypes = [C.c_void_p, dp]
    L.orc_get_state.argtypes = [C.c_void_p, C.c_int, dp]
    L.orc_set_state.argtypes = [C.c_void_p, C.c_int, dp, C.c_long]
    L.orc_step_cells.argtypes = [C.c_void_p, C.c_long, C.POINTER(C.c_long), dp, dp, dp]
    L.orc_cell_types.argtypes = [C.c_void_p, C.POINTER(C.c_ubyte)]
    L.orc_lattice.argtypes = [C.POINTER(C.c_int), dp, C.POINTER(C.c_int)]
    L.orc_feq.argtypes = [C.c_double, dp, C.c_double, C.c_double, C.c_double, dp, dp]
    L.orc_force.argtypes = [C.c_double, dp, C.c_double, C.c_double, dp, dp]
    L.orc_heq.argtypes = [C.c_double, dp, dp]
    L.orc_viscosity.argtypes = [C.POINTER(OrcParams), C.c_double, C.c_double]
    L.orc_viscosity.restype = C.c_double
    L.orc_solve_speed.argtypes = [dp, dp, dp]
    L.orc_solve_speed.restype = C.c_double
    L.orc_porous_velocity.argtypes = [C.POINTER(OrcParams), C.c_double, dp, C.c_double, dp, dp, dp]
    L.orc_porous_velocity_full.argtypes = [C.POINTER(OrcParams), C.c_double, dp, C.c_double, dp, dp, dp]
    L.orc_sym_sqrt.argtypes = [dp, dp]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_fs_state.argtypes = [C.c_void_p, C.POINTER(C.c_ubyte), dp]
    L.orc_fs_state.restype = C.c_double
    L.orc_species_conc.argtypes = [C.c_void_p, C.c_int, dp]
    L.orc_species_conc.restype = C.c_int
    L.orc_species_totals.argtypes = [C.c_void_p, dp]
    L.orc_species_totals.restype = C.c_int
    L.orc_fs_set_state.argtypes = [C.c_void_p, C.POINTER(C.c_ubyte), dp, dp]
    L.orc_fs_set_state.restype = C.c_int
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64))


def params_from_problem(p) -> OrcParams:
    nx, ny, nz = p.shape
    o = OrcParams()
    o.nx, o.ny, o.nz = nx, ny, nz
    o.physics = int(p.physics)
    o.forchheimer = int(bool(p.forchheimer))
    o.eps_grad = int(bool(p.eps_grad))
    o.G = (C.c_double * 3)(*[float(g) for g in p.G])
    o.nu0, o.a0, o.a1, o.alpha, o.cap, o.k1, o.k0 = (float(p.nu0), float(p.a0), float(p.a1),
                                                      float(p.alpha), float(p.cap), float(p.k1), float(p.k0))
    o.tau1, o.tau2, o.tau_d = float(p.tau1), float(p.tau2), float(p.tau_d)
    o.A, o.beta = float(p.A), float(p.beta)
    o.face_kind = (C.c_int * 6)(*[int(f.kind) for f in p.faces])
    o.face_rho = (C.c_double * 6)(*[float(f.rho) for f in p.faces])
    o.face_conc = (C.c_double * 6)(*[float(f.conc) for f in p.faces])
    o.face_angle = (C.c_double * 6)(*[float(f.angle) for f in p.faces])
    o.solid_angle = float(p.solid_angle)
    o.full_tensor = int(p.kinv is not None and np.asarray(p.kinv).shape[0] == 6)
    o.nspecies = int(p.nspecies)
    for k, t in enumerate(p.species_tau_d):
        o.tau_dx[k] = float(t)
        for f in range(6):
            o.face_concx[k][f] = float(p.faces[f].conc_x[k]) if len(p.faces[f].conc_x) > k else 0.0
    return o


def lattice():
    """(velocities (19,3) int, weights (19,), opposite (19,)) in the oracle's order."""
    v = (C.c_int * (3 * NQ))()
    w = np.zeros(NQ)
    o = (C.c_int * NQ)()
    lib().orc_lattice(v, _dp(w), o)
    return np.array(v[:], dtype=np.int64).reshape(NQ, 3), w, np.array(o[:], dtype=np.int64)


def feq(rho, u, eps, tau, A, F):
    out = np.zeros(NQ)
    lib().orc_feq(float(rho), _dp(_vec(u)), float(eps), float(tau), float(A), _dp(_vec(F)), _dp(out))
    return out


def force(rho, u, eps, tau, Fext):
    out = np.zeros(NQ)
    lib().orc_force(float(rho), _dp(_vec(u)), float(eps), float(tau), _dp(_vec(Fext)), _dp(out))
    return out


def heq(epsC, vstar):
    out = np.zeros(NQ)
    lib().orc_heq(float(epsC), _dp(_vec(vstar)), _dp(out))
    return out


def solve_speed(W, lam, mu):
    return lib().orc_solve_speed(_dp(_vec(W)), _dp(_vec(lam)), _dp(_vec(mu)))


def viscosity(problem, C_, t):
    prm = params_from_problem(problem)
    return lib().orc_viscosity(C.byref(prm), float(C_), float(t))


def porous_velocity(problem, eps, kinv, nu, V):
    """(V', F^ext) of one cell; kinv has 3 (diagonal) or 6 ({xx,yy,zz,xy,xz,yz})
    components."""
    prm = params_from_problem(problem)
    Vp = np.zeros(3)
    Fx = np.zeros(3)
    k = _vec(kinv)
    fn = lib().orc_porous_velocity_full if k.size == 6 else lib().orc_porous_velocity
    fn(C.byref(prm), float(eps), _dp(k), float(nu), _dp(_vec(V)), _dp(Vp), _dp(Fx))
    return Vp, Fx


def set_threads(n: int):
    """OpenMP threads of the oracle's following calls from this thread."""
    lib().orc_set_threads(int(n))


def sym_sqrt(k6):
    """The oracle's K^-1/2 of a symmetric tensor {xx,yy,zz,xy,xz,yz}."""
    out = np.zeros(6)
    lib().orc_sym_sqrt(_dp(_vec(k6)), _dp(out))
    return out


class Oracle:
    """Stateful FP64 simulation of one lattice."""

    def __init__(self, problem):
        p = problem.fill_defaults()
        self.problem = p
        self.shape = p.shape
        nx, ny, nz = p.shape
        self.n = nx * ny * nz
        self._keep = [_vec(p.eps).reshape(-1), _vec(p.kinv).reshape(-1), _vec(p.rho0).reshape(-1),
                      _vec(p.vel0).reshape(-1), _vec(p.c0).reshape(-1)]
        self.params = params_from_problem(p)
        solid = None
        if p.solid is not None:
            solid = np.ascontiguousarray(np.asarray(p.solid).reshape(-1) != 0, dtype=np.uint8)
        sp = solid.ctypes.data_as(C.POINTER(C.c_ubyte)) if solid is not None else None
        h = lib().orc_create(C.byref(self.params), *[_dp(a) for a in self._keep], sp)
        if not h:
            raise MemoryError("oracle allocation failed (or a reservoir face with the free surface)")
        self.h = C.c_void_p(h)
        self._keep = None

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int):
        if lib().orc_step(self.h, int(n)) != 0:
            raise MemoryError("oracle allocation failed")
        return self

    @property
    def steps_done(self) -> int:
        return int(lib().orc_steps_done(self.h))

    def moments(self):
        """(rho (nz,ny,nx), V' (3,nz,ny,nx), C (nz,ny,nx)) of the last step."""
        nx, ny, nz = self.shape
        rho = np.zeros(self.n)
        vel = np.zeros(3 * self.n)
        c = np.zeros(self.n)
        lib().orc_moments(self.h, _dp(rho), _dp(vel), _dp(c))
        return rho.reshape(nz, ny, nx), vel.reshape(3, nz, ny, nx), c.reshape(nz, ny, nx)

    def diag(self):
        out = np.zeros(8)
        lib().orc_diag(self.h, _dp(out))
        return out

    def cell_types(self):
        nx, ny, nz = self.shape
        out = (C.c_ubyte * self.n)()
        lib().orc_cell_types(self.h, out)
        return np.frombuffer(out, dtype=np.uint8).copy().reshape(nz, ny, nx)

    def fs_state(self):
        """Free surface: (cell class (nz,ny,nx) 0 gas / 1 interface / 2 liquid,
        liquid mass m (nz,ny,nx), excess mass lost so far)."""
        nx, ny, nz = self.shape
        cls = (C.c_ubyte * self.n)()
        m = np.zeros(self.n)
        lost = lib().orc_fs_state(self.h, cls, _dp(m))
        return (np.frombuffer(cls, dtype=np.uint8).copy().reshape(nz, ny, nx),
                m.reshape(nz, ny, nx), lost)

    def fs_set_state(self, cls, mass, lam):
        """Free surface: replace the classes (0 gas, 1 interface, 2 liquid),
        liquid masses and fill fractions of the current state (arrays of
        ncell values; the populations are replaced with set_state)."""
        c = np.ascontiguousarray(np.asarray(cls).reshape(-1), dtype=np.uint8)
        m = _vec(mass).reshape(-1)
        lm = _vec(lam).reshape(-1)
        assert c.size == m.size == lm.size == self.n
        if lib().orc_fs_set_state(self.h, c.ctypes.data_as(C.POINTER(C.c_ubyte)), _dp(m), _dp(lm)) != 0:
            raise ValueError("not a free-surface problem")

    def species_conc(self, k: int):
        """Concentration of solute k (0: the first) of the last step, (nz,ny,nx)."""
        nx, ny, nz = self.shape
        out = np.zeros(self.n)
        if lib().orc_species_conc(self.h, int(k), _dp(out)) != 0:
            raise IndexError(k)
        return out.reshape(nz, ny, nx)

    def species_totals(self):
        """Sum over fluid cells of eps C_k for every solute."""
        out = np.zeros(4)
        ns = lib().orc_species_totals(self.h, _dp(out))
        return out[:ns]

    def get_state(self, lattice_id: int):
        out = np.zeros(NQ * self.n)
        lib().orc_get_state(self.h, int(lattice_id), _dp(out))
        return out.reshape(NQ, self.n)

    def set_state(self, lattice_id: int, data: np.ndarray, step: int):
        a = _vec(data).reshape(-1)
        assert a.size == NQ * self.n
        lib().orc_set_state(self.h, int(lattice_id), _dp(a), int(step))

    def step_cells(self, cells):
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
        k = cells.size
        fo = np.zeros(k * NQ)
        ho = np.zeros(k * NQ)
        mo = np.zeros(k * 5)
        lib().orc_step_cells(self.h, k, cells.ctypes.data_as(C.POINTER(C.c_long)), _dp(fo), _dp(ho), _dp(mo))
        return fo.reshape(k, NQ), ho.reshape(k, NQ), mo.reshape(k, 5)
