"""Simulation: one lattice on the GPU, with its workspace in a torch tensor.

Thin convenience layer over the C ABI (binding.py): PyTorch provides the
device memory and the stream; every step of the update runs in the HIP
kernels of libporolbm.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import binding as B
from . import inputs as I


def make_desc(p: I.Problem, storage: int = B.LBM_F32, diag_every: int = 0) -> B.lbm_desc:
    d = B.lbm_desc()
    d.nx, d.ny, d.nz = (int(v) for v in p.shape)
    d.physics = int(p.physics)
    d.storage = int(storage)
    d.forchheimer = int(bool(p.forchheimer))
    d.eps_gradient = int(bool(p.eps_grad))
    d.G = (C.c_double * 3)(*[float(g) for g in p.G])
    d.nu0, d.a0, d.a1, d.alpha = float(p.nu0), float(p.a0), float(p.a1), float(p.alpha)
    d.cap, d.k1, d.k0 = float(p.cap), float(p.k1), float(p.k0)
    d.tau1, d.tau2, d.tau_d = float(p.tau1), float(p.tau2), float(p.tau_d)
    d.A, d.beta = float(p.A), float(p.beta)
    for f in range(6):
        F = p.faces[f]
        d.face[f].kind = int(F.kind)
        d.face[f].rho = float(F.rho)
        d.face[f].conc = float(F.conc)
        d.face[f].contact_angle_deg = float(F.angle)
    d.diag_every = int(diag_every)
    d.solid_mask = int(p.solid is not None)
    d.solid_contact_angle_deg = float(p.solid_angle)
    d.full_tensor = int(p.full_tensor)
    d.nspecies = int(p.nspecies)
    for k, t in enumerate(p.species_tau_d):
        d.tau_d_x[k] = float(t)
        for f in range(6):
            cx = p.faces[f].conc_x
            d.face_conc_x[k][f] = float(cx[k]) if len(cx) > k else 0.0
    return d


def check_fields(p: I.Problem) -> None:
    """The per-cell arrays of a problem have the shapes the kernels read
    (lbm_set_medium takes device pointers without sizes, so a short array
    would be read past its end): eps (nz,ny,nx); K^-1 3 planes, or 6 for a
    full tensor; rho0 (nz,ny,nx); V0 3 planes; c0 one plane, or one per solute
    in the miscible model with several solutes; the obstacle mask (nz,ny,nx).
    Raises ValueError."""
    nx, ny, nz = (int(v) for v in p.shape)
    cell = (nz, ny, nx)
    ns = p.nspecies if p.physics == I.MISCIBLE else 1
    want = {"eps": cell, "kinv": ((6 if p.full_tensor else 3),) + cell, "rho0": cell, "vel0": (3,) + cell,
            "c0": cell if ns == 1 else (ns,) + cell}
    if p.solid is not None:
        want["solid"] = cell
    for name, shape in want.items():
        a = getattr(p, name)
        if a is None or tuple(np.shape(a)) != shape:
            raise ValueError(f"{name}: shape {None if a is None else tuple(np.shape(a))}, expected {shape}")


def real_dtype(storage: int):
    import torch
    return torch.float64 if storage == B.LBM_F64 else torch.float32


class Simulation:
    """One lattice resident on a GPU.

    problem: a seeded `inputs.Problem`; storage: LBM_F64 / F32 / BF16_DEV /
    F16_DEV (or "f64", "f32", "bf16", "f16"); stream: a torch.cuda.Stream
    (default: the current stream of the device).
    """

    def __init__(self, problem: I.Problem, storage=B.LBM_F32, device="cuda:0", stream=None,
                 diag_every: int = 0, uniform_medium: bool = True, static_workspace: bool = False):
        import torch
        if isinstance(storage, str):
            storage = B.STORAGE_NAMES[storage]
        p = problem.fill_defaults()
        check_fields(p)
        self.problem = p
        self.storage = storage
        self.device = torch.device(device)
        self.dtype = real_dtype(storage)
        self.desc = make_desc(p, storage, diag_every)
        nbytes = B.lbm_workspace_bytes(self.desc)
        if nbytes == 0:
            raise B.LbmError(B.LBM_EINVAL, "lbm_workspace_bytes")
        self.nbytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.shape = tuple(p.shape)
        # the workspace, the uploads of the fields and the set-up all run on
        # the lattice's stream (work on other streams is not waited for)
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            if static_workspace:
                # the library's own static workspace of this device (lbm_create_static)
                self.ws = None
                self.h = B.lbm_create_static(self.desc, self.stream.cuda_stream)
            else:
                self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                self.h = B.lbm_create(self.desc, self.ws.data_ptr(), nbytes, self.stream.cuda_stream)
            self._set_medium(p, uniform_medium)

    # ------------------------------------------------------------------
    def _dev(self, a):
        import torch
        a = np.ascontiguousarray(a)
        if a.dtype not in (np.float32, np.float64):
            a = a.astype(np.float64)
        return torch.from_numpy(a).to(self.device, self.dtype)

    def _set_medium(self, p: I.Problem, uniform_medium: bool):
        import torch
        m = B.lbm_medium()
        keep = []
        eps_u = bool(uniform_medium and np.all(p.eps == p.eps.flat[0]))
        kinv_u = bool(uniform_medium and not p.full_tensor and
                      all(np.all(p.kinv[a] == p.kinv[a].flat[0]) for a in range(3)))
        if eps_u:
            m.eps = None
            m.eps_uniform = float(p.eps.flat[0])
        else:
            t = self._dev(p.eps)
            keep.append(t)
            m.eps = t.data_ptr()
        if kinv_u:
            m.kinv = None
            m.kinv_uniform = (C.c_double * 3)(*[float(p.kinv[a].flat[0]) for a in range(3)])
        else:
            t = self._dev(p.kinv)
            keep.append(t)
            m.kinv = t.data_ptr()
        for name, arr in (("rho0", p.rho0), ("vel0", p.vel0), ("c0", p.c0)):
            t = self._dev(arr)
            keep.append(t)
            setattr(m, name, t.data_ptr())
        if p.solid is not None:
            t = torch.from_numpy(np.ascontiguousarray(np.asarray(p.solid) != 0, dtype=np.uint8)).to(self.device)
            keep.append(t)
            m.solid = t.data_ptr()
        B.lbm_set_medium(self.h, m)    # synchronises the lattice's stream
        del keep

    def set_stream(self, stream) -> "Simulation":
        """Issue the lattice's later work on `stream` (lbm_set_stream); the
        caller orders it after the work already issued on the old stream."""
        B.lbm_set_stream(self.h, stream.cuda_stream)
        if self.ws is not None:
            self.ws.record_stream(stream)
        self.stream = stream
        return self

    def step(self, n: int = 1) -> "Simulation":
        B.lbm_step(self.h, n)
        return self

    @property
    def steps_done(self) -> int:
        return B.lbm_steps_done(self.h)

    def moments(self, check: bool = True):
        """(rho, V' (3,...), C) as device tensors shaped (nz,ny,nx), and the FP64
        diagnostics as a numpy array of 8."""
        import torch
        nx, ny, nz = self.shape
        with torch.cuda.stream(self.stream):
            rho = torch.empty((nz, ny, nx), dtype=self.dtype, device=self.device)
            vel = torch.empty((3, nz, ny, nx), dtype=self.dtype, device=self.device)
            ns = self.problem.nspecies if self.problem.physics == I.MISCIBLE else 1
            conc = torch.empty(((ns,) if ns > 1 else ()) + (nz, ny, nx), dtype=self.dtype, device=self.device)
        diag = (C.c_double * 8)()
        B.lbm_moments(self.h, rho.data_ptr(), vel.data_ptr(), conc.data_ptr(), diag, check=check)
        return rho, vel, conc, np.array(diag[:])

    def diag(self, check: bool = True) -> np.ndarray:
        diag = (C.c_double * 8)()
        B.lbm_moments(self.h, 0, 0, 0, diag, check=check)
        return np.array(diag[:])

    def populations(self, lattice: int = 0):
        """(19, nz, ny, nx) tensor of the real type: lattice 0 as f - w, 1 as is."""
        import torch
        nx, ny, nz = self.shape
        out = torch.empty((19, nz, ny, nx), dtype=self.dtype, device=self.device)
        B.lbm_populations(self.h, lattice, out.data_ptr())
        return out

    def save_state(self) -> np.ndarray:
        """Checkpoint of the lattice (host bytes, lbm_save_state)."""
        buf = np.empty(B.lbm_state_bytes(self.h), dtype=np.uint8)
        B.lbm_save_state(self.h, buf)
        return buf

    def load_state(self, buf: np.ndarray) -> "Simulation":
        """Resume from a checkpoint taken from a lattice of the same problem
        (lbm_load_state)."""
        B.lbm_load_state(self.h, np.ascontiguousarray(buf, dtype=np.uint8))
        return self

    def solute_totals(self):
        """Miscible: Sum eps C_k over fluid cells for every solute (FP64 list)."""
        return B.lbm_solute_totals(self.h, self.problem.nspecies)

    def free_surface(self, fill: bool = False):
        """Free surface: (classes uint8 (nz,ny,nx) 0 gas / 1 interface / 2 liquid /
        3 solid, liquid mass float64 (nz,ny,nx), lost excess mass) on the device;
        with fill=True also the fill fractions (float64) before the lost mass."""
        import torch
        nx, ny, nz = self.shape
        cls = torch.empty((nz, ny, nx), dtype=torch.uint8, device=self.device)
        mass = torch.empty((nz, ny, nx), dtype=torch.float64, device=self.device)
        lam = torch.empty((nz, ny, nx), dtype=torch.float64, device=self.device) if fill else None
        lost = B.lbm_free_surface(self.h, cls.data_ptr(), mass.data_ptr(), lam.data_ptr() if fill else 0)
        return (cls, mass, lam, lost) if fill else (cls, mass, lost)

    def close(self):
        if getattr(self, "h", None) is not None:
            B.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(sims, nsteps):
    """Advance several simulations (same stream) with batched launches."""
    B.lbm_step_batch([s.h for s in sims], nsteps)
