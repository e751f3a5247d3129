"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every function has the name of the C entry point it calls.  The shared
library libporolbm.so sits next to this file (built by build_lib.py); if it
is missing, loading raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libporolbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = range(6)
LBM_SINGLE, LBM_MISCIBLE, LBM_IMMISCIBLE, LBM_FREESURF = range(4)
LBM_F64, LBM_F32, LBM_BF16_DEV, LBM_F16_DEV, LBM_BF16_SPLIT, LBM_F16_SPLIT = range(6)
LBM_FACE_PERIODIC, LBM_FACE_WALL, LBM_FACE_RESERVOIR = range(3)
LBM_MAX_SPECIES = 4

STORAGE_NAMES = {"f64": LBM_F64, "f32": LBM_F32, "bf16": LBM_BF16_DEV, "f16": LBM_F16_DEV,
                 "bf16s": LBM_BF16_SPLIT, "f16s": LBM_F16_SPLIT}
EXPORTED = ["lbm_workspace_bytes", "lbm_create", "lbm_create_static", "lbm_set_medium", "lbm_step", "lbm_step_batch",
            "lbm_moments", "lbm_populations", "lbm_solute_totals", "lbm_free_surface", "lbm_set_stream", "lbm_steps_done", "lbm_destroy",
            "lbm_lattice", "lbm_strerror", "lbm_state_bytes", "lbm_save_state", "lbm_load_state"]


class lbm_face(C.Structure):
    _fields_ = [("kind", C.c_int), ("rho", C.c_double), ("conc", C.c_double),
                ("contact_angle_deg", C.c_double)]


class lbm_desc(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("physics", C.c_int), ("storage", C.c_int),
        ("forchheimer", C.c_int), ("eps_gradient", C.c_int),
        ("G", C.c_double * 3),
        ("nu0", C.c_double), ("a0", C.c_double), ("a1", C.c_double), ("alpha", C.c_double),
        ("cap", C.c_double), ("k1", C.c_double), ("k0", C.c_double),
        ("tau1", C.c_double), ("tau2", C.c_double), ("tau_d", C.c_double),
        ("A", C.c_double), ("beta", C.c_double),
        ("face", lbm_face * 6),
        ("diag_every", C.c_int),
        ("solid_mask", C.c_int),
        ("solid_contact_angle_deg", C.c_double),
        ("full_tensor", C.c_int),
        ("nspecies", C.c_int),
        ("tau_d_x", C.c_double * (LBM_MAX_SPECIES - 1)),
        ("face_conc_x", (C.c_double * 6) * (LBM_MAX_SPECIES - 1)),
    ]


class lbm_medium(C.Structure):
    _fields_ = [("eps", C.c_void_p), ("kinv", C.c_void_p), ("rho0", C.c_void_p),
                ("vel0", C.c_void_p), ("c0", C.c_void_p), ("eps_uniform", C.c_double),
                ("kinv_uniform", C.c_double * 3), ("solid", C.c_void_p)]


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {lbm_strerror(status)} (status {status})")


_lib = None


def lib():
    """Load libporolbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.lbm_workspace_bytes.restype = C.c_size_t
        L.lbm_workspace_bytes.argtypes = [C.POINTER(lbm_desc)]
        L.lbm_create.restype = C.c_int
        L.lbm_create.argtypes = [C.POINTER(lbm_desc), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.lbm_set_stream.restype = C.c_int
        L.lbm_set_stream.argtypes = [vp, vp]
        L.lbm_create_static.restype = C.c_int
        L.lbm_create_static.argtypes = [C.POINTER(lbm_desc), vp, C.POINTER(vp)]
        L.lbm_set_medium.restype = C.c_int
        L.lbm_set_medium.argtypes = [vp, C.POINTER(lbm_medium)]
        L.lbm_step.restype = C.c_int
        L.lbm_step.argtypes = [vp, C.c_int]
        L.lbm_step_batch.restype = C.c_int
        L.lbm_step_batch.argtypes = [C.POINTER(vp), C.POINTER(C.c_int), C.c_int]
        L.lbm_moments.restype = C.c_int
        L.lbm_moments.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double)]
        L.lbm_populations.restype = C.c_int
        L.lbm_populations.argtypes = [vp, C.c_int, vp]
        L.lbm_steps_done.restype = C.c_longlong
        L.lbm_steps_done.argtypes = [vp]
        L.lbm_destroy.restype = C.c_int
        L.lbm_destroy.argtypes = [vp]
        L.lbm_lattice.restype = None
        L.lbm_lattice.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.lbm_solute_totals.restype = C.c_int
        L.lbm_solute_totals.argtypes = [vp, C.POINTER(C.c_double)]
        L.lbm_free_surface.restype = C.c_int
        L.lbm_free_surface.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double)]
        L.lbm_strerror.restype = C.c_char_p
        L.lbm_strerror.argtypes = [C.c_int]
        L.lbm_state_bytes.restype = C.c_size_t
        L.lbm_state_bytes.argtypes = [vp]
        L.lbm_save_state.restype = C.c_int
        L.lbm_save_state.argtypes = [vp, vp, C.c_size_t]
        L.lbm_load_state.restype = C.c_int
        L.lbm_load_state.argtypes = [vp, vp, C.c_size_t]
        _lib = L
    return _lib


def _check(status: int, where: str) -> int:
    if status != LBM_OK:
        raise LbmError(status, where)
    return status


def lbm_workspace_bytes(desc: lbm_desc) -> int:
    return int(lib().lbm_workspace_bytes(C.byref(desc)))


def lbm_create(desc: lbm_desc, workspace_ptr: int, ws_bytes: int, stream_ptr: int = 0):
    """Returns the handle (a c_void_p); raises LbmError on failure."""
    h = C.c_void_p()
    _check(lib().lbm_create(C.byref(desc), C.c_void_p(workspace_ptr), C.c_size_t(ws_bytes),
                            C.c_void_p(stream_ptr), C.byref(h)), "lbm_create")
    return h


def lbm_create_static(desc: lbm_desc, stream_ptr: int = 0):
    """Handle of a lattice in the library's static workspace of the current
    device (no allocation); raises LbmError on failure."""
    h = C.c_void_p()
    _check(lib().lbm_create_static(C.byref(desc), C.c_void_p(stream_ptr), C.byref(h)), "lbm_create_static")
    return h


def lbm_set_stream(h, stream_ptr: int = 0) -> int:
    return _check(lib().lbm_set_stream(h, C.c_void_p(stream_ptr or None)), "lbm_set_stream")


def lbm_set_medium(h, medium: lbm_medium) -> int:
    return _check(lib().lbm_set_medium(h, C.byref(medium)), "lbm_set_medium")


def lbm_step(h, nsteps: int) -> int:
    return _check(lib().lbm_step(h, int(nsteps)), "lbm_step")


def lbm_step_batch(handles, nsteps) -> int:
    n = len(handles)
    hs = (C.c_void_p * n)(*[hh.value for hh in handles])
    ns = (C.c_int * n)(*[int(s) for s in nsteps])
    return _check(lib().lbm_step_batch(hs, ns, n), "lbm_step_batch")


def lbm_moments(h, rho_ptr: int = 0, vel_ptr: int = 0, conc_ptr: int = 0, diag=None, check=True):
    """diag: a ctypes c_double*8 array or None.  Returns the status."""
    st = lib().lbm_moments(h, C.c_void_p(rho_ptr or None), C.c_void_p(vel_ptr or None),
                           C.c_void_p(conc_ptr or None), diag)
    if check:
        _check(st, "lbm_moments")
    return st


def lbm_populations(h, lattice: int, dst_ptr: int) -> int:
    return _check(lib().lbm_populations(h, int(lattice), C.c_void_p(dst_ptr)), "lbm_populations")


def lbm_solute_totals(h, nspecies: int):
    """Sum eps C_k over fluid cells for every solute (list of nspecies floats)."""
    out = (C.c_double * LBM_MAX_SPECIES)()
    _check(lib().lbm_solute_totals(h, out), "lbm_solute_totals")
    return [float(out[k]) for k in range(nspecies)]


def lbm_free_surface(h, cls_ptr: int = 0, mass_ptr: int = 0, lambda_ptr: int = 0) -> float:
    """Free surface: classes (uint8), masses and fill fractions (double) into
    device buffers (0: skip); returns the lost excess mass."""
    lost = C.c_double(0.0)
    _check(lib().lbm_free_surface(h, C.c_void_p(cls_ptr or None), C.c_void_p(mass_ptr or None),
                                  C.c_void_p(lambda_ptr or None), C.byref(lost)), "lbm_free_surface")
    return float(lost.value)


def lbm_steps_done(h) -> int:
    return int(lib().lbm_steps_done(h))


def lbm_state_bytes(h) -> int:
    return int(lib().lbm_state_bytes(h))


def _host_bytes(buf, writable: bool):
    """buf as one contiguous run of host bytes for the library, which reads or
    writes buf.nbytes bytes from its first element."""
    if not isinstance(buf, np.ndarray) or buf.dtype != np.uint8 or not buf.flags.c_contiguous:
        raise ValueError("checkpoint buffers are C-contiguous numpy uint8 arrays")
    if writable and not buf.flags.writeable:
        raise ValueError("the checkpoint buffer is read-only")
    return C.c_void_p(buf.ctypes.data), C.c_size_t(buf.nbytes)


def lbm_save_state(h, buf) -> int:
    """Write the checkpoint of h into buf (a writable, C-contiguous numpy uint8
    array of at least lbm_state_bytes(h) bytes)."""
    return _check(lib().lbm_save_state(h, *_host_bytes(buf, True)), "lbm_save_state")


def lbm_load_state(h, buf) -> int:
    """Replace h's state by the checkpoint in buf (a C-contiguous numpy uint8
    array)."""
    return _check(lib().lbm_load_state(h, *_host_bytes(buf, False)), "lbm_load_state")


def lbm_destroy(h) -> int:
    return _check(lib().lbm_destroy(h), "lbm_destroy")


def lbm_lattice():
    v = (C.c_int * 57)()
    w = (C.c_double * 19)()
    lib().lbm_lattice(v, w)
    return [tuple(v[3 * q:3 * q + 3]) for q in range(19)], list(w)


def lbm_strerror(status: int) -> str:
    return lib().lbm_strerror(int(status)).decode()
