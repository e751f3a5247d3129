"""The oracle's arithmetic in single precision (test infrastructure): the floor
that FP32 arithmetic of the method itself reaches on a workload, to compare
the FP32 GPU path with.  A copy of oracle/lbm_oracle.c in which every
`double` is `float` and <math.h> is <tgmath.h> (the math functions then take
their float forms) is compiled into a temporary library and driven through
the oracle's own entry points.  Constants stay double literals, so an
expression that mixes one with float values is evaluated in double and
rounded to float where it is stored; every state array, every per-cell
value and every accumulation is float.  Same loops, same order of
operations as the FP64 oracle."""
import ctypes as C
import os
import re
import subprocess

import numpy as np

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def build(tmpdir: str) -> str:
    """Write and compile the float copy; returns the library's path."""
    src = open(os.path.join(ROOT, "oracle", "lbm_oracle.c")).read()
    assert "#include <math.h>" in src
    src = re.sub(r"\bdouble\b", "float", src.replace("#include <math.h>", "#include <tgmath.h>"))
    c_path = os.path.join(tmpdir, "lbm_oracle_float.c")
    with open(c_path, "w") as f:
        f.write(src)
    lib = os.path.join(tmpdir, "liblbm_oracle_float.so")
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                    "-shared", "-o", lib, c_path, "-lm"], check=True)
    return lib


def _ftype(t):
    if t is C.c_double:
        return C.c_float
    if hasattr(t, "_length_"):
        return _ftype(t._type_) * t._length_
    return t


class FloatParams(C.Structure):
    """orc_params with every double field a float."""
    _fields_ = [(n, _ftype(t)) for n, t in O.OrcParams._fields_]


def _params(p) -> FloatParams:
    d = O.params_from_problem(p)
    f = FloatParams()
    for name, t in O.OrcParams._fields_:
        v = getattr(d, name)
        if hasattr(t, "_length_"):
            dst = getattr(f, name)
            for i in range(t._length_):
                if hasattr(t._type_, "_length_"):
                    for j in range(t._type_._length_):
                        dst[i][j] = v[i][j]
                else:
                    dst[i] = v[i]
        else:
            setattr(f, name, v)
    return f


def run(lib_path: str, problem, steps: int):
    """steps of problem in the float copy; returns (rho, V', C) as float64
    arrays in the oracle's layout, like Oracle.moments()."""
    p = problem.fill_defaults()
    nx, ny, nz = p.shape
    n = nx * ny * nz
    L = C.CDLL(lib_path)
    fp = C.POINTER(C.c_float)
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.POINTER(FloatParams), fp, fp, fp, fp, fp, C.POINTER(C.c_ubyte)]
    L.orc_step.argtypes = [C.c_void_p, C.c_int]
    L.orc_moments.argtypes = [C.c_void_p, fp, fp, fp]
    L.orc_destroy.argtypes = [C.c_void_p]
    keep = [np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1))
            for a in (p.eps, p.kinv, p.rho0, p.vel0, p.c0)]
    solid = None
    if p.solid is not None:
        solid = np.ascontiguousarray(np.asarray(p.solid).reshape(-1) != 0, dtype=np.uint8)
    prm = _params(p)
    h = L.orc_create(C.byref(prm), *[a.ctypes.data_as(fp) for a in keep],
                     solid.ctypes.data_as(C.POINTER(C.c_ubyte)) if solid is not None else None)
    assert h, "float oracle allocation failed"
    try:
        L.orc_step(h, steps)
        rho = np.zeros(n, np.float32)
        vel = np.zeros(3 * n, np.float32)
        conc = np.zeros(n, np.float32)
        L.orc_moments(h, rho.ctypes.data_as(fp), vel.ctypes.data_as(fp), conc.ctypes.data_as(fp))
    finally:
        L.orc_destroy(h)
    return (rho.reshape(nz, ny, nx).astype(np.float64), vel.reshape(3, nz, ny, nx).astype(np.float64),
            conc.reshape(nz, ny, nx).astype(np.float64))
