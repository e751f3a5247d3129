"""The C ABI without a GPU: the library loads, exports every entry point of
include/lbm.h, sizes workspaces and rejects invalid arguments before any GPU
call."""
import ctypes as C
import os
import re

import pytest

from paper_0912_4230_amd import binding as B
from paper_0912_4230_amd import inputs as I
from paper_0912_4230_amd.sim import make_desc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_function():
    names = _header_functions()
    assert set(names) == set(B.EXPORTED), names
    L = B.lib()
    for n in names:
        assert hasattr(L, n), n


def test_struct_layout_matches_header(tmp_path):
    """sizeof / offsetof of the ABI structs as the C compiler lays them out
    from include/lbm.h, against the ctypes mirrors of the binding."""
    fields = {"lbm_face": B.lbm_face, "lbm_desc": B.lbm_desc, "lbm_medium": B.lbm_medium}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', "int main(void) {"]
    for name, cls in fields.items():
        lines.append(f'printf("{name} sizeof %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in fields.items():
        assert got[(name, "sizeof")] == C.sizeof(cls), name
        for f in cls._fields_:
            assert got[(name, f[0])] == getattr(cls, f[0]).offset, (name, f[0])


def test_lattice_table():
    vel, w = B.lbm_lattice()
    assert len(set(vel)) == 19
    assert abs(sum(w) - 1.0) < 1e-15
    for q, v in enumerate(vel):
        s2 = sum(c * c for c in v)
        assert w[q] == {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[s2]
    assert B.lbm_strerror(B.LBM_ENOMEM) == "workspace too small"


def _desc(**kw):
    p = I.poiseuille(shape=(8, 6, 5))
    d = make_desc(p, B.LBM_F32)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_workspace_size():
    d = _desc()
    n = 8 * 6 * 5
    ws = B.lbm_workspace_bytes(d)
    assert ws >= 2 * 19 * n * 4 + 4 * n * 4
    d64 = _desc(storage=B.LBM_F64)
    assert B.lbm_workspace_bytes(d64) > ws
    dm = make_desc(I.miscible(shape=(8, 6, 5)), B.LBM_BF16_DEV)
    dm32 = make_desc(I.miscible(shape=(8, 6, 5)), B.LBM_F32)
    assert B.lbm_workspace_bytes(dm) < B.lbm_workspace_bytes(dm32)
    # an obstacle mask adds one 32-bit link word per cell
    assert B.lbm_workspace_bytes(_desc(solid_mask=1)) - ws == -(-n * 4 // 256) * 256


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("physics", 7), ("storage", 9), ("nu0", 0.0), ("nu0", -1.0),
    ("a0", -1.0), ("cap", 0.0), ("diag_every", -2), ("A", 0.01), ("solid_mask", 2),
])
def test_invalid_descriptions_rejected(field, value):
    d = _desc(**{field: value})
    assert B.lbm_workspace_bytes(d) == 0
    h = C.c_void_p()
    st = B.lib().lbm_create(C.byref(d), C.c_void_p(1 << 20), C.c_size_t(1 << 30), None, C.byref(h))
    assert st == B.LBM_EINVAL and not h.value


def test_face_rules():
    d = _desc()
    d.face[0].kind = B.LBM_FACE_WALL      # -x wall but +x periodic: inconsistent
    assert B.lbm_workspace_bytes(d) == 0
    d = _desc()
    d.face[0].kind = B.LBM_FACE_RESERVOIR
    d.face[1].kind = B.LBM_FACE_RESERVOIR
    d.face[0].rho = -1.0
    assert B.lbm_workspace_bytes(d) == 0
    d.face[0].rho = 1.1
    assert B.lbm_workspace_bytes(d) > 0
    d = make_desc(I.drop(shape=(10, 10, 10), radius=3), B.LBM_F32)
    d.tau1 = 0.5
    assert B.lbm_workspace_bytes(d) == 0
    d.tau1 = 0.7
    d.beta = 1.5
    assert B.lbm_workspace_bytes(d) == 0


def test_create_checks_before_gpu():
    d = _desc()
    need = B.lbm_workspace_bytes(d)
    h = C.c_void_p()
    L = B.lib()
    # workspace too small
    assert L.lbm_create(C.byref(d), C.c_void_p(1 << 20), C.c_size_t(need - 1), None, C.byref(h)) == B.LBM_ENOMEM
    # misaligned workspace
    assert L.lbm_create(C.byref(d), C.c_void_p((1 << 20) + 8), C.c_size_t(need), None, C.byref(h)) == B.LBM_EINVAL
    # null arguments
    assert L.lbm_create(None, C.c_void_p(1 << 20), C.c_size_t(need), None, C.byref(h)) == B.LBM_EINVAL
    assert L.lbm_step(None, 1) == B.LBM_EINVAL
    assert L.lbm_moments(None, None, None, None, None) == B.LBM_EINVAL
    assert L.lbm_destroy(None) == B.LBM_EINVAL
    assert L.lbm_steps_done(None) == -1
    # checkpoint calls on a NULL handle
    buf = (C.c_ubyte * 64)()
    assert L.lbm_state_bytes(None) == 0
    assert L.lbm_save_state(None, buf, C.c_size_t(64)) == B.LBM_EINVAL
    assert L.lbm_load_state(None, buf, C.c_size_t(64)) == B.LBM_EINVAL


def test_checkpoint_buffers_checked_in_the_binding():
    """The library reads or writes buf.nbytes bytes from a buffer's first
    element: the binding accepts only C-contiguous uint8 arrays (writable for
    a save) and raises before any library call otherwise.  No GPU call."""
    import numpy as np
    good = np.zeros(64, dtype=np.uint8)
    ro = good.copy()
    ro.flags.writeable = False
    for bad in (np.zeros(128, dtype=np.uint8)[::2], np.zeros(16, dtype=np.float32), ro, bytearray(64)):
        with pytest.raises(ValueError):
            B.lbm_save_state(None, bad)
    for bad in (np.zeros(128, dtype=np.uint8)[::2], np.zeros(16, dtype=np.float32), bytearray(64)):
        with pytest.raises(ValueError):
            B.lbm_load_state(None, bad)
    # a read-only checkpoint loads; a NULL handle is the library's EINVAL
    with pytest.raises(B.LbmError) as e:
        B.lbm_load_state(None, ro)
    assert e.value.status == B.LBM_EINVAL
    with pytest.raises(B.LbmError) as e:
        B.lbm_save_state(None, good)
    assert e.value.status == B.LBM_EINVAL


@pytest.mark.parametrize("storage,nz", [(B.LBM_F64, 255), (B.LBM_F32, 511), (B.LBM_BF16_DEV, 1023)])
def test_maximum_lattice_sizes(storage, nz):
    """Planes are addressed by 32-bit byte offsets from a uniform base (a
    bounce-back selects within a plane pair of padded planes): with
    1024 x 1024 planes, 255 / 511 / 1023 planes (FP64 / FP32 / 16-bit, just
    under 2^28 / 2^29 / 2^30 cells) are accepted, one more is rejected.  No
    GPU call."""
    nx = ny = 1024
    d = _desc(nx=nx, ny=ny, nz=nz, storage=storage)
    ok = B.lbm_workspace_bytes(d)
    assert ok > 2 * 19 * nx * ny * nz * {B.LBM_F64: 8, B.LBM_F32: 4}.get(storage, 2)
    d = _desc(nx=nx, ny=ny, nz=nz + 1, storage=storage)
    assert B.lbm_workspace_bytes(d) == 0


def test_free_surface_descriptions():
    """Free surface: its workspace adds the class, mass and fill-fraction
    planes; reservoir faces are rejected before any GPU call."""
    from paper_0912_4230_amd import inputs as I
    from paper_0912_4230_amd.sim import make_desc
    p = I.slab(shape=(48, 20, 10))
    q = I.Problem(shape=p.shape).fill_defaults()
    ws_fs = B.lbm_workspace_bytes(make_desc(p, B.LBM_F32))
    ws_1 = B.lbm_workspace_bytes(make_desc(q, B.LBM_F32))
    n = 48 * 20 * 10
    assert ws_fs - ws_1 >= 3 * n + 7 * 8 * n
    p.faces[0] = I.Face(kind=I.RESERVOIR)
    p.faces[1] = I.Face(kind=I.RESERVOIR)
    assert B.lbm_workspace_bytes(make_desc(p, B.LBM_F32)) == 0
    # every free-surface generator gives a valid description
    for g in (I.falling_drop(), I.falling_drop(shape=(12, 10, 9), radius=3.0, axis=2), I.pool(), I.slab()):
        assert B.lbm_workspace_bytes(make_desc(g, B.LBM_F64)) > 0


def test_species_and_surface_tension_descriptions():
    """Several solutes: 1-4 and miscible only, further relaxation times > 1/2;
    surface tension: two-fluid or free surface, A >= 0.  Rejected before any
    GPU call (lbm_workspace_bytes = 0)."""
    import numpy as np
    from paper_0912_4230_amd import inputs as I
    from paper_0912_4230_amd.sim import make_desc
    p = I.miscible(shape=(16, 12, 10), seed=0)
    base = B.lbm_workspace_bytes(make_desc(p, B.LBM_F32))
    p.species_tau_d = (0.8, 1.2)
    d = make_desc(p, B.LBM_F32)
    ws3 = B.lbm_workspace_bytes(d)
    # two more lattices, two copies each, plus two moment planes
    assert ws3 > base + 2 * 2 * 19 * 16 * 12 * 10 * 4
    d.nspecies = 5
    assert B.lbm_workspace_bytes(d) == 0
    d.nspecies = 3
    d.tau_d_x[1] = 0.5
    assert B.lbm_workspace_bytes(d) == 0
    d.tau_d_x[1] = float("nan")
    assert B.lbm_workspace_bytes(d) == 0
    q = I.Problem(shape=(8, 8, 8)).fill_defaults()
    dq = make_desc(q, B.LBM_F32)
    dq.nspecies = 2
    assert B.lbm_workspace_bytes(dq) == 0
    dq.nspecies = 1
    assert B.lbm_workspace_bytes(dq) > 0
    # surface tension: free surface yes (A >= 0), single fluid no
    fs = I.slab()
    dfs = make_desc(fs, B.LBM_F32)
    dfs.A = 0.001
    assert B.lbm_workspace_bytes(dfs) > 0
    dfs.A = -0.001
    assert B.lbm_workspace_bytes(dfs) == 0
    dq.A = 0.001
    assert B.lbm_workspace_bytes(dq) == 0
