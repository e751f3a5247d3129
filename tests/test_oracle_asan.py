"""The oracle's C under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): a copy of lbm_oracle.c built with -fsanitize=address,undefined
runs every physics and every entry point the tests use on small grids
(reservoirs, walls, obstacles, full tensors, three solutes, a free surface
with conversions in both directions, state export and import) in a child
process; any invalid access or undefined operation aborts it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
sys.path.insert(0, sys.argv[2])
sys.path.insert(0, sys.argv[3])
import numpy as np
from oracle import oracle as O
from paper_0912_4230_amd import inputs as I

def run(p, steps, fs=False, species=False):
    o = O.Oracle(p)
    o.step(steps // 2)
    st = [o.get_state(k) for k in range(2 if p.physics in (I.MISCIBLE, I.IMMISCIBLE) else 1)]
    o.step(steps - steps // 2)
    o.moments(); o.diag(); o.cell_types()
    if species:
        for k in range(3):
            o.species_conc(k)
        o.species_totals()
    if fs:
        cls, mass, lost = o.fs_state()
        rho = o.moments()[0]
        lam = np.where(cls == 2, 1.0, np.where(cls == 1, mass / np.where(rho > 0, rho, 1.0), 0.0))
        o.fs_set_state(cls, mass, lam)
    for k, s in enumerate(st):
        o.set_state(k, s, steps // 2)
    o.step(2)
    o.close()

with O.library(sys.argv[1]):
    run(I.miscible(shape=(14, 11, 9), seed=1), 24)
    p = I.miscible(shape=(14, 12, 10), seed=2, ring_angle=45.0)
    p.solid = I.sphere_obstacles(p.shape, seed=3, solid_fraction=0.1, radius=(1.5, 2.5))
    run(p, 24)
    sys.path.insert(0, sys.argv[4])
    from test_gpu_species import _three_solutes
    run(_three_solutes(shape=(12, 10, 9), seed=1), 24, species=True)
    run(I.drop(shape=(16, 15, 14), radius=4.0, speed=0.05), 24)
    run(I.penetration(shape=(14, 16, 12), seed=1), 40, fs=True)
    run(I.poiseuille(shape=(6, 5, 12), G=1e-5), 30)
print("asan-clean", flush=True)
'''


def test_oracle_under_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("libasan is not installed")
    lib = str(tmp_path / "liblbm_oracle_asan.so")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-fPIC", "-shared", "-o", lib, os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-lm"], check=True)
    script = tmp_path / "child.py"
    script.write_text(CHILD)
    # the sanitizer runtime goes first; anything already preloaded stays
    pre = os.path.realpath(asan) + (":" + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")
    env = dict(os.environ, LD_PRELOAD=pre, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, str(script), lib, ROOT, ROOT, os.path.join(ROOT, "tests")], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "asan-clean" in r.stdout, r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
