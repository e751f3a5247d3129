"""Build the gfx950 shared library libporolbm.so (in the package directory)
from csrc/ with hipcc, and the measurement probe library libporolbm_probe.so
(profile_run only).  Every call compiles from source."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libporolbm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",                         # no implicit FMA: deterministic arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-variable", "-Wno-unknown-warning-option",
]


PROBE_LIB = os.path.join(HERE, "libporolbm_probe.so")


def build(verbose: bool = False, extra=()) -> str:
    """Compile the lattice library and the measurement probe library."""
    for src, out in ((os.path.join(CSRC, "lbm.hip"), LIB), (os.path.join(CSRC, "probe.hip"), PROBE_LIB)):
        cmd = [HIPCC, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, src, "-o", out + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
