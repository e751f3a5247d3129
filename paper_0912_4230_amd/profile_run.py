"""Small fixed workloads to run under rocprofv3 (kernel trace or PMC counters).

  python -m paper_0912_4230_amd.profile_run step --physics miscible --size 256 --storage f32 --steps 10
  python -m paper_0912_4230_amd.profile_run copy --mib 2048 --reps 5

`step` sets up one lattice of the chosen workload and runs the given number
of steps (one step kernel launch each, plus the colour pass in two-fluid
mode, or the five launches of a free-surface step); `copy` runs torch's device-to-device copy of a buffer of known size,
the reference kernel used to scale the FETCH_SIZE / WRITE_SIZE counters to
bytes.  Both print what they ran, with the byte counts of one launch.
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def problem(physics: str, n: int):
    from paper_0912_4230_amd import inputs as I
    if physics == "miscible":
        return I.miscible(shape=(n, n, n), seed=0)
    if physics == "immiscible":
        return I.drop(shape=(n, n, n), radius=20.0 * n / 128.0)
    if physics == "single":
        return I.poiseuille(shape=(n, n, n))
    if physics == "freesurface":
        return I.penetration(shape=(n, n, n), seed=0)
    if physics == "species":
        # the miscible workload with a second solute (tau_d 0.8, inlet 0.5)
        import numpy as np
        p = I.miscible(shape=(n, n, n), seed=0)
        p.species_tau_d = (0.8,)
        p.faces[0].conc_x = (0.5,)
        p.faces[1].conc_x = (0.0,)
        p.c0 = np.zeros((2, n, n, n))
        return p
    if physics == "wood":
        return I.wood(shape=(n, n, n))
    raise ValueError(physics)


def run_step(args):
    import torch
    from paper_0912_4230_amd.sim import Simulation
    p = problem(args.physics, args.size)
    sim = Simulation(p, storage=args.storage, diag_every=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"profile_run step: {args.physics} {args.size}^3 {args.storage}, {args.steps} steps, "
          f"{dt / args.steps * 1e3:.3f} ms/step (host clock)", flush=True)
    sim.close()


def run_copy(args):
    import torch
    n = args.mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"profile_run copy: {args.reps} launches, each reads {n * 4} B and writes {n * 4} B", flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("step")
    s.add_argument("--physics", default="miscible", choices=["single", "miscible", "immiscible", "freesurface", "species", "wood"])
    s.add_argument("--size", type=int, default=256)
    s.add_argument("--storage", default="f32", choices=["f64", "f32", "bf16", "f16", "bf16s", "f16s"])
    s.add_argument("--steps", type=int, default=10)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=2048)
    c.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    from paper_0912_4230_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        raise SystemExit("libporolbm.so is not built: run __graft_entry__.build()")
    (run_step if args.what == "step" else run_copy)(args)


if __name__ == "__main__":
    main()
