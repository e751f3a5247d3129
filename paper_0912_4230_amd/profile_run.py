"""Small fixed workloads to run under rocprofv3 (kernel trace or PMC counters).

  python -m paper_0912_4230_amd.profile_run step --physics miscible --size 256 --storage f32 --steps 10
  python -m paper_0912_4230_amd.profile_run copy --mib 2048 --reps 5 [--kernel f4]

`step` sets up one lattice of the chosen workload and runs the given number
of steps (one step kernel launch each, plus the colour pass in two-fluid
mode, or the five launches of a free-surface step); `copy` runs torch's
device-to-device copy of a buffer of known size, the reference kernel used
to scale the FETCH_SIZE / WRITE_SIZE counters to bytes, or (--kernel f4) the
float4 non-temporal streaming copy of the probe library, the practical
ceiling of a read-once / write-once stream.  Both print what they ran, with
the byte counts of one launch.
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
        return I.miscible_parallel(n, seed=0) if n >= 384 else I.miscible(shape=(n, n, n), seed=0)
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
    """torch's device copy (the counter calibration reference), or with
    --kernel f4 the probe library's float4 non-temporal streaming copy; the
    rate is timed with HIP events on the stream of the launches."""
    import ctypes
    import torch
    n = args.mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    if args.kernel == "f4":
        from paper_0912_4230_amd.build_lib import PROBE_LIB
        if not os.path.exists(PROBE_LIB):
            raise SystemExit("libporolbm_probe.so is not built: run __graft_entry__.build()")
        probe = ctypes.CDLL(PROBE_LIB)
        probe.probe_copy_f4.restype = ctypes.c_int
        probe.probe_copy_f4.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.c_int]

        def launch():
            rc = probe.probe_copy_f4(b.data_ptr(), a.data_ptr(), n * 4, stream.cuda_stream, args.blocks)
            if rc:
                raise SystemExit(f"probe_copy_f4 failed ({rc})")
    else:
        def launch():
            b.copy_(a)
    launch()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.reps):
        launch()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.reps
    print(f"profile_run copy ({args.kernel}): {args.reps + 1} launches, each reads {n * 4} B and writes {n * 4} B; "
          f"{ms:.3f} ms per launch, {2 * n * 4 / ms / 1e6:.1f} GB/s (HIP events)", flush=True)


def run_streams(args):
    """The probe library's 38-stream kernels (38 planes read and written, one
    cell per thread) over n = size^3 cells of 4- or 2-byte elements: in the
    plane-major layout of the lattice workspace (planes `pad` elements apart
    beyond n), slice-major (all 38 planes of each z-slice of size^2 cells
    contiguous, `pad` elements after each) or row-interleaved (all 38 planes of
    each row of size cells contiguous, `pad` elements after each); with
    --shift every stream reads the upstream cell of its D3Q19 link in a
    periodic cube (the pull of a step without its arithmetic; plane and row
    layouts, size a power of two); with --xcd each XCD sweeps runs of 4
    consecutive blocks of cells, as the lattice step does; --uniform is the
    shifted pull with row groups addressed as the step addresses its planes
    (uniform source-row bases, 32-bit x offsets).  HIP-event rate."""
    import ctypes
    import torch
    from paper_0912_4230_amd.build_lib import PROBE_LIB
    if not os.path.exists(PROBE_LIB):
        raise SystemExit("libporolbm_probe.so is not built: run __graft_entry__.build()")
    probe = ctypes.CDLL(PROBE_LIB)
    probe.probe_streams38.restype = ctypes.c_int
    probe.probe_streams38.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_size_t,
                                      ctypes.c_size_t, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int]
    probe.probe_streams38_cube.restype = ctypes.c_int
    probe.probe_streams38_cube.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int]
    probe.probe_streams_aa.restype = ctypes.c_int
    probe.probe_streams_aa.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                                       ctypes.c_void_p]
    if args.inplace:
        return run_inplace(args, probe)
    probe.probe_streams_uni.restype = ctypes.c_int
    probe.probe_streams_uni.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_size_t, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int]
    n = args.size ** 3
    ns = 19 if args.pairs else 38
    elem = args.elem * (2 if args.pairs else 1)
    if args.pairs and not args.uniform:
        raise SystemExit("streams: --pairs runs with --uniform")
    cube = args.layout == "row" or args.shift or args.xcd or args.uniform
    if cube:
        lg = args.size.bit_length() - 1
        if args.size != 1 << lg or args.layout == "slice":
            raise SystemExit("streams: the row layout and --shift take a power-of-two size, plane or row layout")
    if args.layout == "plane":
        pstride, slice_, sstride = n + args.pad, 0, 0
        total = ns * pstride
    elif args.layout == "slice":
        pstride, slice_, sstride = 0, args.size ** 2, args.size ** 2 + args.pad
        total = args.size * 38 * sstride
    else:
        pstride, pitch = 0, args.size + args.pad
        total = args.size ** 2 * ns * pitch
    dt = {8: torch.int64, 4: torch.float32, 2: torch.int16}[elem]
    a = torch.zeros(total, dtype=dt, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()

    def launch():
        if args.pairs:
            rc = probe.probe_streams_uni(b.data_ptr(), a.data_ptr(), lg, ns, int(args.layout == "row"), pstride,
                                         pitch if args.layout == "row" else 0, stream.cuda_stream, elem)
        elif cube:
            rc = probe.probe_streams38_cube(b.data_ptr(), a.data_ptr(), lg, int(args.layout == "row"),
                                            int(args.shift), 2 if args.uniform else int(args.xcd), pstride, pitch if args.layout == "row" else 0,
                                            stream.cuda_stream, args.elem)
        else:
            rc = probe.probe_streams38(b.data_ptr(), a.data_ptr(), n, pstride, slice_, sstride, stream.cuda_stream,
                                       args.elem)
        if rc:
            raise SystemExit(f"probe_streams38 failed ({rc})")
    launch()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.reps):
        launch()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.reps
    print(f"profile_run streams: {args.layout}{' shifted' if args.shift else ''}{' xcd-groups' if args.xcd else ''}"
          f"{' uniform-rows' if args.uniform else ''}, {args.size}^3 cells, {ns} planes of "
          f"{elem}-byte elements, pad {args.pad} elements: {ms:.3f} ms per launch, "
          f"{2 * 38 * args.elem * n / ms / 1e6:.1f} GB/s (HIP events)", flush=True)


def run_inplace(args, probe):
    """The in-place probe: 38 (or with --pairs 19) planes of 4-byte elements of
    one plane-major copy, every element read and written back by one thread,
    at the cell's own place (even) or its link's upstream cell (odd), with the
    XCD row groups of the lattice step."""
    import torch
    lg = args.size.bit_length() - 1
    if args.size != 1 << lg or args.size < 256 or args.elem != 4 or args.layout != "plane":
        raise SystemExit("streams --inplace: size 256 or 512, 4-byte elements, plane layout")
    n = args.size ** 3
    ns = 19 if args.pairs else 38
    pstride = n + args.pad
    a = torch.zeros(ns * pstride, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    odd = int(args.inplace == "odd")

    def launch():
        rc = probe.probe_streams_aa(a.data_ptr(), lg, ns, odd, pstride, stream.cuda_stream)
        if rc:
            raise SystemExit(f"probe_streams_aa failed ({rc})")
    launch()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.reps):
        launch()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.reps
    print(f"profile_run streams: in place ({args.inplace}), {args.size}^3 cells, {ns} planes of 4-byte elements, "
          f"pad {args.pad} elements: {ms:.3f} ms per launch, {2 * ns * 4 * n / ms / 1e6:.1f} GB/s (HIP events)",
          flush=True)


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
    c.add_argument("--kernel", default="torch", choices=["torch", "f4"])
    c.add_argument("--blocks", type=int, default=8192, help="grid of the f4 probe (256 threads per block)")
    t = sub.add_parser("streams")
    t.add_argument("--size", type=int, default=256)
    t.add_argument("--layout", default="plane", choices=["plane", "slice", "row"])
    t.add_argument("--shift", action="store_true", help="pull every stream from its link's upstream cell")
    t.add_argument("--xcd", action="store_true", help="map blocks to XCD row groups of 4 blocks")
    t.add_argument("--pairs", action="store_true",
                   help="19 planes of elements twice --elem wide (both lattices' values of a link side by side)")
    t.add_argument("--uniform", action="store_true",
                   help="shifted pull with XCD row groups and uniform row bases (size >= 256)")
    t.add_argument("--inplace", choices=["odd", "even"],
                   help="one copy read and written in place: at the link's upstream cell (odd) or the cell (even)")
    t.add_argument("--pad", type=int, default=128, help="elements of padding after each plane (slice)")
    t.add_argument("--elem", type=int, default=4, choices=[4, 2], help="element bytes")
    t.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    from paper_0912_4230_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        raise SystemExit("libporolbm.so is not built: run __graft_entry__.build()")
    {"step": run_step, "copy": run_copy, "streams": run_streams}[args.what](args)


if __name__ == "__main__":
    main()
