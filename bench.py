"""Benchmark of the porous-media lattice Boltzmann step on one MI355X.

Workload (default): the miscible mixture at 256^3 in FP32 -- hydrodynamic
lattice plus solute lattice (D = 0.05) in the seeded spruce-like medium
(porosity 0.4-0.8 sinusoidal along x with period 32, diagonal permeability
100:1:1 with lognormal noise sigma 0.3), hardening viscosity
nu = 0.1 e^{2C} min(e^{1e-4 t}, 10), Darcy + Forchheimer drag, pressure inlet
reservoir at x = 0 (C = 1) and outlet at x = 255.  One step = one pass of the
whole update over the lattice (stream + collide of both lattices; FP64
diagnostics every 100 steps).

Prints one JSON line: MLUPS (million lattice-cell updates per second),
the roofline of the step kernel (algorithmic bytes per launch / measured
kernel time vs 8 TB/s HBM peak), the same run with BF16- and FP16-stored
populations, and the FP64 CPU oracle timed on the host on a bounded sample.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--size N]
                       [--storage f32] [--no-cpu-baseline] [--no-reduced]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per lattice update of the miscible step: both lattices
# read and written once (2 x 19 x 2 populations) + porosity + 3 K^-1 values
def bytes_per_lup(storage_bytes, real_bytes=4, split=False):
    # split 16-bit storage adds one FP32 mass per cell and lattice, read and written
    return 2 * 19 * 2 * storage_bytes + 4 * real_bytes + (2 * 2 * 4 if split else 0)


def storage_bpl(st):
    return {"f64": bytes_per_lup(8, 8), "f32": bytes_per_lup(4), "bf16": bytes_per_lup(2), "f16": bytes_per_lup(2),
            "bf16s": bytes_per_lup(2, split=True), "f16s": bytes_per_lup(2, split=True)}[st]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def ensure_built():
    from paper_0912_4230_amd import binding
    from oracle import oracle
    if not os.path.exists(binding.LIB_PATH) or not os.path.exists(oracle.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def counter_traffic(key):
    """HBM bytes per launch of a kernel from the committed counter record
    (profiles/traffic.json), in GB -- or None when the kernel sources have
    changed since the counters were taken."""
    import json as _json
    from paper_0912_4230_amd.prof_summary import source_sha
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = _json.load(open(path))
    if rec.get("source_sha256") != source_sha() or key not in rec:
        return None
    return round(rec[key]["bytes"] / 1e9, 4)


def time_gpu(problem, storage, steps, warmup):
    import torch
    from paper_0912_4230_amd.sim import Simulation
    sim = Simulation(problem, storage=storage, diag_every=100)
    stream = sim.stream
    sim.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    sim.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    dg = sim.diag(check=False)
    sim.close()
    return ms, dg


class _StorageTag:
    """Text sink for serve()'s JSON records that adds the storage form."""

    def __init__(self, sink, storage):
        self.sink, self.storage = sink, storage

    def write(self, line):
        rec = json.loads(line)
        rec["storage"] = self.storage
        self.sink.write(json.dumps(rec) + "\n")


def serving_leg(storages=("f32", "bf16"), budget_gb=200.0, tick_steps=50, single_mlups=None, jsonl_path=None):
    """The serving workload: 64 requests, Poisson arrivals at 4/s, cubic edge
    log-uniform in [48, 192], 70% miscible / 30% two-fluid, 500-5000 steps,
    seeded spruce-like media (anisotropy U[10, 200]), admitted under an HBM
    budget with lattices resident on the device (continuous batching).  With
    `jsonl_path`, one JSON record per request (its storage added) goes there."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_0912_4230_amd import inputs as I
    from paper_0912_4230_amd.serve import GpuExecutor, serve
    reqs = I.request_stream()
    log("bench: generating the 64 request media")
    with ThreadPoolExecutor(8) as pool:
        probs = dict(zip([r.rid for r in reqs], pool.map(I.request_problem, reqs)))
    out = {"requests": len(reqs), "arrival_rate_per_s": 4.0, "budget_GB": budget_gb, "tick_steps": tick_steps,
           "offered_GLUP": round(sum(r.edge ** 3 * r.steps for r in reqs) / 1e9, 2),
           "percentile_rule": "nearest rank over the 64 latencies (p99 = the largest)"}
    sink = open(jsonl_path, "w") if jsonl_path else None
    for st in storages:
        log(f"bench: serving {st}")
        ex = GpuExecutor(storage=st, problems=probs)
        res = serve(reqs, ex, int(budget_gb * 1e9), tick_steps=tick_steps,
                    jsonl=_StorageTag(sink, st) if sink is not None else None)
        out[st] = {"p50_s": round(res["p50_s"], 3), "p99_s": round(res["p99_s"], 3),
                   "mean_s": round(res["mean_s"], 3), "aggregate_MLUPS": round(res["aggregate_mlups"], 1),
                   "completed": res["completed"], "failed": res["failed"], "max_active": res["max_active"],
                   "span_s": round(res["span_s"], 2), "ticks": res["ticks"],
                   "gpu_busy_s": round(res["busy_s"], 2), "gpu_busy_fraction": round(res["busy_fraction"], 3)}
        if single_mlups and st in single_mlups:
            out[st]["aggregate_vs_single_lattice_256"] = round(res["aggregate_mlups"] / single_mlups[st], 3)
        log(f"bench: serving {st}: {out[st]}")
    if sink is not None:
        sink.close()
    return out


def medium_parallel(n, seed=0, slabs=16):
    """The n^3 miscible problem with its medium generated in z-slabs in
    parallel (inputs.miscible_parallel)."""
    from paper_0912_4230_amd import inputs as I
    return I.miscible_parallel(n, seed=seed, slabs=slabs)


def precision_leg(n=512, steps=2000, timed=200, compare=True, placements=1):
    """Precision form: the miscible workload at n^3 with FP32, BF16- and
    FP16-stored populations (deviations and split) on the same GPU; step time
    over `timed` steps after 20 warm-up steps; with `compare` the run then
    continues to `steps` steps and the 16-bit fields are compared with the
    FP32 ones over the fluid cells (relative L2).  Without `compare`, each
    storage form is timed on `placements` workspaces allocated one after
    another (all held until the last is timed, so that each is fresh device
    memory): at 512^3 the step time depends on where the workspace lands, and
    the leg reports the median with every placement's time."""
    import torch
    from paper_0912_4230_amd.sim import Simulation
    log(f"bench: generating the {n}^3 medium")
    p = medium_parallel(n)
    ncell = n ** 3
    # release the blocks earlier legs left in torch's cache: each lattice of
    # this leg (up to 45 GB) then gets fresh device memory
    torch.cuda.empty_cache()
    res = {"grid": [n, n, n], "timed_steps": timed, "warmup": 20}
    if not compare:
        res["placements"] = placements
    if compare:
        res["steps"] = steps
    ref = None
    for st in ("f32", "bf16", "f16", "bf16s", "f16s"):
        log(f"bench: precision {n}^3 {st}")
        if not compare:
            held, times, nonfinite = [], [], 0
            for k in range(placements):
                sim = Simulation(p, storage=st, diag_every=100)
                sim.step(20)
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(sim.stream)
                sim.step(timed)
                b.record(sim.stream)
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b) / timed)
                nonfinite = max(nonfinite, int(sim.diag(check=False)[7]))
                held.append(sim)
            for sim in held:
                sim.close()
            del held, sim
            torch.cuda.empty_cache()
            ms = sorted(times)[len(times) // 2]
            bpl = storage_bpl(st)
            entry = {"ms_per_step": round(ms, 4), "ms_per_step_placements": [round(t, 4) for t in times],
                     "MLUPS": round(ncell / ms / 1e3, 1), "achieved_GBs": round(bpl * ncell / ms / 1e6, 1),
                     "bytes_per_lup": bpl, "frac_of_hbm_peak": round(bpl * ncell / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "traffic_GB_per_launch": counter_traffic(f"k_step miscible {n} {st}"),
                     "nonfinite": nonfinite}
            if st != "f32":
                entry["speedup_vs_f32"] = round(res["f32"]["ms_per_step"] / ms, 3)
            res[st] = entry
            log(f"bench: precision {n}^3 {st}: {entry}")
            continue
        sim = Simulation(p, storage=st, diag_every=100)
        sim.step(20)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(sim.stream)
        sim.step(timed)
        b.record(sim.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / timed
        if compare:
            sim.step(steps - 20 - timed)
        rho, vel, conc, dg = sim.moments(check=False)
        sim.close()
        del sim
        bpl = storage_bpl(st)
        entry = {"ms_per_step": round(ms, 4), "MLUPS": round(ncell / ms / 1e3, 1),
                 "achieved_GBs": round(bpl * ncell / ms / 1e6, 1), "bytes_per_lup": bpl,
                 "frac_of_hbm_peak": round(bpl * ncell / ms / 1e6 / HBM_PEAK_GBS, 4),
                 "traffic_GB_per_launch": counter_traffic(f"k_step miscible {n} {st}"),
                 "nonfinite": int(dg[7])}
        fields = (rho[:, :, 1:-1], vel[:, :, :, 1:-1], conc[:, :, 1:-1])   # fluid cells: x in [1, n-2]
        if ref is None:
            ref = fields
        else:
            def rel(x, y):
                return float(torch.linalg.vector_norm((x - y).double()) / torch.linalg.vector_norm(y.double()))
            entry["rel_l2_vs_f32"] = {"rho": rel(fields[0], ref[0]), "drho": rel(fields[0] - 1, ref[0] - 1),
                                      "vel": rel(fields[1], ref[1]), "conc": rel(fields[2], ref[2])}
            entry["speedup_vs_f32"] = round(res["f32"]["ms_per_step"] / ms, 3)
        res[st] = entry
        log(f"bench: precision {st}: {entry}")
        del rho, vel, conc
        torch.cuda.empty_cache()
    return res


def obstacle_leg(p, steps, warmup, storages=("f32", "bf16"), solid_fraction=0.1):
    """The miscible workload with obstacle cells: 4^3 solid cubes placed with
    probability 0.1 (seeded), every link into them bounced back.  Algorithmic
    bytes: 320 (FP32) / 168 (16-bit) per fluid cell plus the 4-byte link word
    of every cell."""
    import copy
    from paper_0912_4230_amd import inputs as I
    n = p.shape[0]
    q = copy.copy(p)
    q.solid = I.block_obstacles(p.shape, seed=0, solid_fraction=solid_fraction)
    ncell = n ** 3
    nfluid = int((q.solid == 0).sum())
    out = {"solid_fraction": round(1 - nfluid / ncell, 4), "obstacle": "4^3 cubes, seeded"}
    for st in storages:
        ms, dg = time_gpu(q, st, steps, warmup)
        s = ms / steps
        bpl = storage_bpl(st)
        out[st] = {"ms_per_step": round(s, 5), "MLUPS_all_cells": round(ncell / s / 1e3, 1),
                   "MLUPS_fluid_cells": round(nfluid / s / 1e3, 1),
                   "achieved_GBs": round((nfluid * bpl + ncell * 4) / (s / 1e3) / 1e9, 1),
                   "nonfinite": int(dg[7])}
        log(f"bench: obstacles {st}: {out[st]}")
    return out


def plain_method_leg(steps=1000):
    """The plain method at 32^3 in FP64: Poiseuille flow through a homogeneous
    porous medium (eps 0.7, K 1e-2, G 1e-6, tau 0.8, walls at z = 0, 31), the
    full 1000-step run timed on the device.  The lattice (10 MB of
    populations) stays in the caches, so this is launch- and latency-bound:
    MLUPS only, no roofline."""
    from paper_0912_4230_amd import inputs as I
    p = I.poiseuille(shape=(32, 32, 32))
    ms, dg = time_gpu(p, "f64", steps, 20)
    return {"grid": [32, 32, 32], "storage": "f64", "steps": steps, "ms_per_step": round(ms / steps, 5),
            "MLUPS": round(32 ** 3 * steps / (ms / 1e3) / 1e6, 1), "max_v": dg[6], "nonfinite": int(dg[7])}


def inclined_leg(n, steps, warmup, storages=("f32", "bf16")):
    """The miscible workload in the medium with annual rings inclined by 45
    degrees in the x-y plane: K^-1 is a full symmetric tensor per cell, held
    on the GPU as its eigenframe (unit quaternion) and eigenvalues, 7 planes.
    Algorithmic bytes per cell: populations + porosity + 7 tensor values."""
    from paper_0912_4230_amd import inputs as I
    log(f"bench: generating the {n}^3 inclined-ring medium")
    q = I.miscible(shape=(n, n, n), seed=0, ring_angle=45.0)
    ncell = n ** 3
    out = {"ring_angle_deg": 45.0, "tensor_planes": 7}
    for st in storages:
        ms, dg = time_gpu(q, st, steps, warmup)
        s = ms / steps
        bpl = storage_bpl(st) + 4 * 4     # 7 instead of 3 K^-1 values
        out[st] = {"ms_per_step": round(s, 5), "MLUPS": round(ncell / s / 1e3, 1), "bytes_per_lup": bpl,
                   "achieved_GBs": round(bpl * ncell / (s / 1e3) / 1e9, 1), "nonfinite": int(dg[7])}
        log(f"bench: inclined rings {st}: {out[st]}")
    return out


def fs_bytes_per_live_cell(st):
    """Algorithmic bytes of the free-surface stream/collide launch per liquid or
    interface cell: one lattice read and written + porosity + 3 K^-1 values."""
    sb = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2, "bf16s": 2, "f16s": 2}[st]
    rb = 8 if st == "f64" else 4
    return 2 * 19 * sb + 4 * rb + (2 * 4 if st in ("bf16s", "f16s") else 0)


def freesurface_leg(n, steps, warmup, storages=("f32", "bf16")):
    """Free surface (Sec. 3).  (a) Liquid penetrating the unsaturated
    spruce-like medium, n^3, liquid in the upper half, gravity along the
    grain: five launches per step; algorithmic bytes of the step = the
    stream/collide of the live cells (fs_bytes_per_live_cell) + 2 bytes per
    cell (class read, flag written) + 9 bytes per cell for the class passes.
    (b) The paper's droplet (Sec. 5.3): 140x140x1, R = 8, tau = 0.7, G = 1e-6,
    20000 steps in FP64, timed whole; total-mass error."""
    import torch
    from paper_0912_4230_amd import inputs as I
    from paper_0912_4230_amd.sim import Simulation
    log(f"bench: generating the {n}^3 penetration problem")
    q = I.penetration(shape=(n, n, n), seed=0)
    ncell = n ** 3
    out = {"workload": f"penetration {n}^3: spruce-like medium 100:1:1 (K_ref 1), liquid y >= n/2, G 1e-4 along -y"}
    # the first steps convert the whole initial interface (the flat liquid
    # surface and the pores it touches): the leg warms up past them so that it
    # times the steady penetration
    warmup = max(warmup, 200)
    out["warmup"] = warmup

    def live_cells(sim):
        cls = sim.free_surface()[0]
        return int(((cls == 1) | (cls == 2)).sum().item()), int((cls == 1).sum().item())

    for st in storages:
        sim = Simulation(q, storage=st, diag_every=100)
        M0 = sim.diag()[4]
        sim.step(warmup)
        live0, _ = live_cells(sim)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(sim.stream)
        sim.step(steps)
        t1.record(sim.stream)
        torch.cuda.synchronize()
        s = t0.elapsed_time(t1) / steps
        dg = sim.diag(check=False)
        live1, nif = live_cells(sim)
        live = (live0 + live1) // 2
        b = fs_bytes_per_live_cell(st) * live + 11 * ncell
        out[st] = {"ms_per_step": round(s, 5), "MLUPS_all_cells": round(ncell / s / 1e3, 1),
                   "MLUPS_live_cells": round(live / s / 1e3, 1), "live_cells": live, "interface_cells": nif,
                   "achieved_GBs_step": round(b / (s / 1e3) / 1e9, 1),
                   "traffic_GB_per_launch_stream_collide": counter_traffic(f"k_fs_step penetration {n} {st}"),
                   "mass_drift": float(dg[4] / M0 - 1.0), "nonfinite": int(dg[7])}
        log(f"bench: free surface {st}: {out[st]}")
        sim.close()
        torch.cuda.empty_cache()
    G, R = 1e-6, 8.0
    p = I.falling_drop(shape=(140, 140, 1), radius=R, centre=(70.0, 0.5 + R + 0.5 * G * 10600.0 ** 2, 0.0), G=G,
                       tau=0.7)
    sim = Simulation(p, storage="f64", diag_every=1000)
    M0 = sim.diag()[4]
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(sim.stream)
    sim.step(20000)
    t1.record(sim.stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    dg = sim.diag(check=False)
    out["paper_droplet"] = {"grid": [140, 140, 1], "steps": 20000, "storage": "f64", "total_ms": round(ms, 1),
                            "us_per_step": round(1e3 * ms / 20000, 2), "mass_error": float(abs(dg[4] / M0 - 1.0))}
    log(f"bench: paper droplet: {out['paper_droplet']}")
    sim.close()
    return out


def wood_leg(n, steps, warmup, storages=("f32", "bf16")):
    """The paper's wood workload in 3D (Sec. 5.5): the spruce medium from the
    density law, the porosity law and Eq. Ktensor, rings inclined by 45 degrees
    in the cross-section (full K^-1 tensor per cell), adhesive driven along the
    grain between reservoirs, the hardening law of Eq. nuall with the paper's
    constants.  Algorithmic bytes per cell as the inclined-ring leg."""
    from paper_0912_4230_amd import inputs as I
    log(f"bench: generating the {n}^3 wood medium")
    q = I.wood(shape=(n, n, n))
    ncell = n ** 3
    out = {"workload": f"wood {n}^3: spruce density law, Eq. Ktensor, rings at 45 deg, flow along the grain"}
    for st in storages:
        ms, dg = time_gpu(q, st, steps, warmup)
        s = ms / steps
        bpl = storage_bpl(st) + 4 * 4
        out[st] = {"ms_per_step": round(s, 5), "MLUPS": round(ncell / s / 1e3, 1), "bytes_per_lup": bpl,
                   "achieved_GBs": round(bpl * ncell / (s / 1e3) / 1e9, 1), "max_v": dg[6],
                   "nonfinite": int(dg[7])}
        log(f"bench: wood {st}: {out[st]}")
    return out


def species_leg(n, steps, warmup, storages=("f32", "bf16")):
    """The miscible workload with a second solute (its own lattice, tau_d 0.8,
    inlet concentration 0.5) sharing V' with the first: algorithmic bytes per
    cell = the miscible step's + one more lattice read and written."""
    from paper_0912_4230_amd import inputs as I
    q = I.miscible(shape=(n, n, n), seed=0)
    q.species_tau_d = (0.8,)
    q.faces[0].conc_x = (0.5,)
    q.faces[1].conc_x = (0.0,)
    q.c0 = np.zeros((2, n, n, n))
    ncell = n ** 3
    out = {"workload": f"miscible {n}^3 with 2 solutes (tau_d 0.65 and 0.8)"}
    for st in storages:
        ms, dg = time_gpu(q, st, steps, warmup)
        s = ms / steps
        sb = 4 if st == "f32" else 2
        bpl = storage_bpl(st) + 2 * 19 * sb
        out[st] = {"ms_per_step": round(s, 5), "MLUPS": round(ncell / s / 1e3, 1), "bytes_per_lup": bpl,
                   "achieved_GBs": round(bpl * ncell / (s / 1e3) / 1e9, 1), "nonfinite": int(dg[7])}
        log(f"bench: two solutes {st}: {out[st]}")
    return out


def cpu_baseline(budget_s=15.0):
    """FP64 oracle on the host: miscible physics on a 64^3 crop of the same
    seeded medium, as many steps as fit in about budget_s seconds."""
    from oracle import oracle as O
    from paper_0912_4230_amd import inputs as I
    p = I.miscible(shape=(64, 64, 64), seed=0)
    o = O.Oracle(p)
    o.step(1)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s:
        o.step(5)
        n += 5
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 64 ** 3 * n / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"miscible physics, 64^3 crop of the seeded medium, {n} steps, FP64, {dt:.1f} s"}


def cpu_baseline_full(threads_all):
    """The CPU-baseline protocol in full: the FP64 oracle with one thread and
    with all threads on the Poiseuille channel (32^3, 1000 steps, FP64 plain
    method), and on the miscible and two-fluid physics at 64^3 x 200 steps.
    MLUPS over all cells; a reported baseline, not a target."""
    from oracle import oracle as O
    from paper_0912_4230_amd import inputs as I
    cases = [("poiseuille 32^3 x 1000 (plain method)", lambda: I.poiseuille(shape=(32, 32, 32)), 1000),
             ("miscible 64^3 x 200", lambda: I.miscible(shape=(64, 64, 64), seed=0), 200),
             ("two-fluid drop 64^3 x 200", lambda: I.drop(shape=(64, 64, 64), radius=10.0), 200)]
    out = {"cores_all": threads_all}
    for name, make, steps in cases:
        row = {}
        for nt in (1, threads_all):
            O.set_threads(nt)
            o = O.Oracle(make())
            t0 = time.perf_counter()
            o.step(steps)
            dt = time.perf_counter() - t0
            o.close()
            row[f"threads_{nt}"] = {"MLUPS": round(o.n * steps / dt / 1e6, 2), "seconds": round(dt, 2)}
            log(f"bench: cpu oracle {name}, {nt} threads: {dt:.1f} s")
        out[name] = row
    O.set_threads(threads_all)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reduced", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-log", default=None, help="write one JSON record per served request to this file")
    ap.add_argument("--no-obstacles", action="store_true")
    ap.add_argument("--no-inclined", action="store_true")
    ap.add_argument("--no-freesurface", action="store_true")
    ap.add_argument("--no-wood", action="store_true")
    ap.add_argument("--no-species", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle with 1 and all threads on the 32^3 channel and 64^3 x 200 steps")
    ap.add_argument("--no-512", action="store_true", help="skip the 512^3 precision-form timing")
    ap.add_argument("--precision", action="store_true",
                    help="run the 512^3 precision form to 2000 steps and compare the 16-bit fields with FP32")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the lattice update is not sharded across GPUs in this "
              "build (see the design notes for the slab decomposition); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    ensure_built()
    from paper_0912_4230_amd import inputs as I
    from paper_0912_4230_amd import binding as B

    n = args.size
    log(f"bench: generating the {n}^3 seeded medium")
    p = I.miscible(shape=(n, n, n), seed=0)
    ncell = n ** 3
    sb = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[args.storage]
    rb = 8 if args.storage == "f64" else 4

    log(f"bench: {args.storage} {n}^3 warmup {args.warmup} steps {args.steps}")
    ms, dg = time_gpu(p, args.storage, args.steps, args.warmup)
    ms_step = ms / args.steps
    mlups = ncell * args.steps / (ms / 1e3) / 1e6
    bpl = bytes_per_lup(sb, rb)
    achieved = bpl * ncell / (ms_step / 1e3) / 1e9
    log(f"bench: {ms_step:.4f} ms/step, {mlups:.0f} MLUPS, {achieved:.0f} GB/s algorithmic")

    out = {
        "metric": "MLUPS",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic (seeded spruce-like medium)",
        "config": {"workload": f"miscible mixture {n}^3, {args.storage} populations, D=0.05, "
                               "spruce-like medium 100:1:1, hardening viscosity, Darcy+Forchheimer, "
                               "inlet/outlet reservoirs", "grid": [n, n, n], "cells": ncell,
                   "diag_every": 100},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(f"k_step miscible {n} {args.storage}"),
                     "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_GB_per_launch": round(bpl * ncell / 1e9, 4),
                     "bytes_per_lup": bpl, "kernel": "k_step<miscible>"},
        "diag_final": {"sum_rho": dg[0], "sum_epsC": dg[4], "max_v": dg[6], "nonfinite": dg[7]},
    }
    if not args.no_reduced and args.storage == "f32":
        red = {}
        for st in ("bf16", "f16", "bf16s", "f16s"):
            ms2, dg2 = time_gpu(p, st, args.steps, args.warmup)
            s2 = ms2 / args.steps
            b2 = storage_bpl(st)
            red[st] = {"MLUPS": round(ncell * args.steps / (ms2 / 1e3) / 1e6, 1), "ms_per_step": round(s2, 5),
                       "bytes_per_lup": b2, "achieved_GBs": round(b2 * ncell / (s2 / 1e3) / 1e9, 1),
                       "speedup_vs_f32": round(ms_step / s2, 3),
                       "traffic_GB_per_launch": counter_traffic(f"k_step miscible {n} {st}")}
            log(f"bench: {st}: {s2:.4f} ms/step, speedup {ms_step / s2:.3f}")
        out["reduced_storage"] = red
    if not args.no_obstacles and args.storage == "f32":
        out["obstacles"] = obstacle_leg(p, min(args.steps, 300), args.warmup)
    if args.storage == "f32":
        out["plain_method_32"] = plain_method_leg()
        log(f"bench: plain method 32^3 FP64: {out['plain_method_32']}")
    if not args.no_inclined and args.storage == "f32":
        out["inclined_rings"] = inclined_leg(n, min(args.steps, 300), args.warmup)
    if not args.no_species and args.storage == "f32":
        out["two_solutes"] = species_leg(n, min(args.steps, 300), args.warmup)
    if not args.no_wood and args.storage == "f32":
        out["wood"] = wood_leg(n, min(args.steps, 300), args.warmup)
    if not args.no_freesurface and args.storage == "f32":
        out["free_surface"] = freesurface_leg(n, min(args.steps, 300), args.warmup)
    if args.precision:
        out["precision_form"] = precision_leg()
    elif not args.no_512 and args.storage == "f32":
        out["precision_512"] = precision_leg(512, timed=100, compare=False, placements=3)
    if not args.no_serve:
        single = {"f32": mlups} if args.storage == "f32" else {}
        if "reduced_storage" in out:
            single["bf16"] = out["reduced_storage"]["bf16"]["MLUPS"]
        out["serving"] = serving_leg(single_mlups=single, jsonl_path=args.serve_log)
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    if args.cpu_full:
        out["cpu_baseline_full"] = cpu_baseline_full(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
