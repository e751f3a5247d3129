"""Shared helpers of the GPU tests: run the GPU library and the FP64 oracle on
the same seeded problem and compare fields over fluid cells."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def ensure_built():
    from paper_0912_4230_amd import binding
    from oracle import oracle
    if not os.path.exists(binding.LIB_PATH) or not os.path.exists(oracle.LIB_PATH):
        sys.path.insert(0, ROOT)
        import __graft_entry__
        __graft_entry__.build()


def rel_l2(a, b, mask):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.ndim == 4:
        a = a[:, mask]
        b = b[:, mask]
    else:
        a = a[mask]
        b = b[mask]
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def run_pair(problem, steps, storage, chunks=None, diag_every=0):
    """Run the GPU and the oracle for `steps` steps (in `chunks` calls on the
    GPU side); return (gpu fields, oracle fields, fluid mask, gpu diag, oracle diag)."""
    from oracle import oracle as O
    from paper_0912_4230_amd.sim import Simulation
    sim = Simulation(problem, storage=storage, diag_every=diag_every)
    chunks = chunks or [steps]
    assert sum(chunks) == steps
    for c in chunks:
        sim.step(c)
    rho, vel, conc, dg = sim.moments()
    g = (rho.double().cpu().numpy(), vel.double().cpu().numpy(), conc.double().cpu().numpy())
    o = O.Oracle(problem)
    o.step(steps)
    r = o.moments()
    od = o.diag()
    mask = o.cell_types() == 0
    sim.close()
    o.close()
    return g, r, mask, dg, od


def errors(g, r, mask):
    return {
        "rho": rel_l2(g[0], r[0], mask),
        "drho": rel_l2(g[0] - 1.0, r[0] - 1.0, mask),
        "vel": rel_l2(g[1], r[1], mask),
        "conc": rel_l2(g[2], r[2], mask),
    }


def report(name, errs):
    print(f"[parity] {name}: " + ", ".join(f"{k}={v:.3e}" for k, v in errs.items()), flush=True)


def permutation_to_oracle():
    """perm[q_gpu] = q_oracle with equal velocity vectors."""
    from oracle import oracle as O
    from paper_0912_4230_amd import binding as B
    vg, _ = B.lbm_lattice()
    vo, _, _ = O.lattice()
    vo = [tuple(int(c) for c in v) for v in vo]
    return np.array([vo.index(tuple(v)) for v in vg])
