"""The oracle's pins have teeth: each plausible mistake below, planted in a
temporary copy of oracle/lbm_oracle.c (the oracle itself stays as it is), is
caught by the pin named beside it (no GPU).

Each entry replaces one exact piece of the oracle's source (it must occur
exactly once), builds the copy with the oracle's own compiler flags and runs
the pin against it; the pin must fail with an assertion, i.e. by computing a
wrong number, not by crashing.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

import test_oracle_flows as FL
import test_oracle_freesurface as FS
import test_oracle_identities as ID
import test_oracle_reservoirs as RS
import test_oracle_species as SP
import test_oracle_transport as TR
import test_oracle_twofluid as TF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")

# (name, original text, planted text, pin that must fail, its arguments)
PLANTS = [
    # reservoir planes (Sec. 4 pressure inlet / outlet, reading of fixed equilibria)
    ("solute reservoir without the porosity",
     "ho[q] = WGT[q] * s->eps[i] * cb;", "ho[q] = WGT[q] * cb;",
     RS.test_solute_reservoirs_exact_linear_profile, {}),
    ("second solute's reservoir without the porosity",
     "xo[q] = WGT[q] * s->eps[i] * C;", "xo[q] = WGT[q] * C;",
     RS.test_solute_reservoirs_exact_linear_profile, {}),
    ("two-fluid reservoir without its density",
     "ho[q] = cb * WGT[q] * rb;", "ho[q] = cb * WGT[q];",
     RS.test_two_fluid_reservoirs_exact_linear_colour, {}),
    ("solute advected with V instead of the corrected V'",
     "double D = solute_D(p), vs[3] = {Vp[0], Vp[1], Vp[2]};", "double D = solute_D(p), vs[3] = {V[0], V[1], V[2]};",
     RS.test_solute_reservoirs_with_flow_advection_diffusion, {}),
    # two-fluid mixture viscosity (reading of the two-fluid model)
    ("two-fluid viscosities swapped",
     "return C * nu1 + (1.0 - C) * nu2;", "return C * nu2 + (1.0 - C) * nu1;",
     TF.test_layered_channel_flow_mixture_viscosity, {}),
    ("two-fluid harmonic mixture viscosity",
     "return C * nu1 + (1.0 - C) * nu2;", "return 1.0 / (C / nu1 + (1.0 - C) / nu2);",
     TF.test_layered_channel_flow_mixture_viscosity, {}),
    # hydrodynamic lattice (Sec. 2.1)
    ("no porosity on G in V' (the printed Eq. expandVsub)",
     "W[a] = V[a] + 0.5 * eps * p->G[a];\n        lam[a]", "W[a] = V[a] + 0.5 * p->G[a];\n        lam[a]",
     FL.test_paper_anisotropic_darcy_plateau, {"case": "x"}),
    ("forcing terms without the weight w_i rho",
     "out[q] = WGT[q] * rho * pre * (3.0 * vF", "out[q] = pre * (3.0 * vF",
     ID.test_forcing_moments, {"seed": 0}),
    ("density without the rest population",
     "        drho += fin[q];\n", "        if (q) drho += fin[q];\n",
     TR.test_conservation_periodic_miscible, {}),
    ("collision with the wrong sign",
     "fout[q] = fin[q] - (fin[q] - eq[q]) / tau + T[q];", "fout[q] = fin[q] + (fin[q] - eq[q]) / tau + T[q];",
     FL.test_c1_channel_plateau_and_profile, {}),
    ("bounce-back into the same direction",
     "return L[(long)OPP[q] * s->n + i0];", "return L[(long)q * s->n + i0];",
     FL.test_poiseuille_exact_parabola, {}),
    ("Forchheimer drag with the wrong sign",
     "- eps * Feps * sp * sqrt(kinv[a]) * Vp[a];", "+ eps * Feps * sp * sqrt(kinv[a]) * Vp[a];",
     FL.test_darcy_forchheimer_uniform_balance, {}),
    # solute lattice (Sec. 2.2)
    ("porosity gradient stencil without its factor 3",
     "g[a] += 3.0 * WGT[q] * e * VEL[q][a];", "g[a] += WGT[q] * e * VEL[q][a];",
     TR.test_porous_diffusion_uniform_concentration, {}),
    ("solute diffusivity tau_d / 3",
     "return (p->tau_d - 0.5) / 3.0; }", "return p->tau_d / 3.0; }",
     TR.test_porous_diffusion_uniform_concentration, {}),
    # several solutes
    ("further solute relaxes with the first solute's tau_d",
     "double tau_d = p->tau_dx[k - 1];", "double tau_d = p->tau_d;",
     SP.test_two_solutes_follow_their_own_variance_laws, {}),
    ("further solute drifts with the first solute's D",
     "double D = (tau_d - 0.5) / 3.0, vs[3] = {Vp[0], Vp[1], Vp[2]};",
     "double D = solute_D(p), vs[3] = {Vp[0], Vp[1], Vp[2]};",
     SP.test_porous_diffusion_of_each_solute, {}),
    ("further solute starts from the first solute's plane",
     "C = c0[(size_t)k * n + i];", "C = c0[i];",
     SP.test_each_solute_conserved, {}),
    # free surface (Sec. 3)
    ("mass exchange with the wrong sign",
     "double flux = Fc[(long)OPP[q] * n + j] - own[q];", "double flux = own[q] - Fc[(long)OPP[q] * n + j];",
     FS.test_slab_translates_with_its_velocity, {"speed": 0.05}),
    ("exchange weighted by lambda(x) instead of the mean",
     "flux * 0.5 * (s->lam[i] + s->lam[j]);", "flux * s->lam[i];",
     FS.test_mass_conserved_through_fall_and_impact, {}),
    ("the printed mean weight also on links to liquid cells",
     "dm += s->fst[j] == FS_LIQ ? flux : flux * 0.5 * (s->lam[i] + s->lam[j]);",
     "dm += flux * 0.5 * (s->lam[i] + s->lam[j]);",
     FS.test_mass_conserved_through_fall_and_impact, {}),
    ("reconstruction from f~_i instead of f~_opp(i)",
     "fin[q] = eqA[q] + eqA[OPP[q]] - own[OPP[q]];", "fin[q] = eqA[q] + eqA[OPP[q]] - own[q];",
     FS.test_slab_translates_with_its_velocity, {"speed": 0.05}),
    ("gas density 1.001",
     "#define FS_RHO_A 1.0", "#define FS_RHO_A 1.001",
     FS.test_hydrostatic_pool, {}),
    ("excess shared over k + 1 cells",
     "share[i] = k > 0 ? ex / k : 0.0;", "share[i] = k > 0 ? ex / (k + 1) : 0.0;",
     FS.test_mass_conserved_through_fall_and_impact, {}),
]


def _build(src_text, out_dir, k):
    c = os.path.join(out_dir, f"planted_{k}.c")
    so = os.path.join(out_dir, f"libplanted_{k}.so")
    with open(c, "w") as f:
        f.write(src_text)
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", so, c, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return so


@pytest.fixture(scope="module")
def planted_libs(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    src = open(SRC).read()
    out = str(tmp_path_factory.mktemp("planted"))
    texts = []
    for name, old, new, _, _ in PLANTS:
        assert src.count(old) == 1, f"{name}: the original text must occur exactly once"
        texts.append(src.replace(old, new))
    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as pool:
        return list(pool.map(lambda a: _build(a[1], out, a[0]), enumerate(texts)))


@pytest.mark.parametrize("k", range(len(PLANTS)), ids=[p[0] for p in PLANTS])
def test_planted_mistake_is_caught(orc, planted_libs, k):
    name, old, new, pin, kwargs = PLANTS[k]
    with orc.library(planted_libs[k]):
        with pytest.raises(AssertionError):
            pin(orc, **kwargs)
