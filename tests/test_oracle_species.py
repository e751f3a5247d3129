"""Pins of the oracle's several solutes (no GPU).

Sec. 2.2 builds the solute on its own lattice "to simplify a later extension
to various species": every solute k has its own populations, relaxation time
tau_d,k (D_k = (tau_d,k - 1/2)/3) and reservoir concentrations, and follows
Eqs. equild and boltzeqD with the shared velocity V'.  The viscosity law reads
the first solute's concentration.  What fixes it:

- a second solute identical to the first (same D, initial and boundary values)
  is the first, bit for bit, and the flow is that of the one-solute run;
- two solutes with different D released from one point source follow their
  own discrete variance laws at the same time (exact to 1e-12);
- each solute's mass Sum eps C_k is conserved separately in a periodic
  heterogeneous medium;
- the flow depends on the first solute only (viscosity law), not on the others.
"""
import numpy as np

from paper_0912_4230_amd import inputs as I


def _miscible(shape, species_tau_d=(), seed=0):
    p = I.miscible(shape=shape, seed=seed, reservoirs=False)
    p.species_tau_d = tuple(species_tau_d)
    p.G = (2e-4, -1e-4, 5e-5)
    return p


def test_identical_second_solute_is_the_first(orc):
    shape = (12, 10, 8)
    p1 = I.miscible(shape=shape, seed=3)
    p2 = I.miscible(shape=shape, seed=3)
    p2.species_tau_d = (p1.tau_d,)
    for f in p2.faces:
        f.conc_x = (f.conc,)
    rng = np.random.default_rng(1)
    c = rng.random((8, 10, 12))
    p1.c0 = c.copy()
    p2.c0 = np.stack([c, c])
    a = orc.Oracle(p1).step(60)
    b = orc.Oracle(p2).step(60)
    ra, va, ca = a.moments()
    rb, vb, cb = b.moments()
    assert np.array_equal(ra, rb) and np.array_equal(va, vb) and np.array_equal(ca, cb)
    assert np.array_equal(b.species_conc(1), cb)
    assert np.array_equal(b.get_state(2), b.get_state(1))
    assert np.array_equal(a.get_state(1), b.get_state(1))


def _variance(eps, c, x):
    m = (eps * c).reshape(-1)
    M = m.sum()
    mu = (m * x).sum() / M
    return ((x - mu) ** 2 * m).sum() / M


def test_two_solutes_follow_their_own_variance_laws(orc):
    nx = 500
    taus = (0.65, 1.3)
    p = I.Problem(shape=(nx, 1, 1), physics=I.MISCIBLE, tau_d=taus[0], species_tau_d=(taus[1],)).fill_defaults()
    p.eps[:] = 0.7
    p.c0[:, 0, 0, nx // 2] = 1.0
    o = orc.Oracle(p)
    x = np.arange(nx, dtype=float)
    v0 = [_variance(p.eps, o.species_conc(k), x) for k in (0, 1)]
    for t in (1, 3, 10, 40, 150):
        o.step(t - o.steps_done)
        for k, tau in enumerate(taus):
            D = (tau - 0.5) / 3.0
            vt = _variance(p.eps, o.species_conc(k), x)
            pred = 2 * D * t - (2 * tau * (tau - 1) / 3) * (1 - (1 - 1 / tau) ** t)
            assert abs((vt - v0[k]) - pred) <= 1e-12 * pred, (k, t)


def test_each_solute_conserved(orc):
    shape = (11, 9, 7)
    p = _miscible(shape, species_tau_d=(0.9, 0.55, 1.7), seed=4)
    rng = np.random.default_rng(2)
    p.c0 = rng.random((4, 7, 9, 11))
    o = orc.Oracle(p)
    t0 = o.species_totals()
    assert len(t0) == 4 and (t0 > 0).all()
    # the initial fields are the inputs, solute by solute
    for k in range(4):
        assert np.array_equal(o.species_conc(k), p.c0[k])
        assert abs(t0[k] - (p.eps * p.c0[k]).sum()) <= 1e-13 * t0[k]
    o.step(150)
    t1 = o.species_totals()
    assert np.abs(t1 - t0).max() <= 1e-12 * t0.max()
    # the concentrations have evolved differently
    assert np.abs(o.species_conc(2) - o.species_conc(3)).max() > 1e-3


def test_flow_reads_the_first_solute_only(orc):
    shape = (10, 8, 6)
    base = _miscible(shape, species_tau_d=(0.8,), seed=5)
    rng = np.random.default_rng(3)
    c = rng.random((2, 6, 8, 10))
    base.c0 = c.copy()
    other = _miscible(shape, species_tau_d=(0.8,), seed=5)
    other.c0 = c.copy()
    other.c0[1] = rng.random((6, 8, 10))     # another second solute
    first = _miscible(shape, species_tau_d=(0.8,), seed=5)
    first.c0 = c.copy()
    first.c0[0] = rng.random((6, 8, 10))     # another first solute
    ra, va, _ = orc.Oracle(base).step(40).moments()
    rb, vb, _ = orc.Oracle(other).step(40).moments()
    rc, vc, _ = orc.Oracle(first).step(40).moments()
    assert np.array_equal(ra, rb) and np.array_equal(va, vb)
    assert np.abs(vc - va).max() > 1e-3 * np.abs(va).max()


def test_porous_diffusion_of_each_solute(orc):
    """Uniform concentrations over a heterogeneous porosity at rest stay
    uniform for every solute, each with its own drift D_k grad(eps)/eps
    (Eq. equild); the solutes have different D."""
    nx = 64
    p = I.Problem(shape=(nx, 1, 1), physics=I.MISCIBLE, tau_d=0.8, species_tau_d=(1.4, 0.6)).fill_defaults()
    x = np.arange(nx)
    p.eps[0, 0] = 0.6 + 0.2 * np.sin(2 * np.pi * x / 32.0)
    p.c0[:] = 0.5
    p.kinv[:] = 1e6
    o = orc.Oracle(p).step(3000)
    for k in range(3):
        assert np.abs(o.species_conc(k) - 0.5).max() < 3e-3, k
