"""Seeded input generators (no GPU): the counter-based generator, the
spruce-like medium and the request stream."""
import math

import numpy as np
import pytest

from paper_0912_4230_amd import inputs as I


def test_splitmix64_published_sequence():
    """The first outputs of SplitMix64 from state 0 (Steele, Lea, Flood 2014)."""
    g = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        xs = np.array([0, g, g * np.uint64(2)], dtype=np.uint64)
    out = [int(v) for v in I.splitmix64(xs)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_normals_are_standard():
    x = np.arange(200000) % 400
    y = np.arange(200000) // 400
    xi = I.cell_normal(5, x, y, np.zeros_like(x))
    assert abs(xi.mean()) < 0.01
    assert abs(xi.std() - 1) < 0.01
    assert abs(np.mean(xi ** 4) - 3) < 0.05


def test_medium_crop_equals_full():
    eps, kinv = I.spruce_medium((40, 24, 16), seed=3, ratio=100.0)
    ec, kc = I.spruce_medium((13, 9, 7), seed=3, ratio=100.0, origin=(20, 10, 5))
    assert np.array_equal(ec, eps[5:12, 10:19, 20:33])
    assert np.array_equal(kc, kinv[:, 5:12, 10:19, 20:33])


def test_medium_structure():
    eps, kinv = I.spruce_medium((64, 8, 8), seed=0, ratio=100.0)
    assert eps.min() >= 0.4 - 1e-12 and eps.max() <= 0.8 + 1e-12
    # sinusoid of period 32 along x only
    assert np.allclose(eps[:, :, :32], eps[:, :, 32:])
    assert np.allclose(eps, eps[:1, :1, :])
    # anisotropy exactly 100:1:1 (longitudinal y : radial x : tangential z)
    assert np.allclose(kinv[0] / kinv[1], 100.0, rtol=1e-14)
    assert np.array_equal(kinv[0], kinv[2])
    # the porosity dependence of Eq. Ktensor
    assert abs(I.kappa(0.4) / I.kappa(0.6) - 0.1005) < 1e-3
    assert abs(I.kappa(0.8) / I.kappa(0.6) - 11.48) < 1e-2
    # lognormal noise of sigma 0.3 around the banded mean
    x = np.arange(64)
    band = 1e-2 * I.kappa(eps[0, 0]) / I.kappa(0.6)
    logn = np.log((1.0 / kinv[1]) / band[None, None, :])
    assert abs(logn.std() - 0.3) < 0.02


def test_request_stream():
    reqs = I.request_stream()
    assert len(reqs) == 64
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert abs(len(reqs) / arr[-1] - 4.0) < 1.5
    edges = np.array([r.edge for r in reqs])
    assert edges.min() >= 48 and edges.max() <= 192
    mis = np.mean([r.physics == I.MISCIBLE for r in reqs])
    assert 0.5 < mis < 0.9
    assert all(500 <= r.steps <= 5000 for r in reqs)
    assert reqs == I.request_stream()


def test_problem_shapes():
    p = I.miscible(shape=(20, 12, 8))
    assert p.eps.shape == (8, 12, 20) and p.kinv.shape == (3, 8, 12, 20)
    assert p.faces[0].kind == I.RESERVOIR and math.isclose(p.faces[0].rho, 1 + 3 * 0.0441)
    d = I.drop(shape=(32, 32, 32), radius=5)
    assert d.c0.sum() == (np.sum((np.indices((32, 32, 32)) - 16) ** 2, axis=0) <= 25).sum()
    assert d.faces[4].kind == I.WALL and d.faces[4].angle == 120.0


def test_block_obstacles_crop_and_fraction():
    a = I.block_obstacles((40, 30, 20), seed=0, free_x=0)
    b = I.block_obstacles((20, 10, 8), seed=0, origin=(8, 12, 4), free_x=0)
    assert np.array_equal(a[4:12, 12:22, 8:28], b)
    m = I.block_obstacles((64, 64, 64), seed=1, solid_fraction=0.25)
    assert 0.18 < m.mean() < 0.3
    assert not m[:, :, :2].any() and not m[:, :, -2:].any()
    # whole 4^3 cubes
    c = m[:, :, 4:60].reshape(16, 4, 16, 4, 14, 4)
    assert np.all(c.min(axis=(1, 3, 5)) == c.max(axis=(1, 3, 5)))


def test_field_shapes_checked_before_upload():
    """Simulation refuses arrays that do not have the shapes the kernels
    read (the C ABI takes device pointers without sizes): here the initial
    concentrations of a three-solute problem with one plane too few."""
    from paper_0912_4230_amd.sim import check_fields
    p = I.miscible(shape=(12, 10, 8), seed=0)
    p.species_tau_d = (0.65, 0.8)
    p.c0 = np.zeros((3, 8, 10, 12))
    check_fields(p)
    p.c0 = np.zeros((2, 8, 10, 12))
    with pytest.raises(ValueError, match="c0"):
        check_fields(p)
    q = I.miscible(shape=(12, 10, 8), seed=0)
    q.kinv = q.kinv[:2]
    with pytest.raises(ValueError, match="kinv"):
        check_fields(q)
    r = I.miscible(shape=(12, 10, 8), seed=0, ring_angle=45.0)
    check_fields(r)
