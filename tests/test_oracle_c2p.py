"""Pins of the oracle's conserved<->primitive maps and T(e) (CPU only)."""
import math

import numpy as np
import pytest

import oracle as O


def random_prims(rng, n, vmax=0.9):
    e = 10.0 ** rng.uniform(-3, 2, size=n)
    d = rng.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    speed = vmax * rng.random(n) ** 0.5
    v = d * speed
    nn = 10.0 ** rng.uniform(-2, 1, size=n)
    return np.stack([e, v[0], v[1], v[2], nn])


def test_round_trip_prim_cons_prim():
    rng = np.random.default_rng(0)
    pb = O.Problem(n=(1000, 1, 1))
    prim = random_prims(rng, 1000).reshape(5, 1, 1, 1000)
    U = O.prim_to_cons(pb, prim)
    back, fx = O.cons_to_prim(pb, U)
    assert fx == 0
    v2 = (prim[1:4] ** 2).sum(0)
    g2 = 1.0 / (1.0 - v2)
    tol = 8e-16 * g2
    assert np.all(np.abs(back[0] - prim[0]) <= tol * prim[0] * 4)
    for d in range(3):
        assert np.all(np.abs(back[1 + d] - prim[1 + d]) <= 8 * tol)
    assert np.all(np.abs(back[4] - prim[4]) <= 8 * tol * prim[4])


def test_energy_density_solves_the_quadratic():
    # With W = E + p and p = e/3: e^2 + 2 E e - 3 E^2 + 3 M^2 = 0.
    rng = np.random.default_rng(1)
    pb = O.Problem(n=(500, 1, 1))
    U = np.empty((5, 1, 1, 500))
    E = 10.0 ** rng.uniform(-2, 2, 500)
    frac = rng.random(500) * 0.999
    d = rng.normal(size=(3, 500))
    d /= np.linalg.norm(d, axis=0)
    U[0, 0, 0] = E
    U[1:4, 0, 0] = d * frac * E
    U[4, 0, 0] = 1.0
    prim, fx = O.cons_to_prim(pb, U)
    assert fx == 0
    e = prim[0, 0, 0]
    M2 = (U[1:4, 0, 0] ** 2).sum(0)
    resid = e * e + 2 * E * e - 3 * E * E + 3 * M2
    assert np.all(np.abs(resid) <= 1e-13 * E * E)
    # and v = M / (E + e/3)
    for k in range(3):
        assert np.allclose(prim[1 + k, 0, 0], U[1 + k, 0, 0] / (E + e / 3), rtol=1e-14, atol=0)


def test_rest_frame_identity():
    pb = O.Problem(n=(3, 1, 1))
    U = np.zeros((5, 1, 1, 3))
    U[0] = [[[1.0, 7.5, 30.0]]]
    U[4] = [[[0.1, 0.2, 0.3]]]
    prim, fx = O.cons_to_prim(pb, U)
    assert fx == 0
    assert np.array_equal(prim[0], U[0])
    assert np.array_equal(prim[4], U[4])
    assert np.all(prim[1:4] == 0.0)


def test_temperature_closed_form():
    # e = g pi^2/30 T^4/(hbar c)^3 with g = 47.5: T(30 GeV/fm^3) = 0.3485 GeV
    pb = O.Problem(n=(4, 1, 1))
    e = np.array([1e-3, 1.0, 30.0, 1000.0])
    U = np.zeros((5, 1, 1, 4))
    U[0, 0, 0] = e
    prim, _ = O.cons_to_prim(pb, U)
    T = prim[5, 0, 0]
    hc = 0.1973269804
    back = 47.5 * math.pi ** 2 / 30.0 * T ** 4 / hc ** 3
    assert np.allclose(back, e, rtol=1e-14)
    assert abs(T[2] - 0.3485) < 5e-4


def test_fixups_counted_and_admissible():
    pb = O.Problem(n=(3, 1, 1))
    U = np.zeros((5, 1, 1, 3))
    U[0, 0, 0] = [-1.0, 1.0, 2.0]
    U[1, 0, 0] = [0.0, 1.5, 0.5]   # |M| > E in cell 1
    U[4] = 1.0
    prim, fx = O.cons_to_prim(pb, U)
    assert fx == 2
    assert prim[0, 0, 0, 0] == pytest.approx(1e-12)
    assert np.all(np.abs(prim[1:4]) < 1.0)
    assert np.all(prim[0] > 0)
