"""Pins of the oracle's freeze-out (Cooper-Frye on the fixed-time surface,
massless Boltzmann particles, rapidity 0; the step the paper plans next,
section "Results", closing paragraph) against mathematics that does not go
through its formula:

- a static uniform medium: the thermal Boltzmann spectrum
  E dN/d^3p = g V/(2 pi hbar c)^3 exp(-p/T) in closed form, flat in phi,
  v_n = 0;
- a uniformly moving medium: the spectrum from u.p of the four-vectors,
  integrated over p_T by adaptive quadrature (scipy.integrate.quad), and the
  harmonics by quadrature of the Fourier integrals; dN/dy against the
  textbook integral int dpsi (1 - a cos psi)^-3 = pi (2 + a^2)/(1 - a^2)^(5/2);
- the p_T-differential rows integrated over p_T (Gauss-Legendre panels) give the p_T-
  integrated row;
- symmetries: an isotropic fireball on a cubic grid has v_1 = v_2 = v_3 = 0;
  the mirror images y -> -y and x -> -x flip the sine parts and the cosine
  parts of odd n; permuting the cells changes nothing (a fixed-time surface
  does not see positions);
- T_min removes exactly the cells below it.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O

HBARC = 0.1973269804
G_EOS = 47.5


def temperature(e):
    return (30.0 * e * HBARC ** 3 / (G_EOS * math.pi ** 2)) ** 0.25


def uniform(n, e, v, nn=0.5):
    prim = np.empty((5, n[2], n[1], n[0]))
    prim[0], prim[1], prim[2], prim[3], prim[4] = e, v[0], v[1], v[2], nn
    return prim


def test_static_medium_is_the_thermal_spectrum():
    n = (6, 5, 4)
    pb = O.Problem(n=n, dx=(0.1, 0.2, 0.3))
    e, dof = 7.5, 3.0
    U = O.prim_to_cons(pb, uniform(n, e, (0.0, 0.0, 0.0)))
    pts = [0.2, 1.0, 2.5]
    spec, harm, fx = O.freezeout(pb, U, n_phi=24, pt=pts, dof=dof, n_harm=6)
    assert fx == 0
    T = temperature(e)
    V = 6 * 5 * 4 * 0.1 * 0.2 * 0.3
    pref = dof * V / (2 * math.pi * HBARC) ** 3
    # E dN/d^3p = pref exp(-p/T); at y = 0 the p_T integral of p_T * that is 2 T^3 pref
    assert np.allclose(spec[0], pref * 2 * T ** 3, rtol=1e-13, atol=0)
    for j, p in enumerate(pts):
        assert np.allclose(spec[1 + j], pref * p * math.exp(-p / T), rtol=1e-13, atol=0)
    assert harm[0, 0, 0] == pytest.approx(2 * math.pi * pref * 2 * T ** 3, rel=1e-13)
    assert np.abs(harm[:, 1:]).max() < 1e-14


@pytest.mark.parametrize("v", [(0.6, 0.0, 0.0), (0.3, -0.45, 0.2), (-0.1, 0.7, -0.5)])
def test_moving_medium_against_quadrature(v):
    n = (3, 2, 2)
    pb = O.Problem(n=n)
    e, dof = 12.0, 2.0
    U = O.prim_to_cons(pb, uniform(n, e, v))
    n_phi, n_harm = 64, 6
    pts = [0.3, 1.7]
    spec, harm, _ = O.freezeout(pb, U, n_phi=n_phi, pt=pts, dof=dof, n_harm=n_harm)
    T = temperature(e)
    V = 12 * 1e-3
    pref = dof * V / (2 * math.pi * HBARC) ** 3
    gam = 1 / math.sqrt(1 - sum(c * c for c in v))
    u = np.array([gam, gam * v[0], gam * v[1], gam * v[2]])

    def u_dot_p(pT, phi):  # metric (+, -, -, -), p = (pT, pT cos, pT sin, 0)
        p = np.array([pT, pT * math.cos(phi), pT * math.sin(phi), 0.0])
        return u[0] * p[0] - u[1:] @ p[1:]

    def dn(phi):  # int_0^inf dpT pT * E dN/d^3p, E = pT at y = 0
        val, _ = integrate.quad(lambda pT: pT * pT * math.exp(-u_dot_p(pT, phi) / T), 0, np.inf,
                                epsabs=0, epsrel=1e-13, limit=200)
        return pref * val

    for k in (0, 5, 17, 40, 63):
        phi = 2 * math.pi * k / n_phi
        assert spec[0, k] == pytest.approx(dn(phi), rel=1e-11)
        for j, p in enumerate(pts):
            assert spec[1 + j, k] == pytest.approx(pref * p * math.exp(-u_dot_p(p, phi) / T), rel=1e-12)
    # harmonics: Fourier integrals of the closed-form azimuthal distribution by quadrature
    a = math.hypot(v[0], v[1])
    f = lambda phi: 1.0 / (gam * (1 - v[0] * math.cos(phi) - v[1] * math.sin(phi))) ** 3
    tot, _ = integrate.quad(f, 0, 2 * math.pi, epsabs=0, epsrel=1e-13, limit=200)
    for m in range(1, n_harm + 1):
        c, _ = integrate.quad(lambda p: math.cos(m * p) * f(p), 0, 2 * math.pi, epsabs=1e-15, epsrel=1e-12, limit=400)
        s, _ = integrate.quad(lambda p: math.sin(m * p) * f(p), 0, 2 * math.pi, epsabs=1e-15, epsrel=1e-12, limit=400)
        assert harm[0, m, 0] == pytest.approx(c / tot, abs=1e-11)
        assert harm[0, m, 1] == pytest.approx(s / tot, abs=1e-11)
    # dN/dy: 2 T^3 pref / gamma^3 * int dpsi (1 - a cos psi)^-3 = pi (2 + a^2) / (1 - a^2)^(5/2)
    closed = pref * 2 * T ** 3 / gam ** 3 * math.pi * (2 + a * a) / (1 - a * a) ** 2.5
    assert harm[0, 0, 0] == pytest.approx(closed, rel=1e-12)
    # the elliptic and directed flow point along the transverse velocity
    if a > 0:
        psi1 = math.atan2(harm[0, 1, 1], harm[0, 1, 0])
        assert math.cos(psi1 - math.atan2(v[1], v[0])) == pytest.approx(1.0, abs=1e-12)


def random_event(n, seed, vmax=0.7):
    rng = np.random.default_rng(seed)
    prim = np.empty((5, n[2], n[1], n[0]))
    prim[0] = rng.uniform(0.5, 40.0, size=prim[0].shape)
    v = rng.uniform(-1, 1, size=(3,) + prim[0].shape)
    v *= vmax * rng.uniform(0, 1, size=prim[0].shape) / np.maximum(np.sqrt((v * v).sum(0)), 1e-12)
    prim[1:4] = v
    prim[4] = rng.uniform(0.1, 1.0, size=prim[0].shape)
    return prim


def test_pt_rows_integrate_to_the_integrated_row():
    n = (4, 3, 3)
    pb = O.Problem(n=n)
    U = O.prim_to_cons(pb, random_event(n, 3))
    # composite 30-point Gauss-Legendre on the panels [0, 0.005], then
    # doubling panels up to 82 GeV (every integrand below is e^-40 there)
    x, wgt = np.polynomial.legendre.leggauss(30)
    edges = [0.0] + [0.005 * 2.0 ** k for k in range(15)]
    pts, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        pts.append(0.5 * (b - a) * x + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * wgt)
    pts, ws = np.concatenate(pts), np.concatenate(ws)
    spec, _, _ = O.freezeout(pb, U, n_phi=8, pt=pts, n_harm=0)
    approx = (spec[1:] * (pts * ws)[:, None]).sum(0)
    assert np.allclose(approx, spec[0], rtol=1e-12, atol=0)


def isotropic_fireball(n, dx):
    c = (np.arange(n) - 0.5 * (n - 1)) * dx
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r2 = x * x + y * y + z * z
    prim = np.empty((5, n, n, n))
    prim[0] = 25 * np.exp(-r2 / (2 * 0.6 ** 2)) + 1e-3
    prim[1], prim[2], prim[3] = 0.08 * x, 0.08 * y, 0.08 * z
    prim[4] = 0.5
    return prim


def test_isotropic_fireball_has_no_low_harmonics():
    n = 16
    pb = O.Problem(n=(n, n, n))
    U = O.prim_to_cons(pb, isotropic_fireball(n, 0.1))
    _, harm, _ = O.freezeout(pb, U, n_phi=32, pt=[0.5, 2.0], n_harm=4)
    assert np.abs(harm[:, 1:4, :]).max() < 1e-13
    assert np.abs(harm[:, 4, 1]).max() < 1e-13  # the square grid allows only cos 4 phi


def test_mirror_images_and_permutations():
    n = (6, 5, 4)
    pb = O.Problem(n=n)
    prim = random_event(n, 11)
    kw = dict(n_phi=16, pt=[0.4, 1.3], n_harm=5)
    spec, harm, _ = O.freezeout(pb, O.prim_to_cons(pb, prim), **kw)
    # y -> -y
    py = prim[:, :, ::-1, :].copy()
    py[2] = -py[2]
    sy, hy, _ = O.freezeout(pb, O.prim_to_cons(pb, py), **kw)
    idx = (-np.arange(16)) % 16
    assert np.allclose(sy, spec[:, idx], rtol=1e-13, atol=0)
    assert np.allclose(hy[:, :, 0], harm[:, :, 0], rtol=0, atol=1e-14)
    assert np.allclose(hy[:, 1:, 1], -harm[:, 1:, 1], rtol=0, atol=1e-14)
    # x -> -x: phi -> pi - phi
    px = prim[:, :, :, ::-1].copy()
    px[1] = -px[1]
    sx, hx, _ = O.freezeout(pb, O.prim_to_cons(pb, px), **kw)
    idx = (8 - np.arange(16)) % 16
    assert np.allclose(sx, spec[:, idx], rtol=1e-13, atol=0)
    sign = np.array([(-1.0) ** m for m in range(6)])
    assert np.allclose(hx[:, :, 0], harm[:, :, 0] * sign, rtol=0, atol=1e-14)
    assert np.allclose(hx[:, :, 1], -harm[:, :, 1] * sign, rtol=0, atol=1e-14)
    # any permutation of the cells
    perm = np.random.default_rng(5).permutation(np.prod(n))
    pp = prim.reshape(5, -1)[:, perm].reshape(prim.shape)
    sp, _, _ = O.freezeout(pb, O.prim_to_cons(pb, pp), **kw)
    assert np.allclose(sp, spec, rtol=1e-13, atol=0)


def test_tmin_drops_exactly_the_cold_cells():
    n = (8, 4, 2)
    pb = O.Problem(n=n)
    prim = random_event(n, 17)
    prim[0, :, :, :4] = 1e-3  # cold half (T ~ 26 MeV)
    T_min = 0.1
    spec, _, _ = O.freezeout(pb, O.prim_to_cons(pb, prim), n_phi=12, pt=[1.0], T_min=T_min)
    half = O.Problem(n=(4, 4, 2))
    ph = np.ascontiguousarray(prim[:, :, :, 4:])
    sh, _, _ = O.freezeout(half, O.prim_to_cons(half, ph), n_phi=12, pt=[1.0])
    assert np.allclose(spec, sh, rtol=1e-13, atol=0)
    full, _, _ = O.freezeout(pb, O.prim_to_cons(pb, prim), n_phi=12, pt=[1.0])
    assert np.all(full > spec)
    # T_min above every cell: no particles, dN/dy and every v_n zero (not 0/0)
    none, harm, _ = O.freezeout(pb, O.prim_to_cons(pb, prim), n_phi=12, pt=[1.0], T_min=100.0, n_harm=4)
    assert np.all(none == 0.0) and np.all(harm == 0.0)
