"""Pins of the oracle's WENO5 reconstruction, the 5th-order alternative the
paper names beside WENO7 (CPU only).

As for WENO7, the constants are re-derived with sympy from their
definitions: candidate values of the 3-cell quadratics with the given cell
averages, Jiang-Shu smoothness indicators sum_l dx^(2l-1) int (p^(l))^2, and
ideal weights from matching the 5-cell quartic.  The nonlinear schemes are
further pinned by polynomial exactness, the ENO property, symmetry and order,
and the full scheme by its 5th-order spatial convergence.
"""
import functools
import math

import numpy as np
import pytest
import sympy as sp

import oracle as O
from test_oracle_scheme import exact_flux_derivative, smooth_1d_prim


@functools.lru_cache(maxsize=None)
def derived():
    x = sp.symbols("x")
    f = sp.symbols("f0:5")  # a_{i-2}..a_{i+2}; cell i spans [-1/2, 1/2]
    half = sp.Rational(1, 2)

    def poly_with_averages(offsets):
        deg = len(offsets)
        a = sp.symbols("c0:%d" % deg)
        p = sum(a[m] * x ** m for m in range(deg))
        eqs = [sp.integrate(p, (x, o - half, o + half)) - f[o + 2] for o in offsets]
        return sp.expand(p.subs(sp.solve(eqs, a)))

    q, beta = [], []
    for k in range(3):
        pk = poly_with_averages(list(range(-2 + k, 1 + k)))
        q.append(sp.expand(pk.subs(x, half)))
        beta.append(sp.expand(sum(sp.integrate(sp.diff(pk, x, l) ** 2, (x, -half, half)) for l in range(1, 3))))
    p5 = poly_with_averages(list(range(-2, 3)))
    target = sp.expand(p5.subs(x, half))
    d = sp.symbols("d0:3")
    eqs = sp.Poly(sp.expand(sum(d[k] * q[k] for k in range(3)) - target), *f).coeffs()
    dsol = sp.solve(eqs, d)
    return f, q, beta, [dsol[d[k]] for k in range(3)]


def ref_weno5(vals, scheme, eps=1e-6, p=2):
    f, q, beta, dvals = derived()
    sub = dict(zip(f, [sp.Float(v, 40) for v in vals]))
    qv = [q[k].evalf(40, subs=sub) for k in range(3)]
    bv = [beta[k].evalf(40, subs=sub) for k in range(3)]
    d = [sp.Float(dv, 40) for dv in dvals]
    if scheme == "linear":
        return float(sum(d[k] * qv[k] for k in range(3)))
    if scheme == "js":
        a = [d[k] / (eps + bv[k]) ** 2 for k in range(3)]
    else:
        tau = abs(bv[0] - bv[2])
        a = [d[k] * (1 + (tau / (bv[k] + eps)) ** p) for k in range(3)]
    s = sum(a)
    return float(sum(a[k] / s * qv[k] for k in range(3)))


def test_ideal_weights_are_1_6_3_over_10():
    *_, dvals = derived()
    assert [sp.nsimplify(v) for v in dvals] == [sp.Rational(1, 10), sp.Rational(6, 10), sp.Rational(3, 10)]


def test_smoothness_indicators_are_the_jiang_shu_forms():
    f, _, beta, _ = derived()
    a, b, c, d, e = f
    js = [sp.Rational(13, 12) * (a - 2 * b + c) ** 2 + sp.Rational(1, 4) * (a - 4 * b + 3 * c) ** 2,
          sp.Rational(13, 12) * (b - 2 * c + d) ** 2 + sp.Rational(1, 4) * (b - d) ** 2,
          sp.Rational(13, 12) * (c - 2 * d + e) ** 2 + sp.Rational(1, 4) * (3 * c - 4 * d + e) ** 2]
    for k in range(3):
        assert sp.expand(beta[k] - js[k]) == 0


@pytest.mark.parametrize("scheme", ["linear", "js", "z"])
def test_matches_definition_on_random_data(scheme):
    rng = np.random.default_rng(12)
    for trial in range(40):
        scale = 10.0 ** rng.uniform(-3, 2)
        vals = rng.normal(size=5) * scale + (scale if trial % 2 else 0.0)
        got = O.weno5(vals, scheme)
        ref = ref_weno5(vals, scheme)
        assert abs(got - ref) <= 1e-13 * max(1.0, np.abs(vals).max()), (trial, got, ref)


def cell_averages(coeffs, centres, h):
    out = np.zeros_like(centres)
    for m, c in enumerate(coeffs):
        F = lambda t: t ** (m + 1) / (m + 1)
        out += c * (F(centres + h / 2) - F(centres - h / 2)) / h
    return out


@pytest.mark.parametrize("degree", range(0, 7))
def test_linear_weights_face_value_exact_up_to_degree_4(degree):
    rng = np.random.default_rng(70 + degree)
    coeffs = rng.normal(size=degree + 1)
    dx = 0.25
    fv = cell_averages(coeffs, np.arange(-2, 3) * dx, dx)
    got = O.weno5(fv, "linear")
    exact = sum(c * (dx / 2) ** m for m, c in enumerate(coeffs))
    if degree <= 4:
        assert abs(got - exact) < 1e-12 * max(1.0, np.abs(coeffs).max())
    else:
        assert abs(got - exact) > 1e-9


@pytest.mark.parametrize("scheme", ["js", "z"])
@pytest.mark.parametrize("degree", range(0, 3))
def test_nonlinear_weights_exact_up_to_degree_2(scheme, degree):
    rng = np.random.default_rng(120 + degree)
    coeffs = rng.normal(size=degree + 1) * 5
    dx = 0.3
    fv = cell_averages(coeffs, np.arange(-2, 3) * dx, dx)
    got = O.weno5(fv, scheme)
    exact = sum(c * (dx / 2) ** m for m, c in enumerate(coeffs))
    assert abs(got - exact) < 1e-12 * max(1.0, np.abs(coeffs).max())


@pytest.mark.parametrize("scheme", ["js", "z"])
def test_eno_property_at_a_jump(scheme):
    vals = np.array([1.0, 1.0, 1.0, 1.0, 10.0])  # step between a_{i+1} and a_{i+2}
    got = O.weno5(vals, scheme)
    assert 1.0 - 1e-9 <= got <= 1.0 + 1e-3
    assert abs(O.weno5(vals, "linear") - 1.0) > 0.05  # 3/10 * (-1/6) * 9


@pytest.mark.parametrize("scheme", ["linear", "js", "z"])
def test_odd_symmetry_bitwise(scheme):
    rng = np.random.default_rng(6)
    for _ in range(50):
        v = rng.normal(size=5) * 3
        assert O.weno5(-v, scheme) == -O.weno5(v, scheme)


def test_weno5_z_face_value_converges_at_fifth_order():
    errs = []
    for h in (1 / 16, 1 / 32, 1 / 64):
        x0 = 0.1234
        xs = x0 + np.arange(-2, 3) * h
        avg = 2 + (np.cos(2 * np.pi * (xs - h / 2)) - np.cos(2 * np.pi * (xs + h / 2))) / (2 * np.pi * h)
        exact = np.sin(2 * np.pi * (x0 + h / 2)) + 2
        errs.append(abs(O.weno5(avg, "z") - exact))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) > 4.6, (errs, orders)


@pytest.mark.parametrize("scheme", ["z5", "linear5"])
def test_spatial_order_five(scheme):
    L = 2.0
    errs = []
    for N in (64, 128, 256):
        _, p = smooth_1d_prim(N, L)
        pb = O.Problem(n=(N, 1, 1), dx=(L / N, 1.0, 1.0), bc=("periodic",) * 3, weno=scheme)
        U = O.prim_to_cons(pb, p.reshape(5, 1, 1, N))
        Lh, _, fx = O.rhs(pb, U, 1.0)
        assert fx == 0
        ex = -exact_flux_derivative(N, L, N * 9)
        errs.append(np.abs(Lh.reshape(5, N) - ex).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) >= 4.8, (errs, orders)


def test_weno5_uniform_state_and_mirror_symmetry():
    from paper_1511_02137_amd import workloads as W
    pb = O.Problem(n=(12, 10, 9), bc=("outflow",) * 3, weno="z5")
    U = O.prim_to_cons(pb, W.uniform_prim(pb.n, e=3.7, v=(0.31, -0.22, 0.45), nn=0.6))
    L, _, _ = O.rhs(pb, U, 1.0)
    assert np.all(L == 0.0)
    w = W.small_event(n=(16, 14, 12))
    pb = O.Problem(n=w.n, weno="z5")
    prim = w.prim0.copy()
    U = O.prim_to_cons(pb, prim)
    pm = prim[:, :, :, ::-1].copy()
    pm[1] = -pm[1]
    Um = O.prim_to_cons(pb, pm)
    L1, _, _ = O.rhs(pb, U, 1.0)
    L2, _, _ = O.rhs(pb, Um, 1.0)
    sign = np.array([1, -1, 1, 1, 1])[:, None, None, None]
    assert np.array_equal(L1, sign * L2[:, :, :, ::-1])
