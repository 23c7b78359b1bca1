"""Pins of the oracle's WENO7 reconstruction (CPU only).

The constants are re-derived here with sympy from their definitions: candidate
values from the 4-cell polynomial with the given cell averages, smoothness
indicators from the Jiang-Shu integral sum_l dx^(2l-1) int (p^(l))^2, and the
ideal weights from matching the 7-cell polynomial.  The nonlinear schemes are
further pinned by polynomial exactness, the ENO property and order of accuracy.
"""
import functools

import numpy as np
import pytest
import sympy as sp

import oracle as O


@functools.lru_cache(maxsize=None)
def derived():
    x = sp.symbols("x")
    f = sp.symbols("f0:7")  # a_{i-3}..a_{i+3}; cell i spans [-1/2, 1/2]
    half = sp.Rational(1, 2)

    def poly_with_averages(offsets):
        deg = len(offsets)
        a = sp.symbols("c0:%d" % deg)
        p = sum(a[m] * x ** m for m in range(deg))
        eqs = [sp.integrate(p, (x, o - half, o + half)) - f[o + 3] for o in offsets]
        return sp.expand(p.subs(sp.solve(eqs, a)))

    q, beta = [], []
    for k in range(4):
        pk = poly_with_averages(list(range(-3 + k, 1 + k)))
        q.append(sp.expand(pk.subs(x, half)))
        beta.append(sp.expand(sum(sp.integrate(sp.diff(pk, x, l) ** 2, (x, -half, half)) for l in range(1, 4))))
    p7 = poly_with_averages(list(range(-3, 4)))
    target = sp.expand(p7.subs(x, half))
    d = sp.symbols("d0:4")
    eqs = sp.Poly(sp.expand(sum(d[k] * q[k] for k in range(4)) - target), *f).coeffs()
    dsol = sp.solve(eqs, d)
    dvals = [dsol[d[k]] for k in range(4)]
    return f, q, beta, dvals, target


def ref_weno(vals, scheme, eps=1e-6, p=2):
    f, q, beta, dvals, target = derived()
    sub = dict(zip(f, [sp.Float(v, 40) for v in vals]))
    qv = [q[k].evalf(40, subs=sub) for k in range(4)]
    bv = [beta[k].evalf(40, subs=sub) for k in range(4)]
    d = [sp.Float(dv, 40) for dv in dvals]
    if scheme == "linear":
        return float(sum(d[k] * qv[k] for k in range(4)))
    if scheme == "js":
        a = [d[k] / (eps + bv[k]) ** 2 for k in range(4)]
    else:
        tau = abs(bv[0] + 3 * bv[1] - 3 * bv[2] - bv[3])
        a = [d[k] * (1 + (tau / (bv[k] + eps)) ** p) for k in range(4)]
    s = sum(a)
    return float(sum(a[k] / s * qv[k] for k in range(4)))


def test_ideal_weights_are_1_12_18_4_over_35():
    *_, dvals, _ = derived()
    assert [sp.nsimplify(v) for v in dvals] == [sp.Rational(1, 35), sp.Rational(12, 35), sp.Rational(18, 35),
                                               sp.Rational(4, 35)]


def test_smoothness_indicators_have_denominator_240():
    f, q, beta, *_ = derived()
    for b in beta:
        coeffs = sp.Poly(240 * b, *f).coeffs()
        assert all(c.is_integer for c in coeffs)


@pytest.mark.parametrize("scheme", ["linear", "js", "z"])
def test_matches_definition_on_random_data(scheme):
    rng = np.random.default_rng(11)
    for trial in range(40):
        scale = 10.0 ** rng.uniform(-3, 2)
        vals = rng.normal(size=7) * scale + (scale if trial % 2 else 0.0)
        got = O.weno7(vals, scheme)
        ref = ref_weno(vals, scheme)
        assert abs(got - ref) <= 1e-13 * max(1.0, np.abs(vals).max()), (trial, got, ref)


def cell_averages(coeffs, centres, h):
    """Exact cell averages of the polynomial sum c_m x^m over [x - h/2, x + h/2]."""
    out = np.zeros_like(centres)
    for m, c in enumerate(coeffs):
        F = lambda t: t ** (m + 1) / (m + 1)
        out += c * (F(centres + h / 2) - F(centres - h / 2)) / h
    return out


@pytest.mark.parametrize("degree", range(0, 9))
def test_linear_weights_flux_difference_exact_up_to_degree_7(degree):
    # Point values f(x_j) treated as cell averages of h: the difference of the
    # two reconstructed face values is h(x_i + dx/2) - h(x_i - dx/2) exactly
    # for h of degree <= 7 (the degree-7 error constant is the same at both
    # faces and cancels), and not for degree 8.
    rng = np.random.default_rng(degree)
    coeffs = rng.normal(size=degree + 1)
    dx = 0.25
    xs = np.arange(-4, 5) * dx  # cells i-4..i+4 around x_i = 0
    fv = cell_averages(coeffs, xs, dx)
    right = O.weno7(fv[1:8], "linear")   # face i+1/2 from a_{i-3..i+3}
    left = O.weno7(fv[0:7], "linear")    # face i-1/2
    hp = sum(c * (dx / 2) ** m for m, c in enumerate(coeffs))
    hm = sum(c * (-dx / 2) ** m for m, c in enumerate(coeffs))
    err = abs((right - left) - (hp - hm))
    if degree <= 7:
        assert err < 1e-12 * max(1.0, np.abs(coeffs).max())
    else:
        assert err > 1e-9


@pytest.mark.parametrize("degree", range(0, 8))
def test_linear_weights_face_value_exact_up_to_degree_6(degree):
    rng = np.random.default_rng(50 + degree)
    coeffs = rng.normal(size=degree + 1)
    dx = 0.25
    xs = np.arange(-3, 4) * dx
    fv = cell_averages(coeffs, xs, dx)
    got = O.weno7(fv, "linear")
    exact = sum(c * (dx / 2) ** m for m, c in enumerate(coeffs))
    if degree <= 6:
        assert abs(got - exact) < 1e-12 * max(1.0, np.abs(coeffs).max())
    else:
        assert abs(got - exact) > 1e-9


@pytest.mark.parametrize("scheme", ["js", "z"])
@pytest.mark.parametrize("degree", range(0, 4))
def test_nonlinear_weights_exact_up_to_degree_3(scheme, degree):
    rng = np.random.default_rng(100 + degree)
    coeffs = rng.normal(size=degree + 1) * 5
    dx = 0.3
    xs = np.arange(-3, 4) * dx
    fv = cell_averages(coeffs, xs, dx)
    got = O.weno7(fv, scheme)
    exact = sum(c * (dx / 2) ** m for m, c in enumerate(coeffs))
    assert abs(got - exact) < 1e-12 * max(1.0, np.abs(coeffs).max())


@pytest.mark.parametrize("scheme", ["js", "z"])
def test_eno_property_at_a_jump(scheme):
    # A step between a_{i+2} and a_{i+3}: only stencil 0..2 are smooth.  The
    # reconstruction must stay within the data range (no Gibbs overshoot) and
    # be close to the smooth side's value.
    vals = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 10.0])
    got = O.weno7(vals, scheme)
    assert 1.0 - 1e-9 <= got <= 1.0 + 1e-3
    lin = O.weno7(vals, "linear")
    assert abs(lin - 1.0) > 0.05  # the linear scheme does feel the jump (4/35 * 0.75 * 9)


@pytest.mark.parametrize("scheme", ["linear", "js", "z"])
def test_odd_symmetry_bitwise(scheme):
    rng = np.random.default_rng(5)
    for _ in range(50):
        v = rng.normal(size=7) * 3
        assert O.weno7(-v, scheme) == -O.weno7(v, scheme)


def test_weno_z_converges_at_seventh_order():
    # Reconstruction of the face value of h(x) = sin(2 pi x) + 2 from cell
    # averages on a sweep of dx; the error must fall like dx^7.
    errs = []
    hs = [1 / 16, 1 / 32, 1 / 64]
    for h in hs:
        x0 = 0.1234
        xs = x0 + np.arange(-3, 4) * h
        avg = 2 + (np.cos(2 * np.pi * (xs - h / 2)) - np.cos(2 * np.pi * (xs + h / 2))) / (2 * np.pi * h)
        exact = np.sin(2 * np.pi * (x0 + h / 2)) + 2
        errs.append(abs(O.weno7(avg, "z") - exact))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) > 6.5, (errs, orders)


@pytest.mark.parametrize("scheme", ["js", "z"])
def test_flat_stencils_are_well_conditioned(scheme):
    # Outflow ghost cells make some stencils exactly flat.  There the
    # smoothness indicators must vanish exactly (evaluated from differences),
    # not leave rounding residue comparable with epsilon: the result must
    # agree with the 40-digit evaluation of the definition to ~1e-15.
    rng = np.random.default_rng(17)
    for trial in range(30):
        c = rng.uniform(0.5, 5.0) * rng.choice([-1, 1])
        tail = c + rng.normal(size=3) * rng.uniform(1e-3, 0.3)
        for vals in (np.r_[[c] * 4, tail], np.r_[tail[::-1], [c] * 4], np.r_[[c] * 5, tail[:2]]):
            got = O.weno7(vals, scheme)
            ref = ref_weno(vals, scheme)
            assert abs(got - ref) <= 1.5e-15 * max(1.0, np.abs(vals).max()), (trial, vals, got - ref)
