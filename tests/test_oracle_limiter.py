"""Pins of the oracle's positivity-preserving flux limiter (CPU only).

Reading (after Zhang and Shu, the paper's WENO reference): each face flux F
becomes theta F + (1 - theta) F_LF, F_LF the first-order Lax-Friedrichs flux
F+(u_i) + F-(u_{i+1}), with theta the chord-rule value that keeps both half
states next to the face, u_i - mu (F - f_i/2) and u_{i+1} + mu (F - f_{i+1}/2)
with mu = 2 dt sum_d 1/dx_d, inside {E - |M| >= 1e-13, N >= 1e-13}.

What the pins check, each against something other than the oracle's formula:
  * the premise: u +- f_d(u) is admissible for every admissible u (with the
    closed form (E'^2 - |M'|^2) = (8/9) e^2 gamma^2 (1 +- v_d)^2), and the
    half-state decomposition of a forward-Euler update (algebra, numpy);
  * one face: the limited half states are admissible; theta never exceeds
    the largest admissible theta found by bisection, equals it when only the
    (linear) charge constraint binds, and the limited flux is exactly the
    stated convex combination; theta = 1 leaves the flux untouched;
  * whole runs: no effect on a flow that needs no limiting (bitwise), exact
    uniform states, conservation with periodic boundaries, mirror symmetry;
  * a jet in a 24 x 20 x 22 box and a near-vacuum Riemann problem where the
    unlimited scheme leaves E < |M| or N < 0: with the limiter every step
    stays admissible without recovery fix-ups, and the Riemann run still
    converges to the exact solution.
"""
import math
import sys
import os

import numpy as np
import pytest

import oracle as O
from paper_1511_02137_amd import workloads as W

sys.path.insert(0, os.path.dirname(__file__))
from test_oracle_riemann import exact_solution, line  # noqa: E402

EPS = 1e-13


def cons(e, v, n):
    """Conserved (E, Mx, My, Mz, N) of primitives, p = e/3 (textbook relations)."""
    v = np.asarray(v, dtype=np.float64)
    g2 = 1.0 / (1.0 - v @ v)
    w = 4.0 / 3.0 * e * g2
    return np.array([w - e / 3.0, w * v[0], w * v[1], w * v[2], n * math.sqrt(g2)])


def flux(u, d, e, v):
    """Physical flux along axis d of the state u with primitives (e, v)."""
    f = np.empty(5)
    f[0] = u[1 + d]
    for m in range(3):
        f[1 + m] = u[1 + m] * v[d] + (e / 3.0 if m == d else 0.0)
    f[4] = u[4] * v[d]
    return f


def random_state(rng, vmax=0.999):
    e = 10.0 ** rng.uniform(-8, 2)
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    v = direction * rng.uniform(0, vmax)
    n = 10.0 ** rng.uniform(-6, 1)
    return e, v, n


def gap(s):
    return s[0] - math.sqrt(s[1] ** 2 + s[2] ** 2 + s[3] ** 2)


def test_lax_friedrichs_states_are_admissible():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        e, v, n = random_state(rng)
        u = cons(e, v, n)
        g2 = 1.0 / (1.0 - v @ v)
        for d in range(3):
            f = flux(u, d, e, v)
            for sgn in (1.0, -1.0):
                s = u + sgn * f
                m2 = s[1] ** 2 + s[2] ** 2 + s[3] ** 2
                closed = 8.0 / 9.0 * e * e * g2 * (1.0 + sgn * v[d]) ** 2
                assert s[0] * s[0] - m2 == pytest.approx(closed, rel=1e-6, abs=1e-12 * s[0] * s[0])
                assert s[0] > 0 and s[0] * s[0] > m2 and s[4] > 0


def test_half_state_decomposition_of_the_update():
    rng = np.random.default_rng(1)
    dt, dx = 0.02, np.array([0.1, 0.13, 0.07])
    lam = dt / dx
    w = lam / lam.sum()
    mu = 2.0 * dt * (1.0 / dx).sum()
    u = rng.normal(size=5)
    f = rng.normal(size=(3, 5))
    Fm, Fp = rng.normal(size=(3, 5)), rng.normal(size=(3, 5))  # faces i-1/2, i+1/2
    update = u - (lam[:, None] * (Fp - Fm)).sum(axis=0)
    R = u[None, :] - mu * (Fp - 0.5 * f)
    L = u[None, :] + mu * (Fm - 0.5 * f)
    assert np.allclose((w[:, None] * 0.5 * (R + L)).sum(axis=0), update, rtol=1e-13, atol=1e-13)
    # with the first-order flux the half state is the stated convex combination
    e1, v1, n1 = 2.0, np.array([0.3, -0.1, 0.2]), 0.5
    e2, v2, n2 = 0.7, np.array([-0.6, 0.4, 0.1]), 0.2
    uA, uB = cons(e1, v1, n1), cons(e2, v2, n2)
    fA, fB = flux(uA, 0, e1, v1), flux(uB, 0, e2, v2)
    FLF = 0.5 * (fA + uA) + 0.5 * (fB - uB)
    RA = uA - mu * (FLF - 0.5 * fA)
    assert np.allclose(RA, (1 - mu / 2) * uA + mu / 2 * (uB - fB), rtol=1e-13, atol=1e-14)


def half_states(pb, d, uA, uB, H):
    mu = 2.0 * pb.dt * sum(1.0 / x for x in pb.dx)
    pa, _ = O.cons_to_prim(O.Problem(n=(1, 1, 1)), uA.reshape(5, 1, 1, 1))
    pbb, _ = O.cons_to_prim(O.Problem(n=(1, 1, 1)), uB.reshape(5, 1, 1, 1))
    fA = flux(uA, d, pa[0].item(), pa[1:4].ravel())
    fB = flux(uB, d, pbb[0].item(), pbb[1:4].ravel())
    return uA - mu * (H - 0.5 * fA), uB + mu * (H - 0.5 * fB), 0.5 * (fA + uA) + 0.5 * (fB - uB)


def admissible(s, tol=0.0):
    return gap(s) >= EPS - tol and s[4] >= EPS - tol


def largest_theta(pb, d, uA, uB, H):
    """Bisection for the largest theta with both half states admissible."""
    _, _, FLF = half_states(pb, d, uA, uB, H)

    def ok(t):
        ra, lb, _ = half_states(pb, d, uA, uB, t * H + (1 - t) * FLF)
        return admissible(ra) and admissible(lb)

    if ok(1.0):
        return 1.0
    lo, hi = 0.0, 1.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if ok(mid):
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("d", [0, 1, 2])
def test_single_face_limiter_against_bisection(d):
    pb = O.Problem(n=(8, 8, 8))
    rng = np.random.default_rng(10 + d)
    limited = 0
    for k in range(300):
        e1, v1, n1 = random_state(rng, 0.95)
        e2, v2, n2 = random_state(rng, 0.95)
        uA, uB = cons(e1, v1, n1), cons(e2, v2, n2)
        _, _, FLF = half_states(pb, d, uA, uB, np.zeros(5))
        scale = max(abs(uA).max(), abs(uB).max())
        H = FLF + rng.normal(size=5) * scale * 10.0 ** rng.uniform(-3, 1)
        Hl, th = O.limit_face(pb, d, uA, uB, H)
        assert 0.0 <= th <= 1.0
        if th == 1.0:
            assert np.array_equal(Hl, H)
            continue
        limited += 1
        assert np.allclose(Hl, th * H + (1 - th) * FLF, rtol=1e-12, atol=1e-15 * scale)
        ra, lb, _ = half_states(pb, d, uA, uB, Hl)
        tol = 1e-12 * scale
        assert admissible(ra, tol) and admissible(lb, tol), (k, gap(ra), gap(lb), ra[4], lb[4])
        best = largest_theta(pb, d, uA, uB, H)
        assert th <= best + 1e-9, (k, th, best)
    assert limited > 50


def test_charge_constraint_gives_exact_root():
    """When only N would go negative, the constraint is linear and the chord
    rule returns the exact largest theta."""
    pb = O.Problem(n=(8, 8, 8))
    uA = cons(1.0, np.array([0.1, 0.0, 0.0]), 0.5)
    uB = cons(1.2, np.array([0.0, 0.1, 0.0]), 0.4)
    _, _, FLF = half_states(pb, 0, uA, uB, np.zeros(5))
    H = FLF.copy()
    H[4] += 3.0  # drives N of the low-side half state negative only
    Hl, th = O.limit_face(pb, 0, uA, uB, H)
    assert 0.0 < th < 1.0
    ra, lb, _ = half_states(pb, 0, uA, uB, Hl)
    assert ra[4] == pytest.approx(EPS, abs=1e-15)
    assert th == pytest.approx(largest_theta(pb, 0, uA, uB, H), abs=1e-12)


def jet_box(lim, bc="outflow", n=(24, 20, 22), mirror=False):
    dx = (0.1, 0.1, 0.1)
    L = [n[k] * 0.1 for k in range(3)]
    prim = W.ellipsoid_prim(n, dx, tuple(0.2 * x for x in L), 27.0)
    pb = O.Problem(n=n, bc=(bc,) * 3, deposit="ngp", limiter=lim)
    d = (-0.9916173911378503, 0.02872803653083503, 0.12597479712246648)
    x0 = (0.25 * L[0] + 0.0137, -L[0] / 3.2, -1.2 * L[0] / 3.2)  # off the cell faces
    if mirror:  # x -> -x
        prim = prim[:, :, :, ::-1].copy()
        prim[1] = -prim[1]
        d = (-d[0], d[1], d[2])
        x0 = (-x0[0], x0[1], x0[2])
    return pb, O.prim_to_cons(pb, prim), [O.Jet(x0=x0, dir=d, E0=92.3)]


def test_unlimited_run_leaves_the_admissible_set():
    pb, U, jets = jet_box("none")
    st = O.run(pb, U, 30, jets)
    g = st.U[0] - np.sqrt(st.U[1] ** 2 + st.U[2] ** 2 + st.U[3] ** 2)
    assert st.fixups > 0 or g.min() < 0


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_limited_run_stays_admissible_every_step(bc):
    pb, U, jets = jet_box("pp", bc)
    Ej, ledger = None, 0.0
    step = 0
    for _ in range(30):
        st = O.run(pb, U, 1, jets, step0=step, Ejet=Ej, ledger=ledger)
        U, Ej, ledger, step = st.U, st.Ejet, st.ledger, st.step
        g = U[0] - np.sqrt(U[1] ** 2 + U[2] ** 2 + U[3] ** 2)
        assert st.fixups == 0 and g.min() >= EPS * (1 - 1e-3) and U[4].min() >= EPS, (step, g.min())


def test_limiter_conserves_with_periodic_boundaries():
    pb, U, jets = jet_box("pp", "periodic")
    s0 = O.sums(pb, U)
    st = O.run(pb, U, 30, jets)
    s1 = O.sums(pb, st.U)
    # N has no source; E gains exactly the deposited energy (the ledger)
    assert abs(s1[4] - s0[4]) <= 1e-13 * abs(s0[4])
    assert abs((s1[0] - s0[0]) - st.ledger) <= 1e-12 * abs(s0[0])
    unlimited = O.run(O.Problem(**{**pb.__dict__, "limiter": "none"}), U, 30, jets)
    assert not np.array_equal(unlimited.U, st.U)  # the limiter did act


def test_limiter_is_mirror_symmetric():
    pb, U, jets = jet_box("pp")
    pbm, Um, jetsm = jet_box("pp", mirror=True)
    a = O.run(pb, U, 30, jets).U
    b = O.run(pbm, Um, 30, jetsm).U
    b = b[:, :, :, ::-1]
    b[1] = -b[1]
    assert np.array_equal(a, b)


def test_limiter_inactive_on_smooth_flow_is_bitwise():
    w = W.small_event(n=(20, 18, 16), steps=5, with_jet=False)
    runs = []
    for lim in ("none", "pp"):
        pb = O.Problem(n=w.n, dx=w.dx, dt=w.dt, t0=w.t0, limiter=lim)
        runs.append(O.run(pb, O.prim_to_cons(pb, w.prim0), 5).U)
    assert np.array_equal(runs[0], runs[1])


def test_limiter_keeps_uniform_state_exact():
    n = (10, 8, 6)
    pb = O.Problem(n=n, limiter="pp", bc=("periodic", "outflow", "periodic"))
    U = O.prim_to_cons(pb, W.uniform_prim(n))
    L, _, fx = O.rhs(pb, U, 1.0)
    assert fx == 0 and np.all(L == 0.0)
    plain = O.Problem(n=n, bc=("periodic", "outflow", "periodic"))
    assert np.array_equal(O.run(pb, U, 3).U, O.run(plain, U, 3).U)


def riemann(N, eR, lim):
    L = 2.0
    dx = L / N
    dt = 0.2 * dx
    steps = int(round(0.4 / dt))
    pb = O.Problem(n=(N, 1, 1), dx=(dx, 1.0, 1.0), dt=dt, bc=("outflow", "periodic", "periodic"), t0=0.0,
                   limiter=lim)
    x = W.centres(N, dx)
    prim = np.zeros((5, 1, 1, N))
    prim[0] = np.where(x < 0, 10.0, eR)
    prim[4] = np.where(x < 0, 1.0, (eR / 10.0) ** 0.75)
    st = O.run(pb, O.prim_to_cons(pb, prim), steps)
    pr, fx = O.cons_to_prim(pb, st.U)
    return x, steps * dt, st, pr, fx


def test_near_vacuum_riemann_problem():
    """e_L = 10, e_R = 1e-8: without the limiter E < |M| and N < 0 appear;
    with it the run stays admissible and converges to the exact solution."""
    eR = 1e-8
    _, _, st, _, fx = riemann(100, eR, "none")
    g = st.U[0] - np.sqrt(st.U[1] ** 2 + st.U[2] ** 2 + st.U[3] ** 2)
    assert fx > 0 and g.min() < 0 and st.U[4].min() < 0
    l1 = []
    for N in (100, 200, 400):
        x, t, st, pr, fx = riemann(N, eR, "pp")
        g = st.U[0] - np.sqrt(st.U[1] ** 2 + st.U[2] ** 2 + st.U[3] ** 2)
        assert fx == 0 and g.min() > 0 and st.U[4].min() > 0
        e_ex = exact_solution(x / t, 10.0, eR, 1.0, (eR / 10.0) ** 0.75)[0]
        l1.append(np.abs(line(pr, 0, 0) - e_ex).sum() * 2.0 / N)
    l1 = np.array(l1)
    assert np.all(np.log2(l1[:-1] / l1[1:]) >= 0.8), l1
