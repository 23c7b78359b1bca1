"""Pins of the oracle's stage right-hand side and RK3 step (CPU only).

Each test checks the oracle against something the mathematics fixes:
invariance of a uniform state, mirror symmetry, exact conservation with
periodic boundaries, the energy budget with a jet, the closed form of the
source (Eq. 3), bitwise restart, and the orders of accuracy in space and time.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1511_02137_amd import workloads as W

HBARC = 0.1973269804


def small_problem(n=(16, 16, 16), bc="outflow", **kw):
    return O.Problem(n=n, bc=(bc, bc, bc), **kw)


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_uniform_state_rhs_is_exactly_zero(bc):
    pb = small_problem((12, 10, 9), bc)
    prim = W.uniform_prim(pb.n, e=3.7, v=(0.31, -0.22, 0.45), nn=0.6)
    U = O.prim_to_cons(pb, prim)
    L, _, fx = O.rhs(pb, U, 1.0)
    assert fx == 0
    assert np.all(L == 0.0)


def test_uniform_state_preserved_by_steps():
    pb = small_problem((8, 8, 8), "periodic")
    prim = W.uniform_prim(pb.n, e=3.7, v=(0.31, -0.22, 0.45), nn=0.6)
    U0 = O.prim_to_cons(pb, prim)
    st = O.run(pb, U0, 3)
    # only the RK convex combinations round: a few ulp per step
    assert np.all(np.abs(st.U - U0) <= 3 * 4 * np.spacing(np.abs(U0)))


def asymmetric_prim(n, seed=3):
    """Smooth, asymmetric initial state: off-centre Gaussian with a swirling flow."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    x = W.centres(nx, 0.1)[None, None, :]
    y = W.centres(ny, 0.1)[None, :, None]
    z = W.centres(nz, 0.1)[:, None, None]
    c = rng.uniform(-0.3, 0.3, size=3)
    r2 = (x - c[0]) ** 2 / 0.2 + (y - c[1]) ** 2 / 0.3 + (z - c[2]) ** 2 / 0.25
    prim = np.empty((5, nz, ny, nx))
    prim[0] = 20 * np.exp(-r2) + 0.05
    prim[1] = 0.3 * np.tanh(y - c[1]) * np.exp(-r2 / 4)
    prim[2] = -0.25 * np.tanh(x - c[0] + 0.1 * z) * np.exp(-r2 / 4)
    prim[3] = 0.1 * np.sin(3 * x) * np.cos(2 * y)
    prim[4] = 0.5 + 0.2 * np.exp(-r2)
    return prim


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry_bitwise(axis):
    n = (14, 12, 10)
    pb = small_problem(n, "outflow")
    prim = asymmetric_prim(n)
    arr_axis = 2 - axis  # numpy axis of the spatial direction
    mprim = np.flip(prim, axis=1 + arr_axis).copy()
    mprim[1 + axis] *= -1.0
    U = O.prim_to_cons(pb, prim)
    Um = O.prim_to_cons(pb, mprim)
    a = O.run(pb, U, 3).U
    b = O.run(pb, Um, 3).U
    bb = np.flip(b, axis=1 + arr_axis).copy()
    bb[1 + axis] *= -1.0
    assert np.array_equal(a, bb)


def test_axis_permutation_bitwise():
    # x <-> y exchange of the data and of the grid is an exact symmetry.
    n = (12, 12, 10)
    pb = small_problem(n, "outflow")
    prim = asymmetric_prim(n)
    pprim = np.swapaxes(prim, 2, 3).copy()
    pprim[[1, 2]] = pprim[[2, 1]]
    a = O.run(pb, O.prim_to_cons(pb, prim), 2).U
    b = O.run(pb, O.prim_to_cons(pb, pprim), 2).U
    bb = np.swapaxes(b, 2, 3).copy()
    bb[[1, 2]] = bb[[2, 1]]
    assert np.array_equal(a, bb)


def test_conservation_periodic_no_source():
    w = W.small_event(1, with_jet=False)
    pb = O.Problem(n=w.n, bc=("periodic",) * 3)
    U0 = O.prim_to_cons(pb, w.prim0)
    s0 = O.sums(pb, U0)
    st = O.run(pb, U0, 10)
    s1 = O.sums(pb, st.U)
    assert st.fixups == 0
    assert np.all(np.abs(s1 - s0) <= 1e-13 * s0[0])


def test_energy_budget_periodic_with_jet():
    w = W.small_event(1)
    pb = O.Problem(n=w.n, bc=("periodic",) * 3)
    U0 = O.prim_to_cons(pb, w.prim0)
    jets = [O.Jet(**j.__dict__) for j in w.jets]
    s0 = O.sums(pb, U0)
    st = O.run(pb, U0, 10, jets)
    s1 = O.sums(pb, st.U)
    assert st.ledger > 0.1
    assert abs((s1[0] - s0[0]) - st.ledger) <= 1e-13 * s0[0]
    d = np.array(w.jets[0].dir)
    for k in range(3):
        assert abs((s1[1 + k] - s0[1 + k]) - d[k] * st.ledger) <= 1e-13 * s0[0]
    assert abs(s1[4] - s0[4]) <= 1e-13 * s0[4]
    assert st.Ejet[0] == pytest.approx(w.jets[0].E0 - st.ledger, rel=1e-13)


def test_energy_budget_gaussian_deposit():
    w = W.small_gradient_event(n=(24, 24, 24), steps=4)
    pb = O.Problem(n=w.n, bc=("periodic",) * 3, deposit="gauss")
    U0 = O.prim_to_cons(pb, w.prim0)
    jets = [O.Jet(**j.__dict__) for j in w.jets]
    s0 = O.sums(pb, U0)
    st = O.run(pb, U0, 4, jets)
    s1 = O.sums(pb, st.U)
    assert st.ledger > 0.01
    assert abs((s1[0] - s0[0]) - st.ledger) <= 1e-13 * s0[0]


@pytest.mark.parametrize("crcf", [1.0, 9.0 / 4.0])
def test_source_closed_form_uniform_medium(crcf):
    # Uniform medium at rest, e = 30 GeV/fm^3: D = 0 exactly and the stage RHS
    # at the jet cell is P/dV with P from Eq. (3), T from e = g pi^2/30 T^4/(hbar c)^3.
    n = (10, 10, 10)
    pb = small_problem(n, "outflow")
    U = O.prim_to_cons(pb, W.uniform_prim(n, e=30.0, v=(0, 0, 0), nn=1.0))
    jet = O.Jet(x0=(0.05, -0.05, 0.05), dir=(0.6, 0.8, 0.0), cr_over_cf=crcf)
    T = (30.0 * 30.0 * HBARC ** 3 / (47.5 * math.pi ** 2)) ** 0.25
    assert abs(T - 0.3485) < 5e-4
    dV = 0.1 ** 3
    i = int(math.floor((0.05 + 0.5) / 0.1 + 1e-9))
    j = int(math.floor((-0.05 + 0.5) / 0.1 + 1e-9))
    k = i
    for ell in (0.0, 0.02, 0.01):
        L, P, _ = O.rhs(pb, U, 1.0 + ell, [jet])
        Pexp = 2.5 * crcf * T * T / HBARC + 4.0 * crcf * T ** 3 * ell / HBARC ** 2
        assert P[0] == pytest.approx(Pexp, rel=1e-14)
        # the jet has moved by ell along dir; it stays in the same cell here
        assert L[0, k, j, i] == pytest.approx(Pexp / dV, rel=1e-14)
        assert L[1, k, j, i] == pytest.approx(0.6 * Pexp / dV, rel=1e-14)
        assert L[2, k, j, i] == pytest.approx(0.8 * Pexp / dV, rel=1e-14)
        assert L[3, k, j, i] == 0.0 and L[4, k, j, i] == 0.0
        mask = np.ones(L.shape[1:], bool)
        mask[k, j, i] = False
        assert np.all(L[:, mask] == 0.0)


def test_jet_outside_box_or_not_started_deposits_nothing():
    n = (8, 8, 8)
    pb = small_problem(n)
    U = O.prim_to_cons(pb, W.uniform_prim(n, e=30.0, v=(0, 0, 0)))
    for jet, t in [(O.Jet(x0=(0.41, 0.0, 0.0)), 1.0), (O.Jet(x0=(0.0, 0.0, 0.0), t_start=2.0), 1.5),
                   (O.Jet(x0=(0.3, 0.0, 0.0)), 1.2)]:
        L, P, _ = O.rhs(pb, U, t, [jet])
        assert P[0] == 0.0 and np.all(L == 0.0)


def test_jet_depletion_stops_the_deposit():
    """A jet with little energy in a hot medium (periodic, so that the box's
    energy changes only by the source): each step removes from the jet
    exactly what the ledger gains and the box's total energy gains (Eq. 2's
    source is the jet's loss); the step that would take the jet below zero
    still deposits in full (the jet was alive at its start) and leaves E_jet
    = 0; after it nothing is deposited and the state keeps its energy."""
    n = (12, 12, 12)
    pb = small_problem(n, bc="periodic")
    U = O.prim_to_cons(pb, W.uniform_prim(n, e=30.0, v=(0.1, 0.0, 0.0)))
    jet = O.Jet(x0=(0.013, 0.021, -0.017), E0=0.2)
    dV = 1e-3
    st = O.RunState(U=U, Ejet=np.array([jet.E0]))
    E_prev, led_prev, depleted_at = float(st.U[0].sum() * dV), 0.0, None
    for k in range(8):
        Ej_prev = float(st.Ejet[0])
        st = O.run(pb, st.U, 1, [jet], step0=k, Ejet=st.Ejet, ledger=st.ledger)
        E_now = float(st.U[0].sum() * dV)
        gain = st.ledger - led_prev
        assert E_now - E_prev == pytest.approx(gain, rel=1e-9, abs=1e-13)
        if depleted_at is None:
            assert gain > 0
            if st.Ejet[0] == 0.0:
                depleted_at = k
                assert gain >= Ej_prev
            else:
                assert Ej_prev - st.Ejet[0] == pytest.approx(gain, rel=1e-12)
        else:
            assert gain == 0.0 and st.Ejet[0] == 0.0
        E_prev, led_prev = E_now, st.ledger
    assert depleted_at is not None and depleted_at < 7


def test_ngp_tie_goes_to_upper_cell():
    # x = 0 lies on the face between cells 3 and 4 of an 8-cell axis.
    n = (8, 8, 8)
    pb = small_problem(n)
    U = O.prim_to_cons(pb, W.uniform_prim(n, e=30.0, v=(0, 0, 0)))
    L, P, _ = O.rhs(pb, U, 1.0, [O.Jet(x0=(0.0, 0.0, 0.0))])
    idx = np.argwhere(L[0] != 0.0)
    assert idx.tolist() == [[4, 4, 4]]


def test_restart_is_bitwise():
    w = W.small_event(1, n=(16, 16, 16))
    pb = O.Problem(n=w.n)
    U0 = O.prim_to_cons(pb, w.prim0)
    jets = [O.Jet(**j.__dict__) for j in w.jets]
    full = O.run(pb, U0, 6, jets)
    a = O.run(pb, U0, 3, jets)
    b = O.run(pb, a.U, 3, jets, step0=a.step, Ejet=a.Ejet, ledger=a.ledger)
    assert np.array_equal(full.U, b.U)
    assert full.ledger == b.ledger and np.array_equal(full.Ejet, b.Ejet)


def smooth_1d_prim(N, L):
    x = W.centres(N, L / N)
    k = 2 * math.pi / L
    return x, np.stack([1.0 + 0.3 * np.sin(k * x), 0.3 * np.sin(k * x + 1.0), 0.1 * np.cos(k * x),
                        0.05 * np.sin(2 * k * x), 1.0 + 0.2 * np.cos(k * x)])


def exact_flux_derivative(N, L, Nf=2048):
    """d f_x / dx at the N cell centres, by FFT on a fine grid that contains them."""
    assert Nf % N == 0
    x, p = smooth_1d_prim(Nf, L)
    e, vx, vy, vz, n = p
    g2 = 1.0 / (1.0 - vx * vx - vy * vy - vz * vz)
    pres = e / 3.0
    w = (e + pres) * g2
    Mx, My, Mz = w * vx, w * vy, w * vz
    f = np.stack([Mx, Mx * vx + pres, My * vx, Mz * vx, n * np.sqrt(g2) * vx])
    kk = 2 * math.pi * np.fft.fftfreq(Nf, d=L / Nf)
    df = np.real(np.fft.ifft(1j * kk * np.fft.fft(f, axis=1), axis=1))
    step = Nf // N
    # fine centres with an odd/even shift: pick the fine points that coincide
    xs_fine = x
    xs = W.centres(N, L / N)
    idx = np.searchsorted(xs_fine, xs - 1e-12)
    assert np.allclose(xs_fine[idx], xs, atol=1e-12), step
    return df[:, idx]


@pytest.mark.parametrize("scheme", ["z", "linear"])
def test_spatial_order_seven(scheme):
    L = 2.0
    errs = []
    Ns = [64, 128, 256]
    for N in Ns:
        # the fine grid holds the coarse centres when Nf / N is odd
        Nf = N * 9
        _, p = smooth_1d_prim(N, L)
        pb = O.Problem(n=(N, 1, 1), dx=(L / N, 1.0, 1.0), bc=("periodic",) * 3, weno=scheme)
        U = O.prim_to_cons(pb, p.reshape(5, 1, 1, N))
        Lh, _, fx = O.rhs(pb, U, 1.0)
        assert fx == 0
        ex = -exact_flux_derivative(N, L, Nf)
        errs.append(np.abs(Lh.reshape(5, N) - ex).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) >= 6.8, (errs, orders)


def test_time_order_three():
    N, L = 32, 2.0
    _, p = smooth_1d_prim(N, L)
    res = {}
    for m in (1, 2, 4, 8):
        dt = 0.5 * (L / N) / m
        pb = O.Problem(n=(N, 1, 1), dx=(L / N, 1.0, 1.0), dt=dt, bc=("periodic",) * 3)
        U = O.prim_to_cons(pb, p.reshape(5, 1, 1, N))
        res[m] = O.run(pb, U, 8 * m).U
    d1 = np.abs(res[1] - res[2]).max()
    d2 = np.abs(res[2] - res[4]).max()
    d3 = np.abs(res[4] - res[8]).max()
    o1, o2 = math.log2(d1 / d2), math.log2(d2 / d3)
    assert min(o1, o2) >= 2.9, (d1, d2, d3)


def test_sums_match_numpy():
    w = W.small_event(2, n=(10, 12, 14))
    pb = O.Problem(n=w.n)
    U = O.prim_to_cons(pb, w.prim0)
    s = O.sums(pb, U)
    ref = U.reshape(5, -1).sum(axis=1) * 0.1 ** 3
    assert np.allclose(s, ref, rtol=1e-14, atol=1e-15 * ref[0])


@pytest.mark.parametrize("n", [(8, 8, 8), (10, 6, 7), (6, 12, 4)])
def test_eps2_closed_form_uniform_field(n):
    # uniform e: eps2 = (sum y^2 * nx - sum x^2 * ny) / (sum y^2 * nx + sum x^2 * ny),
    # with sum_i x_i^2 = dx^2 n (n^2 - 1) / 12 for centred cells.
    pb = O.Problem(n=n)
    U = O.prim_to_cons(pb, W.uniform_prim(n, e=2.0, v=(0, 0, 0)))
    nx, ny, _ = n
    sx = 0.01 * nx * (nx * nx - 1) / 12
    sy = 0.01 * ny * (ny * ny - 1) / 12
    ref = (sy * nx - sx * ny) / (sy * nx + sx * ny)
    assert O.eps2(pb, U) == pytest.approx(ref, abs=1e-14)


@pytest.mark.parametrize("n", [(8, 8, 8), (10, 6, 7), (6, 12, 9), (7, 9, 4)])
def test_eps2_closed_form_picks_the_z0_planes(n):
    """A uniform background at rest plus one hot cell on each of the planes
    next to z = 0.  The z = 0 value is the mean of the two middle planes
    (even nz: planes nz/2 - 1 and nz/2, at z = -+dz/2) or the middle plane
    (odd nz): a spike on those planes enters with weight 1/2 (even) or 1
    (odd), a spike on any other plane not at all.  With sum_i x_i^2 =
    dx^2 n (n^2 - 1)/12 for centred cells the background sums are closed
    forms, so eps2 is known exactly; choosing other planes, a wrong weight or
    a shifted origin changes it."""
    nx, ny, nz = n
    bg, s = 0.5, 40.0
    prim = W.uniform_prim(n, e=bg, v=(0, 0, 0))
    # spikes: (i, j, plane)
    if nz % 2 == 0:
        planes, wt = (nz // 2 - 1, nz // 2), 0.5
    else:
        planes, wt = ((nz - 1) // 2,), 1.0
    cells = [(1, ny - 2, planes[0]), (nx - 1, 2, planes[-1])]
    off = [(nx // 2, 0, planes[-1] + 1), (0, ny // 2, planes[0] - 1)]  # neighbouring planes: no weight
    for i, j, k in cells + off:
        prim[0, k, j, i] += s
    pb = O.Problem(n=n)
    U = O.prim_to_cons(pb, prim)
    dx = 0.1
    xc = lambda i, m: (i - 0.5 * (m - 1)) * dx
    sx = dx * dx * nx * (nx * nx - 1) / 12
    sy = dx * dx * ny * (ny * ny - 1) / 12
    num = bg * (sy * nx - sx * ny)
    den = bg * (sy * nx + sx * ny)
    for i, j, _ in cells:
        num += wt * s * (xc(j, ny) ** 2 - xc(i, nx) ** 2)
        den += wt * s * (xc(j, ny) ** 2 + xc(i, nx) ** 2)
    assert O.eps2(pb, U) == pytest.approx(num / den, rel=1e-13, abs=1e-14)
