"""Pins of the oracle's Gaussian jet deposit (CPU only).

The delta function of Eq. (2) is spread over a separable Gaussian footprint of
width sigma = dx, seven cells per axis around the nearest cell, each 1-D
weight vector normalised to unit sum, and the temperature of Eq. (3) is the
average of the cell temperatures over the same footprint.  These tests check
the footprint against what a Gaussian of that width centred on the jet must
satisfy, not against a second copy of the formula:

* the support is the 7^3 block around the nearest cell (a wrong window or
  centre cell fails);
* the deposit is an outer product of three 1-D profiles (a non-separable or
  mis-indexed footprint fails);
* each profile's log has second differences equal to -dx^2/sigma^2 = -1
  (a wrong width fails), and its first differences place the centre on the
  jet's position at the stage time (a wrong centre, a sign error or a stale
  position fails);
* the total equals P of Eq. (3) at the averaged temperature, and on a medium
  whose e varies along x that temperature is the footprint average of the
  cell temperatures (the nearest cell's T, or T of the averaged e, fail);
* near the box edge the cells outside are dropped and the deposit shrinks by
  their weight.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1511_02137_amd import workloads as W

HBARC = 0.1973269804
DX = 0.1


def temperature(e):
    # e = g pi^2 / 30 T^4 / (hbar c)^3 with g = 47.5 (T(30 GeV/fm^3) = 0.3485 GeV
    # is pinned by test_source_closed_form_uniform_medium)
    return (30.0 * e * HBARC ** 3 / (47.5 * math.pi ** 2)) ** 0.25


def nearest(x, n):
    return int(math.floor((x + 0.5 * n * DX) / DX + 1e-9))


def deposit(pb, U, jet, t):
    """S(U) of one stage: L with the jet minus L without it (D is the same)."""
    L1, P, _ = O.rhs(pb, U, t, [jet])
    L0, _, _ = O.rhs(pb, U, t, [])
    return L1 - L0, P[0]


def profiles(S0):
    """1-D marginals (x, y, z) of the energy deposit, each summing to one."""
    tot = S0.sum()
    return S0.sum(axis=(0, 1)) / tot, S0.sum(axis=(0, 2)) / tot, S0.sum(axis=(1, 2)) / tot


def check_gaussian_profile(a, lo, n, x_jet):
    """a: the 7 in-box weights of one axis starting at cell lo."""
    la = np.log(a)
    # width: second differences of log w are -dx^2/sigma^2 = -1
    assert np.allclose(np.diff(la, 2), -1.0, rtol=0, atol=1e-12), np.diff(la, 2)
    # centre: log(w_{m+1}/w_m) = -(x_{m+1} + x_m - 2 x_jet) / (2 dx)
    xc = (np.arange(lo, lo + len(a)) - 0.5 * (n - 1)) * DX
    est = 0.5 * (xc[1:] + xc[:-1]) + DX * np.diff(la)
    assert np.allclose(est, x_jet, rtol=0, atol=1e-12), (est, x_jet)


@pytest.mark.parametrize("ell", [0.0, 0.02, 0.01])
def test_gaussian_footprint_on_uniform_medium(ell):
    n = (16, 16, 16)
    pb = O.Problem(n=n, deposit="gauss")
    e = 30.0
    U = O.prim_to_cons(pb, W.uniform_prim(n, e=e, v=(0, 0, 0), nn=1.0))
    d = np.array([0.48, -0.64, 0.6])
    x0 = np.array([0.0137, -0.0421, 0.0283])
    jet = O.Jet(x0=tuple(x0), dir=tuple(d))
    S, P = deposit(pb, U, jet, 1.0 + ell)
    xj = x0 + d * ell
    ctr = [nearest(xj[k], n[k]) for k in range(3)]
    # support: the 7^3 block around the nearest cell
    nz = np.argwhere(S[0] != 0.0)
    lo = [ctr[k] - 3 for k in range(3)]
    assert nz.shape[0] == 343
    for k, ax in zip(range(3), (2, 1, 0)):
        assert nz[:, ax].min() == lo[k] and nz[:, ax].max() == lo[k] + 6
    # momentum along the jet, no charge source
    for k in range(3):
        assert np.allclose(S[1 + k], d[k] * S[0], rtol=0, atol=1e-15 * S[0].max())
    assert np.all(S[4] == 0.0)
    # total: P of Eq. (3) at the uniform T (averaging any normalised footprint gives T)
    T = temperature(e)
    Pexp = 2.5 * T * T / HBARC + 4.0 * T ** 3 * ell / HBARC ** 2
    assert P == pytest.approx(Pexp, rel=1e-13)
    assert S[0].sum() * DX ** 3 == pytest.approx(Pexp, rel=1e-13)
    # separable: the deposit is the outer product of its marginals
    blk = S[0][lo[2]:lo[2] + 7, lo[1]:lo[1] + 7, lo[0]:lo[0] + 7]
    ax_, ay_, az_ = profiles(blk)
    outer = blk.sum() * az_[:, None, None] * ay_[None, :, None] * ax_[None, None, :]
    assert np.allclose(blk, outer, rtol=1e-13, atol=0)
    # Gaussian of width dx centred on the jet's position at the stage time
    for k, prof in zip(range(3), (ax_, ay_, az_)):
        check_gaussian_profile(prof, lo[k], n[k], xj[k])


def test_gaussian_temperature_is_footprint_average():
    """A medium at rest whose e grows linearly along x: P must be Eq. (3) at
    T_jet = sum_c w_c T(e_c), with w_c the deposit's own shares."""
    n = (16, 12, 14)
    pb = O.Problem(n=n, deposit="gauss")
    prim = W.uniform_prim(n, e=30.0, v=(0, 0, 0), nn=1.0)
    x = (np.arange(n[0]) - 0.5 * (n[0] - 1)) * DX
    prim[0] = (30.0 + 20.0 * x)[None, None, :]
    U = O.prim_to_cons(pb, prim)
    x0 = (0.0173, 0.0236, -0.0318)
    S, P = deposit(pb, U, O.Jet(x0=x0), 1.0)
    w = S[0] / S[0].sum()
    Tc = temperature(prim[0])
    T_avg = float((w * Tc).sum())
    assert P == pytest.approx(2.5 * T_avg * T_avg / HBARC, rel=1e-13)
    # the readings it is not: the nearest cell's T, or T of the averaged e
    i, j, k = (nearest(x0[a], n[a]) for a in range(3))
    T_ngp = float(Tc[k, j, i])
    T_of_e = temperature(float((w * prim[0]).sum()))
    for T_alt in (T_ngp, T_of_e):
        assert abs(2.5 * T_alt * T_alt / HBARC - P) > 1e-7 * P
    # the footprint is still the Gaussian around the jet
    lo = [nearest(x0[a], n[a]) - 3 for a in range(3)]
    blk = S[0][lo[2]:lo[2] + 7, lo[1]:lo[1] + 7, lo[0]:lo[0] + 7]
    for a, prof in zip(range(3), profiles(blk)):
        check_gaussian_profile(prof, lo[a], n[a], x0[a])


def test_gaussian_footprint_clipped_at_the_box_edge():
    """Cells of the footprint outside the box are dropped: the deposit is the
    in-box part of the same Gaussian, and its total is P times the in-box
    weight (which P_eff reports and the ledger books)."""
    n = (12, 12, 12)
    pb = O.Problem(n=n, deposit="gauss")
    e = 30.0
    U = O.prim_to_cons(pb, W.uniform_prim(n, e=e, v=(0, 0, 0), nn=1.0))
    x0 = (0.5317, -0.0212, 0.0119)  # nearest x cell 11, the last one: cells 12..14 are outside
    S, P_eff = deposit(pb, U, O.Jet(x0=x0), 1.0)
    T = temperature(e)
    P = 2.5 * T * T / HBARC
    nz = np.argwhere(S[0] != 0.0)
    assert nz[:, 2].min() == 8 and nz[:, 2].max() == 11
    assert nz.shape[0] == 4 * 49
    # in-box weight of the x profile: the full 7-cell Gaussian is known from its
    # width and centre, so the kept fraction follows from the four in-box cells
    xc = (np.arange(8, 15) - 0.5 * (n[0] - 1)) * DX
    g = np.exp(-((xc - x0[0]) / DX) ** 2 / 2)
    frac = g[:4].sum() / g.sum()
    assert P_eff == pytest.approx(P * frac, rel=1e-13)
    assert S[0].sum() * DX ** 3 == pytest.approx(P * frac, rel=1e-13)
    lo = [8, nearest(x0[1], n[1]) - 3, nearest(x0[2], n[2]) - 3]
    blk = S[0][lo[2]:lo[2] + 7, lo[1]:lo[1] + 7, 8:12]
    ax_, ay_, az_ = profiles(blk)
    check_gaussian_profile(ax_, 8, n[0], x0[0])
    check_gaussian_profile(ay_, lo[1], n[1], x0[1])
