"""Complex-step derivatives of the oracle against central finite differences
of its real-valued runs (CPU only).

The complex-step run is the same template code in std::complex<double>; this
pins that every branch of the scheme (fix-ups, |tau|, deposit windows) is
continued analytically, so it can serve as the gradient oracle.
"""
import numpy as np
import pytest

import oracle as O
from paper_1511_02137_amd import workloads as W

N = (16, 16, 16)
STEPS = 3


@pytest.fixture(scope="module")
def setup():
    w = W.small_gradient_event(n=N, steps=STEPS)
    # put the jet inside the small box, off all faces
    w.jets[0].x0 = (-0.3345, 0.031, 0.013)
    pb = O.Problem(n=w.n, deposit="gauss")
    return w, pb


def eps2_run(pb, prim0, jets, steps):
    U = O.prim_to_cons(pb, prim0)
    st = O.run(pb, U, steps, jets)
    return O.eps2(pb, st.U)


@pytest.mark.parametrize("which", ["kappa_rad", "kappa_coll", "x0", "y0"])
def test_complex_step_matches_finite_differences_params(setup, which):
    w, pb = setup
    base = [O.Jet(**j.__dict__) for j in w.jets]
    val, der = O.eps2_complex_step(pb, w.prim0, STEPS, base, which)
    assert val == pytest.approx(eps2_run(pb, w.prim0, base, STEPS), rel=1e-14, abs=1e-16)

    def perturbed(s):
        js = [O.Jet(**j.__dict__) for j in w.jets]
        if which in ("kappa_rad", "kappa_coll"):
            setattr(js[0], which, getattr(js[0], which) + s)
        else:
            x0 = list(js[0].x0)
            x0["xyz".index(which[0])] += s
            js[0].x0 = tuple(x0)
        return js

    ref = {"kappa_rad": 4.0, "kappa_coll": 2.5, "x0": 0.3345, "y0": 0.3}[which]
    h = 1e-4 * ref
    fd = (eps2_run(pb, w.prim0, perturbed(h), STEPS) - eps2_run(pb, w.prim0, perturbed(-h), STEPS)) / (2 * h)
    assert der != 0.0
    assert abs(der - fd) <= 1e-6 * abs(der) + 1e-12, (der, fd)


def smooth_direction(shape, seed):
    """Seeded smooth perturbation: a few low Fourier modes per axis."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    out = np.zeros(shape)
    for _ in range(4):
        kx, ky, kz = rng.integers(0, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        out += rng.normal() * (np.cos(2 * np.pi * kx * np.arange(nx) / nx + ph[0])[None, None, :]
                               * np.cos(2 * np.pi * ky * np.arange(ny) / ny + ph[1])[None, :, None]
                               * np.cos(2 * np.pi * kz * np.arange(nz) / nz + ph[2])[:, None, None])
    return out


@pytest.mark.parametrize("kind,h,tol", [("smooth1", 1e-4, 1e-5), ("smooth2", 1e-4, 1e-5), ("rough", 1e-7, 1e-6)])
def test_complex_step_matches_finite_differences_initial_field(setup, kind, h, tol):
    # A rough (cell-by-cell random) direction crosses the kink of |tau| in the
    # nearly uniform background, so central differences only agree for tiny h;
    # smooth directions agree at the h = 1e-4 of the gradient runs.
    w, pb = setup
    jets = [O.Jet(**j.__dict__) for j in w.jets]
    if kind == "rough":
        de = np.random.default_rng(7).normal(size=pb.shape) * w.prim0[0]
    else:
        de = smooth_direction(pb.shape, int(kind[-1])) * w.prim0[0]
    _, der = O.eps2_complex_step(pb, w.prim0, STEPS, jets, "e_init", de=de)
    pp = w.prim0.copy()
    pp[0] += h * de
    pm = w.prim0.copy()
    pm[0] -= h * de
    fd = (eps2_run(pb, pp, jets, STEPS) - eps2_run(pb, pm, jets, STEPS)) / (2 * h)
    assert abs(der - fd) <= tol * abs(der), (der, fd)


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_jvp_matches_finite_differences(bc):
    """The oracle's complex-step Jacobian-vector product of whole steps against
    central differences of its real runs, in a smooth direction of all five
    fields."""
    w = W.small_gradient_event(n=(12, 10, 8), steps=3)
    w.jets[0].x0 = (-0.2345, 0.031, 0.013)
    pb = O.Problem(n=w.n, bc=(bc,) * 3, deposit="gauss")
    jets = [O.Jet(**j.__dict__) for j in w.jets]
    U0 = O.prim_to_cons(pb, w.prim0)
    V = np.stack([smooth_direction(pb.shape, 20 + f) for f in range(5)]) * np.abs(U0).max(axis=(1, 2, 3))[:, None, None, None]
    Ur, JV = O.jvp(pb, U0, V, 3, jets)
    Ureal = O.run(pb, U0, 3, jets).U  # complex division and roots round differently
    assert np.abs(Ur - Ureal).max() <= 1e-13 * np.abs(Ureal).max()
    # WENO-Z weights on the flat outflow ghosts bend sharply (beta ~ h^2 against
    # eps = 1e-6), so the differences converge only for h <= 1e-7 there.
    h = 1e-8
    Up = O.run(pb, U0 + h * V, 3, jets).U
    Um = O.run(pb, U0 - h * V, 3, jets).U
    fd = (Up - Um) / (2 * h)
    err = np.abs(fd - JV).max() / np.abs(JV).max()
    assert err <= 1e-6, err
