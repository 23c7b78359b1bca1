"""Seeded synthetic inputs shaped like the paper's runs.

The paper's figures come from a 256^3 grid with dx = 0.1 fm, dt = 0.02 fm/c,
p = e/3 and an ellipsoidal initial state at t0 = 1 fm/c (Results section,
Fig. 3 caption).  The ellipsoidal-flow initial condition it cites is not
reproduced here; a Gaussian ellipsoid of energy density with a Hubble-like
flow stands in for it.  Jets start on straight lines at the speed of light.

This module only draws inputs: primitive fields (e, vx, vy, vz, n) on the grid
and jet descriptions.  It holds none of the method's arithmetic (no
primitive->conserved map, no fluxes, no source), so both the library and the
CPU oracle can take their inputs from it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

HBARC = 0.1973269804  # GeV fm
EOS_DOF = 47.5        # degrees of freedom in e = g pi^2/30 T^4


@dataclass
class JetSpec:
    x0: Tuple[float, float, float]
    dir: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    E0: float = 50.0
    t_start: float = 1.0
    kappa_rad: float = 4.0
    kappa_coll: float = 2.5
    cr_over_cf: float = 1.0


@dataclass
class Workload:
    name: str
    n: Tuple[int, int, int]              # (nx, ny, nz)
    dx: Tuple[float, float, float]
    dt: float
    t0: float
    steps: int
    bc: Tuple[str, str, str] = ("outflow", "outflow", "outflow")
    deposit: str = "ngp"
    prim0: np.ndarray = field(default=None, repr=False)  # (5, nz, ny, nx) float64: e, vx, vy, vz, n
    jets: List[JetSpec] = field(default_factory=list)
    e0: float = 30.0

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])


def centres(n: int, dx: float) -> np.ndarray:
    """Cell centres of a symmetric cell-centred axis: x_i = (i - (n-1)/2) dx."""
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * dx


def ellipsoid_prim(n, dx, sigma, e0, background=1e-3, hubble=0.05, vmax=0.9) -> np.ndarray:
    """Gaussian ellipsoid e = e0 exp(-sum x_d^2 / 2 s_d^2) + background,
    Hubble-like flow v = hubble * x (per fm) rescaled to |v| <= vmax along its
    own direction, and a charge density n = 0.5 (e/e0)^(3/4) fm^-3.
    Returns (5, nz, ny, nx) float64 [e, vx, vy, vz, n]."""
    nx, ny, nz = n
    x = centres(nx, dx[0])[None, None, :]
    y = centres(ny, dx[1])[None, :, None]
    z = centres(nz, dx[2])[:, None, None]
    sx, sy, sz = sigma
    e = e0 * np.exp(-x * x / (2 * sx * sx) - y * y / (2 * sy * sy) - z * z / (2 * sz * sz)) + background
    vx = np.broadcast_to(hubble * x, e.shape)
    vy = np.broadcast_to(hubble * y, e.shape)
    vz = np.broadcast_to(hubble * z, e.shape)
    speed = np.sqrt(vx * vx + vy * vy + vz * vz)
    scale = np.where(speed > vmax, vmax / np.maximum(speed, 1e-300), 1.0)
    prim = np.empty((5, nz, ny, nx), dtype=np.float64)
    prim[0] = e
    prim[1] = vx * scale
    prim[2] = vy * scale
    prim[3] = vz * scale
    prim[4] = 0.5 * (e / e0) ** 0.75
    return prim


def _cap_direction(rng, half_angle_deg: float) -> Tuple[float, float, float]:
    """Unit vector uniform on the spherical cap of the given half-angle about +x."""
    c = rng.uniform(math.cos(math.radians(half_angle_deg)), 1.0)
    phi = rng.uniform(0.0, 2 * math.pi)
    s = math.sqrt(max(0.0, 1.0 - c * c))
    return (c, s * math.cos(phi), s * math.sin(phi))


def _isotropic(rng) -> Tuple[float, float, float]:
    c = rng.uniform(-1.0, 1.0)
    phi = rng.uniform(0.0, 2 * math.pi)
    s = math.sqrt(max(0.0, 1.0 - c * c))
    return (c, s * math.cos(phi), s * math.sin(phi))


def small_event(seed: int = 1, n=(32, 32, 32), steps: int = 10, with_jet: bool = True) -> Workload:
    """32^3 event: e0 = 30 GeV/fm^3 jittered +-10 % (first draw of the seed),
    widths (0.6, 0.9, 1.2) fm, one 50 GeV jet from (-0.8, 0, 0) fm along +x."""
    rng = np.random.default_rng(seed)
    e0 = 30.0 * (1.0 + 0.1 * (2.0 * rng.random() - 1.0))
    dx = (0.1, 0.1, 0.1)
    prim = ellipsoid_prim(n, dx, (0.6, 0.9, 1.2), e0)
    jets = [JetSpec(x0=(-0.8, 0.0, 0.0))] if with_jet else []
    return Workload("small_event_%dx%dx%d" % tuple(n), tuple(n), dx, 0.02, 1.0, steps, prim0=prim, jets=jets, e0=e0)


def paper_event(seed: int = 2, n=(256, 256, 256), steps: int = 120) -> Workload:
    """The paper's shape: 256^3, dx = 0.1 fm, dt = 0.02 fm/c, t = 1 -> 3.4 fm/c.
    Widths (4, 6, 8) fm, e0 = 30 GeV/fm^3, one jet from a seeded point of the
    x = -6 fm plane (y, z uniform in [-3, 3] fm), direction uniform in the 30
    degree cap about +x, energy uniform in [20, 100] GeV."""
    rng = np.random.default_rng(seed)
    y0 = rng.uniform(-3.0, 3.0)
    z0 = rng.uniform(-3.0, 3.0)
    d = _cap_direction(rng, 30.0)
    E = rng.uniform(20.0, 100.0)
    dx = (0.1, 0.1, 0.1)
    prim = ellipsoid_prim(n, dx, (4.0, 6.0, 8.0), 30.0)
    jets = [JetSpec(x0=(-6.0, y0, z0), dir=d, E0=E)]
    return Workload("paper_event_%dx%dx%d" % tuple(n), tuple(n), dx, 0.02, 1.0, steps, prim0=prim, jets=jets)


def fp32_event(seed: int = 3, n=(256, 256, 256), njets: int = 3) -> Workload:
    """The small event's initial state (in fm) on a large grid with 1-3 jets:
    jet 0 is the small event's jet, the others start uniformly in the ball
    r <= 1 fm with isotropic directions and 20-100 GeV.  At 512^3 the grid
    spacing halves (dx = 0.05 fm, dt = 0.01 fm/c, 60 steps)."""
    rng = np.random.default_rng(seed)
    e0 = 30.0 * (1.0 + 0.1 * (2.0 * rng.random() - 1.0))
    if n[0] >= 512:
        dx, dt, steps = (0.05, 0.05, 0.05), 0.01, 60
    else:
        dx, dt, steps = (0.1, 0.1, 0.1), 0.02, 120
    prim = ellipsoid_prim(n, dx, (0.6, 0.9, 1.2), e0)
    jets = [JetSpec(x0=(-0.8, 0.0, 0.0))]
    for _ in range(max(0, njets - 1)):
        while True:
            p = rng.uniform(-1.0, 1.0, size=3)
            if float(p @ p) <= 1.0:
                break
        jets.append(JetSpec(x0=tuple(float(v) for v in p), dir=_isotropic(rng), E0=float(rng.uniform(20, 100))))
    return Workload("fp32_event_%dx%dx%d" % tuple(n), tuple(n), dx, dt, 1.0, steps, prim0=prim, jets=jets, e0=e0)


def ensemble(seed: int = 4, n_events: int = 64, edges=(64, 96, 128), steps: int = 50) -> List[Workload]:
    """Uneven ensemble: each axis edge drawn from `edges`; widths uniform in
    0.2-0.35 of the box edge, e0 uniform in 20-40 GeV/fm^3, 0-3 jets with
    origins uniform in [-L/4, L/4]^3, isotropic directions, 20-100 GeV."""
    out = []
    for k, ss in enumerate(np.random.SeedSequence(seed).spawn(n_events)):
        rng = np.random.default_rng(ss)
        n = tuple(int(rng.choice(edges)) for _ in range(3))
        dx = (0.1, 0.1, 0.1)
        L = [n[d] * dx[d] for d in range(3)]
        sig = tuple(float(rng.uniform(0.2, 0.35) * L[d]) for d in range(3))
        e0 = float(rng.uniform(20.0, 40.0))
        prim = ellipsoid_prim(n, dx, sig, e0)
        jets = []
        for _ in range(int(rng.integers(0, 4))):
            x0 = tuple(float(rng.uniform(-L[d] / 4, L[d] / 4)) for d in range(3))
            jets.append(JetSpec(x0=x0, dir=_isotropic(rng), E0=float(rng.uniform(20.0, 100.0))))
        out.append(Workload("ensemble_%d" % k, n, dx, 0.02, 1.0, steps, prim0=prim, jets=jets, e0=e0))
    return out


def gradient_event(seed: int = 5, n=(128, 128, 128), steps: int = 100) -> Workload:
    """Differentiable run: widths (2, 3, 4) fm, e0 = 30 GeV/fm^3, one 50 GeV
    jet along +x with a Gaussian deposit.  The origin sits off the cell faces
    so that finite differences never see the deposit footprint jump."""
    del seed
    dx = (0.1, 0.1, 0.1)
    prim = ellipsoid_prim(n, dx, (2.0, 3.0, 4.0), 30.0)
    jets = [JetSpec(x0=(-3.0045, 0.37, 0.013))]
    return Workload("gradient_event_%dx%dx%d" % tuple(n), tuple(n), dx, 0.02, 1.0, steps, deposit="gauss",
                    prim0=prim, jets=jets)


def small_gradient_event(n=(32, 32, 32), steps: int = 10) -> Workload:
    """32^3 version of the differentiable run (small event's initial state)."""
    w = small_event(seed=1, n=n, steps=steps, with_jet=False)
    w.name = "small_gradient_event_%dx%dx%d" % tuple(n)
    w.deposit = "gauss"
    w.jets = [JetSpec(x0=(-0.8345, 0.031, 0.013))]
    return w


def uniform_prim(n, e=3.0, v=(0.3, -0.2, 0.1), nn=0.7) -> np.ndarray:
    nx, ny, nz = n
    prim = np.empty((5, nz, ny, nx))
    prim[0], prim[1], prim[2], prim[3], prim[4] = e, v[0], v[1], v[2], nn
    return prim


def peripheral_jet_event(n=(24, 20, 22), steps: int = 30, mirror: bool = False) -> Workload:
    """A 92 GeV jet crossing the dilute edge of a small fireball (widths 0.2 of
    the box, e0 = 27 GeV/fm^3, background 1e-3) with an NGP deposit: the kind
    of event in which the unlimited WENO scheme leaves E < |M| behind the
    deposit.  The origin sits off the cell faces; mirror=True gives the x ->
    -x mirror image."""
    dx = (0.1, 0.1, 0.1)
    L = [n[k] * dx[k] for k in range(3)]
    prim = ellipsoid_prim(n, dx, tuple(0.2 * x for x in L), 27.0)
    d = (-0.9916173911378503, 0.02872803653083503, 0.12597479712246648)
    x0 = (0.25 * L[0] + 0.0137, -L[0] / 3.2, -1.2 * L[0] / 3.2)
    if mirror:
        prim = prim[:, :, :, ::-1].copy()
        prim[1] = -prim[1]
        d = (-d[0], d[1], d[2])
        x0 = (-x0[0], x0[1], x0[2])
    jets = [JetSpec(x0=x0, dir=d, E0=92.3)]
    return Workload("peripheral_jet_%dx%dx%d" % tuple(n), tuple(n), dx, 0.02, 1.0, steps, prim0=prim, jets=jets,
                    e0=27.0)


def vacuum_riemann(N: int = 200, e_right: float = 1e-8, axis: int = 0, ntrans: int = 4) -> Workload:
    """Riemann problem of a fluid at rest, e = 10 | e_right (GeV/fm^3), charge
    n = 1 | (e_right/10)^(3/4), on [-1, 1] fm along `axis` (outflow), ntrans
    periodic cells across; dt = 0.2 dx, t = 0 -> 0.4 fm/c."""
    dx = [1.0, 1.0, 1.0]
    dx[axis] = 2.0 / N
    n = [ntrans, ntrans, ntrans]
    n[axis] = N
    bc = ["periodic"] * 3
    bc[axis] = "outflow"
    dt = 0.2 * dx[axis]
    x = centres(N, dx[axis])
    shape = [1, 1, 1]
    shape[2 - axis] = N
    left = (x < 0).reshape(shape)
    prim = np.zeros((5, n[2], n[1], n[0]))
    prim[0] = np.where(left, 10.0, e_right)
    prim[4] = np.where(left, 1.0, (e_right / 10.0) ** 0.75)
    return Workload("vacuum_riemann_%d_axis%d" % (N, axis), tuple(n), tuple(dx), dt, 0.0, int(round(0.4 / dt)),
                    bc=tuple(bc), prim0=prim, jets=[])
