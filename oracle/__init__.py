"""CPU oracle for the jet + ideal-hydro stage -- TEST INFRASTRUCTURE ONLY.

A plain FP64 implementation (``hydro_oracle.cpp``) of the scheme the paper
describes: Eq. (1) ideal hydrodynamics with a source, Eq. (2) point sources of
jets, Eq. (3) energy loss, 7th-order WENO (5th order as the alternative the
paper also names) and third-order Runge-Kutta
(section "Simulation setup"), EOS p = e/3 (Fig. 3 caption).  This module only
marshals numpy arrays into that library through ctypes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product library never does; it shares no code
with this directory.

Parity status per function (pins in tests/test_oracle_*.py):
  weno7, weno5     pinned (sympy derivation, polynomial exactness, order)
  cons_to_prim     pinned (round trip, quadratic identity)
  prim_to_cons     pinned (round trip)
  rhs / run        pinned (uniform state, mirror symmetry, conservation,
                   convergence order, exact Riemann solution, energy budget,
                   source closed form)
  sums             pinned (numpy sum)
  eps2             pinned (closed form on a separable field; z = 0 planes
                   with hot cells next to them)
  freezeout        pinned (static uniform medium: closed form and v_n = 0;
                   boosted uniform medium: quadrature of the analytic
                   spectrum; p_T integral of the differential rows against
                   the integrated row; isotropic fireball: v_1..v_3 = 0;
                   mirror images; particle number against the Boltzmann
                   density's closed form)
  eps2_complex_step pinned (central finite differences of run)
  jvp              pinned (central finite differences of run)
  musta_flux, run with flux="musta"
                   pinned (consistency, stage fixed point, mirror symmetry,
                   second order on smooth data, Riemann convergence with
                   near-monotone profiles, conservation, symmetries)
  limit_face, run with limiter="pp"
                   pinned (admissibility invariant, brute-force largest
                   theta, exact root for linear constraints, inactive on
                   smooth flows, conservation, the LF premise u +- f(u))
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# HYDRO_ORACLE_LIB names another build of the same source (the sanitized one
# that oracle/build_oracle.py --sanitize writes), for a child process only.
_LIB_PATH = os.environ.get("HYDRO_ORACLE_LIB") or os.path.join(_HERE, "libhydro_oracle.so")
_lib = None


class OCfg(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double * 3),
        ("t0", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("bc", ctypes.c_int32 * 3),
        ("weno", ctypes.c_int32),
        ("deposit", ctypes.c_int32),
        ("weno_p", ctypes.c_int32),
        ("weno_eps", ctypes.c_double),
        ("eos_dof", ctypes.c_double),
        ("hbarc", ctypes.c_double),
        ("limiter", ctypes.c_int32),
        ("flux", ctypes.c_int32),
        ("musta_k", ctypes.c_int32),
    ]


class OJet(ctypes.Structure):
    _fields_ = [
        ("x0", ctypes.c_double * 3),
        ("dir", ctypes.c_double * 3),
        ("E0", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("kappa_rad", ctypes.c_double),
        ("kappa_coll", ctypes.c_double),
        ("cr_over_cf", ctypes.c_double),
    ]


WENO = {"z": 0, "js": 1, "linear": 2, "z5": 3, "js5": 4, "linear5": 5}
BC = {"outflow": 0, "periodic": 1}
DEPOSIT = {"ngp": 0, "gauss": 1}
LIMITER = {"none": 0, "pp": 1}
FLUX = {"weno": 0, "musta": 1}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    stale = not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(
        os.path.join(_HERE, "hydro_oracle.cpp"))
    if stale and not os.environ.get("HYDRO_ORACLE_LIB"):
        from . import build_oracle
        build_oracle.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    llp = ctypes.POINTER(ctypes.c_longlong)
    cp = ctypes.POINTER(OCfg)
    jp = ctypes.POINTER(OJet)
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_weno7.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.oracle_weno7.restype = ctypes.c_double
    lib.oracle_weno5.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.oracle_weno5.restype = ctypes.c_double
    lib.oracle_prim_to_cons.argtypes = [cp, dp, dp]
    lib.oracle_cons_to_prim.argtypes = [cp, dp, dp, llp]
    lib.oracle_rhs.argtypes = [cp, jp, ctypes.c_int, ip, dp, ctypes.c_double, dp, dp, llp]
    lib.oracle_run.argtypes = [cp, jp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_longlong, dp, dp, llp]
    lib.oracle_sums.argtypes = [cp, dp, dp]
    lib.oracle_eps2.argtypes = [cp, dp, dp]
    lib.oracle_eps2_complex_step.argtypes = [cp, jp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_double, dp, dp, dp]
    lib.oracle_jvp.argtypes = [cp, jp, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, dp, dp]
    lib.oracle_freezeout.argtypes = [cp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, dp, dp, llp]
    lib.oracle_limit_face.argtypes = [cp, ctypes.c_int, dp, dp, dp, dp]
    lib.oracle_musta_flux.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, dp]
    lib.oracle_count_flops.argtypes = [ctypes.c_int, ctypes.c_int, llp]
    for name in ("oracle_prim_to_cons", "oracle_cons_to_prim", "oracle_rhs", "oracle_run",
                 "oracle_sums", "oracle_eps2", "oracle_eps2_complex_step", "oracle_jvp", "oracle_limit_face",
                 "oracle_musta_flux", "oracle_count_flops", "oracle_freezeout"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Problem:
    """Grid, time step and scheme switches (defaults: the paper's shape)."""
    n: Sequence[int] = (32, 32, 32)
    dx: Sequence[float] = (0.1, 0.1, 0.1)
    t0: float = 1.0
    dt: float = 0.02
    bc: Sequence[str] = ("outflow", "outflow", "outflow")
    weno: str = "z"
    deposit: str = "ngp"
    weno_p: int = 2
    weno_eps: float = 1e-6
    eos_dof: float = 47.5
    hbarc: float = 0.1973269804
    limiter: str = "none"
    flux: str = "weno"      # "weno": WENO of the LF split fluxes; "musta": MUSTA-FORCE
    musta_k: int = 2

    def c(self) -> OCfg:
        c = OCfg()
        for d in range(3):
            c.n[d] = int(self.n[d])
            c.dx[d] = float(self.dx[d])
            c.bc[d] = BC[self.bc[d]] if isinstance(self.bc[d], str) else int(self.bc[d])
        c.t0, c.dt = float(self.t0), float(self.dt)
        c.weno = WENO[self.weno]
        c.deposit = DEPOSIT[self.deposit]
        c.weno_p = int(self.weno_p)
        c.weno_eps = float(self.weno_eps)
        c.eos_dof = float(self.eos_dof)
        c.hbarc = float(self.hbarc)
        c.limiter = LIMITER[self.limiter] if isinstance(self.limiter, str) else int(self.limiter)
        c.flux = FLUX[self.flux] if isinstance(self.flux, str) else int(self.flux)
        c.musta_k = int(self.musta_k)
        return c

    @property
    def shape(self):
        return (int(self.n[2]), int(self.n[1]), int(self.n[0]))

    @property
    def ncell(self):
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclass
class Jet:
    x0: Sequence[float]
    dir: Sequence[float] = (1.0, 0.0, 0.0)
    E0: float = 50.0
    t_start: float = 1.0
    kappa_rad: float = 4.0
    kappa_coll: float = 2.5
    cr_over_cf: float = 1.0

    def c(self) -> OJet:
        j = OJet()
        for d in range(3):
            j.x0[d] = float(self.x0[d])
            j.dir[d] = float(self.dir[d])
        j.E0, j.t_start = float(self.E0), float(self.t_start)
        j.kappa_rad, j.kappa_coll, j.cr_over_cf = float(self.kappa_rad), float(self.kappa_coll), float(
            self.cr_over_cf)
        return j


def _jets(jets):
    jets = list(jets or [])
    arr = (OJet * max(1, len(jets)))()
    for i, j in enumerate(jets):
        arr[i] = j.c() if isinstance(j, Jet) else j
    return arr, len(jets)


def threads() -> int:
    """OpenMP threads the oracle runs on."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Run later oracle calls on n OpenMP threads."""
    _load().oracle_set_threads(int(n))


def weno5(a, scheme: str = "z", eps: float = 1e-6, p: int = 2) -> float:
    """WENO5 value at x_{i+1/2} from a_{i-2}..a_{i+2}; scheme z, js or linear."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == (5,)
    return float(_load().oracle_weno5(_dp(a), WENO[scheme], eps, p))


def weno7(a, scheme: str = "z", eps: float = 1e-6, p: int = 2) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == (7,)
    return float(_load().oracle_weno7(_dp(a), WENO[scheme], eps, p))


def prim_to_cons(pb: Problem, prim: np.ndarray) -> np.ndarray:
    prim = np.ascontiguousarray(prim, dtype=np.float64).reshape(5, *pb.shape)
    U = np.empty_like(prim)
    c = pb.c()
    rc = _load().oracle_prim_to_cons(ctypes.byref(c), _dp(prim), _dp(U))
    assert rc == 0
    return U


def cons_to_prim(pb: Problem, U: np.ndarray):
    """Returns ([e, vx, vy, vz, n, T] of shape (6, nz, ny, nx), fix-up count)."""
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(5, *pb.shape)
    out = np.empty((6,) + pb.shape)
    fx = ctypes.c_longlong(0)
    c = pb.c()
    rc = _load().oracle_cons_to_prim(ctypes.byref(c), _dp(U), _dp(out), ctypes.byref(fx))
    assert rc == 0
    return out, fx.value


def rhs(pb: Problem, U: np.ndarray, t: float, jets=None, chi=None):
    """L(U) = D(U) + S(U); returns (L, P_eff per jet, fix-ups)."""
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(5, *pb.shape)
    L = np.empty_like(U)
    arr, nj = _jets(jets)
    P = np.zeros(max(1, nj))
    chi_arr = (ctypes.c_int * max(1, nj))(*([1] * max(1, nj) if chi is None else list(chi)))
    fx = ctypes.c_longlong(0)
    c = pb.c()
    rc = _load().oracle_rhs(ctypes.byref(c), arr, nj, chi_arr, _dp(U), float(t), _dp(L), _dp(P),
                            ctypes.byref(fx))
    assert rc == 0
    return L, P[:nj], fx.value


@dataclass
class RunState:
    U: np.ndarray
    step: int = 0
    Ejet: np.ndarray = field(default_factory=lambda: np.zeros(0))
    ledger: float = 0.0
    fixups: int = 0


def run(pb: Problem, U: np.ndarray, nsteps: int, jets=None, step0: int = 0, Ejet=None,
        ledger: float = 0.0) -> RunState:
    """nsteps SSP-RK3 steps from step index step0; returns the new state."""
    U = np.array(U, dtype=np.float64, copy=True).reshape(5, *pb.shape)
    arr, nj = _jets(jets)
    if Ejet is None:
        Ejet = np.array([j.E0 for j in (jets or [])], dtype=np.float64)
    E = np.zeros(max(1, nj))
    E[:nj] = Ejet
    led = ctypes.c_double(ledger)
    fx = ctypes.c_longlong(0)
    c = pb.c()
    rc = _load().oracle_run(ctypes.byref(c), arr, nj, _dp(U), int(nsteps), int(step0), _dp(E),
                            ctypes.byref(led), ctypes.byref(fx))
    assert rc == 0
    return RunState(U=U, step=step0 + nsteps, Ejet=E[:nj].copy(), ledger=led.value, fixups=fx.value)


def sums(pb: Problem, U: np.ndarray) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(5, *pb.shape)
    out = np.zeros(5)
    c = pb.c()
    assert _load().oracle_sums(ctypes.byref(c), _dp(U), _dp(out)) == 0
    return out


def eps2(pb: Problem, U: np.ndarray) -> float:
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(5, *pb.shape)
    out = ctypes.c_double(0.0)
    c = pb.c()
    assert _load().oracle_eps2(ctypes.byref(c), _dp(U), ctypes.byref(out)) == 0
    return out.value


EPS2_PARAM = {"kappa_rad": 0, "kappa_coll": 1, "x0": 2, "y0": 3, "z0": 4, "e_init": 5}


def eps2_complex_step(pb: Problem, prim0: np.ndarray, nsteps: int, jets, which: str, jet: int = 0,
                      h: float = 1e-30, de: np.ndarray | None = None):
    """(eps2, d eps2 / d input) by the complex-step method."""
    prim0 = np.ascontiguousarray(prim0, dtype=np.float64).reshape(5, *pb.shape)
    arr, nj = _jets(jets)
    val = ctypes.c_double(0.0)
    der = ctypes.c_double(0.0)
    dptr = None
    if de is not None:
        de = np.ascontiguousarray(de, dtype=np.float64).reshape(pb.shape)
        dptr = _dp(de)
    c = pb.c()
    rc = _load().oracle_eps2_complex_step(ctypes.byref(c), arr, nj, _dp(prim0), int(nsteps),
                                          EPS2_PARAM[which], int(jet), float(h), dptr,
                                          ctypes.byref(val), ctypes.byref(der))
    assert rc == 0
    return val.value, der.value


def jvp(pb: Problem, U0: np.ndarray, V: np.ndarray, nsteps: int, jets=None, h: float = 1e-30):
    """(U(nsteps), J V) of nsteps steps from step 0 by the complex-step method:
    the run from U0 + i h V, jets at their E0."""
    U0 = np.ascontiguousarray(U0, dtype=np.float64).reshape(5, *pb.shape)
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(5, *pb.shape)
    arr, nj = _jets(jets)
    Uo = np.empty_like(U0)
    JV = np.empty_like(U0)
    c = pb.c()
    rc = _load().oracle_jvp(ctypes.byref(c), arr, nj, _dp(U0), _dp(V), int(nsteps), float(h), _dp(Uo), _dp(JV))
    assert rc == 0
    return Uo, JV


def freezeout(pb: Problem, U: np.ndarray, n_phi: int = 64, pt=(), T_min: float = 0.0, dof: float = 1.0,
              n_harm: int = 8):
    """Cooper-Frye freeze-out of U on its fixed-time surface, massless
    Boltzmann particles of degeneracy dof, at rapidity 0 along z.  Returns
    (spectra, harm, fixups): spectra[0, k] = dN/(dy dphi) and
    spectra[1 + j, k] = dN/(p_T dp_T dy dphi) at p_T = pt[j] [GeV^-2], at
    phi_k = 2 pi k / n_phi; harm[r, 0, 0] = dN/dy of row r and
    harm[r, n] = (<cos n phi>, <sin n phi>) of row r."""
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(5, *pb.shape)
    pt = np.ascontiguousarray(np.array(pt, dtype=np.float64).reshape(-1))
    npt = int(pt.size)
    spec = np.zeros((1 + npt, int(n_phi)))
    harm = np.zeros((1 + npt, int(n_harm) + 1, 2))
    fx = ctypes.c_longlong(0)
    c = pb.c()
    ptp = _dp(pt) if npt else None
    rc = _load().oracle_freezeout(ctypes.byref(c), _dp(U), int(n_phi), npt, ptp, float(T_min), float(dof),
                                  int(n_harm), _dp(spec), _dp(harm), ctypes.byref(fx))
    assert rc == 0
    return spec, harm, fx.value


def limit_face(pb: Problem, d: int, uA, uB, H):
    """The positivity-preserving limiter on one face along axis d (0 x, 1 y,
    2 z) between conserved states uA (low side) and uB: (limited H, theta)."""
    uA = np.ascontiguousarray(uA, dtype=np.float64)
    uB = np.ascontiguousarray(uB, dtype=np.float64)
    Hc = np.array(H, dtype=np.float64)
    th = ctypes.c_double()
    c = pb.c()
    rc = _load().oracle_limit_face(ctypes.byref(c), int(d), _dp(uA), _dp(uB), _dp(Hc), ctypes.byref(th))
    assert rc == 0
    return Hc, th.value


def musta_flux(d: int, uL, uR, k: int, states: bool = False):
    """MUSTA-FORCE flux along axis d of the face states uL, uR (k stages); with
    states=True also the local states the last stage started from."""
    a = np.ascontiguousarray(uL, dtype=np.float64)
    b = np.ascontiguousarray(uR, dtype=np.float64)
    F, ak, bk = np.empty(5), np.empty(5), np.empty(5)
    assert _load().oracle_musta_flux(int(d), _dp(a), _dp(b), int(k), _dp(F), _dp(ak), _dp(bk)) == 0
    return (F, ak, bk) if states else F


def count_flops(what: str, scheme: str = "z"):
    """{add, mul, div, sqrt} counts of one plain-formulation call: what =
    "weno7", "weno5" (scheme z, js or linear) or "c2p"."""
    out = (ctypes.c_longlong * 4)()
    code = {"weno7": 0, "weno5": 1, "c2p": 2}[what]
    assert _load().oracle_count_flops(code, {"z": 0, "js": 1, "linear": 2}[scheme], out) == 0
    return dict(zip(("add", "mul", "div", "sqrt"), list(out)))
