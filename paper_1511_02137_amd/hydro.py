"""Python binding of libhydro (include/hydro.h) through ctypes.

Argument marshalling only: torch tensors provide device memory and the
stream; every step of the computation runs in the library's HIP kernels.
If the library is missing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhydro.so")

HYDRO_OK, HYDRO_EINVAL, HYDRO_ENOMEM, HYDRO_EDEVICE, HYDRO_ENONPHYS, HYDRO_ESTATE = 0, -1, -2, -3, -4, -5
F64, F32 = 0, 1
BC = {"outflow": 0, "periodic": 1}
WENO = {"z": 0, "js": 1, "linear": 2, "z5": 3, "js5": 4, "linear5": 5}
DEPOSIT = {"ngp": 0, "gauss": 1}
LIMITER = {"none": 0, "pp": 1}
FLUX = {"weno": 0, "musta": 1}

EXPORTED = [
    "hydro_default_config", "hydro_workspace_bytes", "hydro_init", "hydro_add_jet", "hydro_rk3_step",
    "hydro_primitives", "hydro_rhs", "hydro_sums", "hydro_get_state", "hydro_set_state", "hydro_diag",
    "hydro_last_error", "hydro_destroy", "hydro_profile", "hydro_profile_read", "hydro_set_option",
    "hydro_get_option", "hydro_reset", "hydro_set_jet", "hydro_loss_eps2", "hydro_adjoint_step",
    "hydro_init_vjp", "hydro_batch_workspace_bytes", "hydro_batch_create", "hydro_batch_add_jet", "hydro_batch_run",
    "hydro_batch_rhs", "hydro_batch_set_option", "hydro_batch_get_option", "hydro_batch_autotune",
    "hydro_batch_sums", "hydro_batch_get_state", "hydro_batch_diag", "hydro_batch_last_error",
    "hydro_batch_destroy", "hydro_sums_noalloc", "hydro_freezeout", "hydro_step_sums",
    "hydro_rk3_step_record", "hydro_adjoint_recorded",
]
OPT_YZ_KERNEL, OPT_MARCH_SEG, OPT_X_KERNEL, OPT_ADJ_SKIP_N, OPT_TILE_ORDER, OPT_ADJ_LINES = 0, 1, 2, 3, 4, 5
BOPT_BLOCKS_X, BOPT_BLOCKS_Y, BOPT_BLOCKS_Z, BOPT_GRAPH, BOPT_X_ROWS = 0, 1, 2, 3, 4
KERNELS = ["xface", "xbound", "ymarch", "jet", "zmarch", "sums", "adjoint"]


class HydroError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libhydro error %d: %s" % (code, msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double * 3),
        ("t0", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("bc", ctypes.c_int32 * 3),
        ("precision", ctypes.c_int32),
        ("weno", ctypes.c_int32),
        ("deposit", ctypes.c_int32),
        ("weno_eps", ctypes.c_double),
        ("weno_p", ctypes.c_int32),
        ("strict", ctypes.c_int32),
        ("eos_dof", ctypes.c_double),
        ("hbarc", ctypes.c_double),
        ("limiter", ctypes.c_int32),
        ("flux", ctypes.c_int32),
        ("musta_k", ctypes.c_int32),
    ]


class JetC(ctypes.Structure):
    _fields_ = [
        ("x0", ctypes.c_double * 3),
        ("dir", ctypes.c_double * 3),
        ("E0", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("kappa_rad", ctypes.c_double),
        ("kappa_coll", ctypes.c_double),
        ("cr_over_cf", ctypes.c_double),
    ]


class FreezeoutParams(ctypes.Structure):
    _fields_ = [
        ("n_phi", ctypes.c_int32),
        ("n_pt", ctypes.c_int32),
        ("n_harm", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("pt", ctypes.c_double * 15),
        ("T_min", ctypes.c_double),
        ("dof", ctypes.c_double),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhydro.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libhydro.so is not built (run paper_1511_02137_amd/build.py): " + path)
    lib = ctypes.CDLL(path)
    vp, cp, dp = ctypes.c_void_p, ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_double)
    lib.hydro_default_config.argtypes = [cp]
    lib.hydro_default_config.restype = None
    lib.hydro_workspace_bytes.argtypes = [cp, ctypes.c_int]
    lib.hydro_workspace_bytes.restype = ctypes.c_size_t
    lib.hydro_init.argtypes = [cp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.hydro_add_jet.argtypes = [vp, ctypes.POINTER(JetC), ctypes.POINTER(ctypes.c_int)]
    lib.hydro_rk3_step.argtypes = [vp, vp, ctypes.c_int, vp]
    lib.hydro_primitives.argtypes = [vp, vp, vp, vp]
    lib.hydro_rhs.argtypes = [vp, vp, ctypes.c_double, vp, vp]
    lib.hydro_sums.argtypes = [vp, vp, dp, vp]
    lib.hydro_sums_noalloc.argtypes = [vp, vp, vp, vp]
    lib.hydro_step_sums.argtypes = [vp, dp]
    lib.hydro_freezeout.argtypes = [vp, vp, ctypes.POINTER(FreezeoutParams), vp, vp, vp]
    lib.hydro_get_state.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), dp, ctypes.c_int]
    lib.hydro_set_state.argtypes = [vp, ctypes.c_int64, dp, ctypes.c_int, ctypes.c_double]
    lib.hydro_diag.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.hydro_last_error.argtypes = [vp]
    lib.hydro_last_error.restype = ctypes.c_char_p
    lib.hydro_destroy.argtypes = [vp]
    lib.hydro_destroy.restype = None
    lib.hydro_profile.argtypes = [vp, ctypes.c_int]
    lib.hydro_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.hydro_reset.argtypes = [vp, vp, vp, vp]
    lib.hydro_set_jet.argtypes = [vp, ctypes.c_int, ctypes.POINTER(JetC)]
    lib.hydro_loss_eps2.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp]
    lib.hydro_adjoint_step.argtypes = [vp, vp, ctypes.c_int64, dp, ctypes.c_int, vp, vp, vp]
    lib.hydro_init_vjp.argtypes = [vp, vp, vp, vp, vp]
    lib.hydro_rk3_step_record.argtypes = [vp, vp, ctypes.c_int, vp]
    lib.hydro_adjoint_recorded.argtypes = [vp, vp, vp, vp]
    lib.hydro_get_option.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.hydro_profile_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.hydro_batch_workspace_bytes.argtypes = [cp, ctypes.c_int]
    lib.hydro_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.hydro_batch_create.argtypes = [cp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, ctypes.c_size_t,
                                       vp, ctypes.POINTER(vp)]
    lib.hydro_batch_add_jet.argtypes = [vp, ctypes.c_int, ctypes.POINTER(JetC), ctypes.POINTER(ctypes.c_int)]
    lib.hydro_batch_run.argtypes = [vp, ctypes.c_int, vp]
    lib.hydro_batch_rhs.argtypes = [vp, vp]
    lib.hydro_batch_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_longlong]
    lib.hydro_batch_get_option.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
    lib.hydro_batch_autotune.argtypes = [vp, ctypes.c_char_p, vp, ctypes.POINTER(ctypes.c_int)]
    lib.hydro_batch_sums.argtypes = [vp, ctypes.c_int, dp]
    lib.hydro_batch_get_state.argtypes = [vp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int64), dp, ctypes.c_int]
    lib.hydro_batch_diag.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.hydro_batch_last_error.argtypes = [vp]
    lib.hydro_batch_last_error.restype = ctypes.c_char_p
    lib.hydro_batch_destroy.argtypes = [vp]
    lib.hydro_batch_destroy.restype = None
    for name in ("hydro_batch_create", "hydro_batch_add_jet", "hydro_batch_run", "hydro_batch_rhs",
                 "hydro_batch_set_option", "hydro_batch_get_option", "hydro_batch_autotune", "hydro_batch_sums",
                 "hydro_batch_get_state", "hydro_batch_diag"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("hydro_init", "hydro_add_jet", "hydro_rk3_step", "hydro_primitives", "hydro_rhs", "hydro_sums",
                 "hydro_get_state", "hydro_set_state", "hydro_diag", "hydro_profile", "hydro_profile_read",
                 "hydro_set_option", "hydro_get_option", "hydro_reset", "hydro_set_jet", "hydro_loss_eps2",
                 "hydro_adjoint_step", "hydro_init_vjp", "hydro_sums_noalloc", "hydro_freezeout"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def make_config(n, dx=(0.1, 0.1, 0.1), dt=0.02, t0=1.0, bc=("outflow",) * 3, precision="f64", weno="z",
                deposit="ngp", weno_eps=1e-6, strict=False, eos_dof=47.5, hbarc=0.1973269804,
                limiter="none", flux="weno", musta_k=2) -> Config:
    lib = load_library()
    c = Config()
    lib.hydro_default_config(ctypes.byref(c))
    for d in range(3):
        c.n[d] = int(n[d])
        c.dx[d] = float(dx[d])
        c.bc[d] = BC[bc[d]] if isinstance(bc[d], str) else int(bc[d])
    c.t0, c.dt = float(t0), float(dt)
    c.precision = F32 if precision in ("f32", F32) else F64
    c.weno = WENO[weno] if isinstance(weno, str) else int(weno)
    c.deposit = DEPOSIT[deposit] if isinstance(deposit, str) else int(deposit)
    c.weno_eps = float(weno_eps)
    c.strict = 1 if strict else 0
    c.eos_dof, c.hbarc = float(eos_dof), float(hbarc)
    c.limiter = LIMITER[limiter] if isinstance(limiter, str) else int(limiter)
    c.flux = FLUX[flux] if isinstance(flux, str) else int(flux)
    c.musta_k = int(musta_k)
    return c


def workspace_bytes(cfg: Config, adjoint_k: int = 0) -> int:
    return int(load_library().hydro_workspace_bytes(ctypes.byref(cfg), int(adjoint_k)))


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Hydro:
    """One event on one GPU: conserved fields U (torch, [5, nz, ny, nx]) and
    the library context.  prim0: (5, nz, ny, nx) float64 [e, vx, vy, vz, n]
    as numpy (host) or a torch tensor (host or device)."""

    def __init__(self, cfg: Config, prim0, device: str = "cuda", adjoint_k: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libhydro needs a GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.cfg = cfg
        self.device = torch.device(device)
        self.dtype = torch.float32 if cfg.precision == F32 else torch.float64
        nx, ny, nz = cfg.n[0], cfg.n[1], cfg.n[2]
        self.shape = (nz, ny, nx)
        self.U = torch.empty((5, nz, ny, nx), dtype=self.dtype, device=self.device)
        nbytes = workspace_bytes(cfg, adjoint_k)
        if nbytes == 0:
            raise HydroError(HYDRO_EINVAL, "invalid configuration")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self._ws_ptr = self.ws.data_ptr() + off
        self._ws_bytes = nbytes
        if prim0 is None:
            pptr = None
            self._prim_keep = None
        elif isinstance(prim0, np.ndarray):
            p = np.ascontiguousarray(prim0, dtype=np.float64)
            assert p.shape == (5, nz, ny, nx), p.shape
            self._prim_keep = p
            pptr = p.ctypes.data
        else:
            p = prim0.to(dtype=torch.float64).contiguous()
            assert tuple(p.shape) == (5, nz, ny, nx)
            self._prim_keep = p
            pptr = p.data_ptr()
        h = ctypes.c_void_p()
        rc = self.lib.hydro_init(ctypes.byref(cfg), pptr, self.U.data_ptr(), self._ws_ptr, self._ws_bytes,
                                 _stream_handle(), ctypes.byref(h))
        if rc != HYDRO_OK:
            raise HydroError(rc, self.lib.hydro_last_error(None).decode())
        self.ctx = h
        self.njet = 0

    def _check(self, rc):
        if rc != HYDRO_OK:
            raise HydroError(rc, self.lib.hydro_last_error(self.ctx).decode())

    @staticmethod
    def _jet(x0, dir, E0, t_start, kappa_rad, kappa_coll, cr_over_cf) -> JetC:
        j = JetC()
        for d in range(3):
            j.x0[d] = float(x0[d])
            j.dir[d] = float(dir[d])
        j.E0, j.t_start = float(E0), float(t_start)
        j.kappa_rad, j.kappa_coll, j.cr_over_cf = float(kappa_rad), float(kappa_coll), float(cr_over_cf)
        return j

    def set_jet(self, jid: int, x0, dir=(1.0, 0.0, 0.0), E0=50.0, t_start=1.0, kappa_rad=4.0, kappa_coll=2.5,
                cr_over_cf=1.0):
        j = self._jet(x0, dir, E0, t_start, kappa_rad, kappa_coll, cr_over_cf)
        self._check(self.lib.hydro_set_jet(self.ctx, int(jid), ctypes.byref(j)))

    def reset(self, prim0, stream=None):
        """U from device FP64 primitives (5, nz, ny, nx); step 0, jet energies E0, ledger 0."""
        import torch
        p = prim0.to(device=self.device, dtype=torch.float64).contiguous()
        self._prim_keep = p
        self._check(self.lib.hydro_reset(self.ctx, p.data_ptr(), self.U.data_ptr(), _stream_handle(stream)))

    def loss_eps2(self, U=None, seed=None, scale: float = 1.0, stream=None):
        """eps2 of U as a device float64 scalar; if seed is a tensor like U it
        receives scale * d eps2 / dU."""
        import torch
        U = self.U if U is None else U
        out = torch.empty((), dtype=torch.float64, device=self.device)
        sp = seed.data_ptr() if seed is not None else None
        self._check(self.lib.hydro_loss_eps2(self.ctx, U.data_ptr(), out.data_ptr(), sp, float(scale),
                                             _stream_handle(stream)))
        return out

    def adjoint_step(self, U_ckpt, step0: int, E_jet0, nsteps: int, lam, grad_jets, stream=None):
        """Reverse sweep over nsteps steps from checkpoint U_ckpt (step step0,
        jet energies E_jet0); lam (like U) in: dJ/dU(step0+nsteps), out:
        dJ/dU(step0); grad_jets (njet, 5) float64 device tensor is incremented."""
        E = (ctypes.c_double * max(1, self.njet))(*[float(v) for v in (E_jet0 if E_jet0 is not None else [])])
        gp = grad_jets.data_ptr() if grad_jets is not None else None
        self._check(self.lib.hydro_adjoint_step(self.ctx, U_ckpt.data_ptr(), int(step0), E if self.njet else None,
                                                int(nsteps), lam.data_ptr(), gp, _stream_handle(stream)))

    def step_record(self, nsteps: int, stream=None):
        """hydro_rk3_step_record: nsteps steps (as step) keeping their stage
        states in the adjoint workspace for adjoint_recorded."""
        self._check(self.lib.hydro_rk3_step_record(self.ctx, self.U.data_ptr(), int(nsteps), _stream_handle(stream)))

    def adjoint_recorded(self, lam, grad_jets, stream=None):
        """hydro_adjoint_recorded: reverse sweep over the recorded steps; lam
        (like U) in: dJ/dU after them, out: before them; grad_jets (njet, 5)
        float64 device tensor is incremented."""
        gp = grad_jets.data_ptr() if grad_jets is not None else None
        self._check(self.lib.hydro_adjoint_recorded(self.ctx, lam.data_ptr(), gp, _stream_handle(stream)))

    def init_vjp(self, prim0, lam, stream=None):
        """(dU/dprim)^T lam at prim0 (device float64) -> (5, nz, ny, nx) float64."""
        import torch
        p = prim0.to(device=self.device, dtype=torch.float64).contiguous()
        out = torch.empty((5,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.hydro_init_vjp(self.ctx, p.data_ptr(), lam.data_ptr(), out.data_ptr(),
                                            _stream_handle(stream)))
        return out

    def add_jet(self, x0, dir=(1.0, 0.0, 0.0), E0=50.0, t_start=1.0, kappa_rad=4.0, kappa_coll=2.5,
                cr_over_cf=1.0) -> int:
        j = JetC()
        for d in range(3):
            j.x0[d] = float(x0[d])
            j.dir[d] = float(dir[d])
        j.E0, j.t_start = float(E0), float(t_start)
        j.kappa_rad, j.kappa_coll, j.cr_over_cf = float(kappa_rad), float(kappa_coll), float(cr_over_cf)
        jid = ctypes.c_int(-1)
        self._check(self.lib.hydro_add_jet(self.ctx, ctypes.byref(j), ctypes.byref(jid)))
        self.njet += 1
        return jid.value

    def step(self, nsteps: int = 1, stream=None):
        self._check(self.lib.hydro_rk3_step(self.ctx, self.U.data_ptr(), int(nsteps), _stream_handle(stream)))

    def rhs(self, U=None, t: float = None, stream=None):
        """L(U) = D(U) + S(U) at time t (default: the current step's time)."""
        import torch
        U = self.U if U is None else U
        if t is None:
            t = self.get_state()[0]
        out = torch.empty_like(U)
        self._check(self.lib.hydro_rhs(self.ctx, U.data_ptr(), float(t), out.data_ptr(), _stream_handle(stream)))
        return out

    def primitives(self, U=None, stream=None):
        import torch
        U = self.U if U is None else U
        out = torch.empty((6,) + self.shape, dtype=self.dtype, device=self.device)
        self._check(self.lib.hydro_primitives(self.ctx, U.data_ptr(), out.data_ptr(), _stream_handle(stream)))
        return out

    def sums(self, U=None, stream=None) -> np.ndarray:
        U = self.U if U is None else U
        out = (ctypes.c_double * 6)()
        self._check(self.lib.hydro_sums(self.ctx, U.data_ptr(), out, _stream_handle(stream)))
        return np.array(list(out))

    def step_sums(self) -> np.ndarray:
        """hydro_step_sums: the sums taken by the last step and the ledger."""
        out = (ctypes.c_double * 6)()
        self._check(self.lib.hydro_step_sums(self.ctx, out))
        return np.array(list(out))

    def sums_noalloc(self, out, U=None, stream=None):
        """hydro_sums_noalloc: the sums and the ledger into out (a device
        float64 tensor of 6 elements), asynchronously, with no allocation."""
        U = self.U if U is None else U
        self._check(self.lib.hydro_sums_noalloc(self.ctx, U.data_ptr(), out.data_ptr(), _stream_handle(stream)))
        return out

    def freezeout(self, n_phi: int = 64, pt=(), T_min: float = 0.0, dof: float = 1.0, n_harm: int = 8, U=None,
                  stream=None):
        """hydro_freezeout: (spectra [1 + n_pt, n_phi], harm [1 + n_pt, n_harm + 1, 2]) as device
        float64 tensors (written asynchronously on the stream)."""
        import torch
        U = self.U if U is None else U
        pt = [float(v) for v in pt]
        fp = FreezeoutParams()
        fp.n_phi, fp.n_pt, fp.n_harm, fp.reserved = int(n_phi), len(pt), int(n_harm), 0
        for j, v in enumerate(pt[:15]):
            fp.pt[j] = v
        fp.T_min, fp.dof = float(T_min), float(dof)
        spec = torch.empty((1 + len(pt), int(n_phi)), dtype=torch.float64, device=self.device)
        harm = torch.empty((1 + len(pt), int(n_harm) + 1, 2), dtype=torch.float64, device=self.device)
        self._check(self.lib.hydro_freezeout(self.ctx, U.data_ptr(), ctypes.byref(fp), spec.data_ptr(),
                                             harm.data_ptr(), _stream_handle(stream)))
        return spec, harm

    def get_state(self):
        t = ctypes.c_double(0)
        st = ctypes.c_int64(0)
        E = (ctypes.c_double * max(1, self.njet))()
        self._check(self.lib.hydro_get_state(self.ctx, ctypes.byref(t), ctypes.byref(st), E, self.njet))
        return t.value, st.value, np.array(list(E)[: self.njet])

    def set_state(self, step: int, E_jet, ledger: float):
        E = (ctypes.c_double * max(1, self.njet))(*[float(v) for v in E_jet])
        self._check(self.lib.hydro_set_state(self.ctx, int(step), E, self.njet, float(ledger)))

    def fixups(self) -> int:
        f = ctypes.c_int64(0)
        self._check(self.lib.hydro_diag(self.ctx, ctypes.byref(f)))
        return f.value

    def set_option(self, option: int, value: int):
        self._check(self.lib.hydro_set_option(self.ctx, int(option), int(value)))

    def get_option(self, option: int) -> int:
        v = ctypes.c_int(0)
        self._check(self.lib.hydro_get_option(self.ctx, int(option), ctypes.byref(v)))
        return v.value

    def profile(self, enable: bool = True):
        """Bracket every later launch of step() with HIP events on its stream."""
        self._check(self.lib.hydro_profile(self.ctx, 1 if enable else 0))

    def profile_read(self):
        """{kernel class: (total ms, launches)} since the last read."""
        nk = len(KERNELS)
        ms = (ctypes.c_double * nk)()
        n = (ctypes.c_int64 * nk)()
        self._check(self.lib.hydro_profile_read(self.ctx, ms, n, nk))
        return {KERNELS[k]: (ms[k], n[k]) for k in range(nk)}

    def close(self):
        """Destroys the context and releases its workspace (the library no
        longer uses it)."""
        if getattr(self, "ctx", None):
            import torch
            self.lib.hydro_destroy(self.ctx)
            self.ctx = None
            torch.cuda.synchronize(self.device)  # no launch of the context still reads it
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_workload(w, precision: str = "f64", weno: str = "z", bc=None, adjoint_k: int = 0, device="cuda",
                  limiter: str = "none", flux: str = "weno", musta_k: int = 2) -> Hydro:
    """Hydro for a paper_1511_02137_amd.workloads.Workload, with its jets."""
    cfg = make_config(w.n, w.dx, w.dt, w.t0, bc or w.bc, precision, weno, w.deposit, limiter=limiter, flux=flux,
                      musta_k=musta_k)
    h = Hydro(cfg, w.prim0, device=device, adjoint_k=adjoint_k)
    for j in w.jets:
        h.add_jet(j.x0, j.dir, j.E0, j.t_start, j.kappa_rad, j.kappa_coll, j.cr_over_cf)
    return h


class Batch:
    """Events advanced together by the batch API (include/hydro.h): cfgs a
    list of Config (shared precision and scheme), prims a list of FP64
    primitive arrays (numpy or torch, (5, nz, ny, nx)) or None.  U[e] are
    the events' conserved fields (torch, [5, nz, ny, nx])."""

    def __init__(self, cfgs, prims=None, device: str = "cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libhydro needs a GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        n = len(cfgs)
        self.n = n
        self.cfgs = (Config * n)(*cfgs)
        self.device = torch.device(device)
        self.dtype = torch.float32 if cfgs[0].precision == F32 else torch.float64
        self.shapes = [(c.n[2], c.n[1], c.n[0]) for c in cfgs]
        self.U = [torch.empty((5,) + sh, dtype=self.dtype, device=self.device) for sh in self.shapes]
        nbytes = int(self.lib.hydro_batch_workspace_bytes(self.cfgs, n))
        if nbytes == 0:
            raise HydroError(HYDRO_EINVAL, "invalid or incompatible batch configurations")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ws_ptr = self.ws.data_ptr() + (-self.ws.data_ptr()) % 256
        self._keep = []
        pp = None
        if prims is not None:
            ptrs = []
            for e, p in enumerate(prims):
                if p is None:
                    ptrs.append(None)
                    continue
                if isinstance(p, np.ndarray):
                    a = np.ascontiguousarray(p, dtype=np.float64)
                    ptr = a.ctypes.data
                else:
                    a = p.to(dtype=torch.float64).contiguous()
                    ptr = a.data_ptr()
                assert tuple(a.shape) == (5,) + self.shapes[e], (a.shape, self.shapes[e])
                self._keep.append(a)
                ptrs.append(ptr)
            pp = (ctypes.c_void_p * n)(*ptrs)
        Up = (ctypes.c_void_p * n)(*[u.data_ptr() for u in self.U])
        h = ctypes.c_void_p()
        rc = self.lib.hydro_batch_create(self.cfgs, n, pp, Up, ws_ptr, nbytes, _stream_handle(), ctypes.byref(h))
        if rc != HYDRO_OK:
            raise HydroError(rc, self.lib.hydro_batch_last_error(None).decode())
        self.b = h
        self.njet = [0] * n

    def _check(self, rc):
        if rc != HYDRO_OK:
            raise HydroError(rc, self.lib.hydro_batch_last_error(self.b).decode())

    def add_jet(self, event: int, x0, dir=(1.0, 0.0, 0.0), E0=50.0, t_start=1.0, kappa_rad=4.0, kappa_coll=2.5,
                cr_over_cf=1.0) -> int:
        j = Hydro._jet(x0, dir, E0, t_start, kappa_rad, kappa_coll, cr_over_cf)
        jid = ctypes.c_int(-1)
        self._check(self.lib.hydro_batch_add_jet(self.b, int(event), ctypes.byref(j), ctypes.byref(jid)))
        self.njet[event] += 1
        return jid.value

    def run(self, nsteps: int = 1, stream=None):
        self._check(self.lib.hydro_batch_run(self.b, int(nsteps), _stream_handle(stream)))

    def rhs(self, stream=None):
        self._check(self.lib.hydro_batch_rhs(self.b, _stream_handle(stream)))

    def autotune(self, cache_path: Optional[str] = None, stream=None) -> bool:
        """Pick the workgroup counts; True if they came from the cache."""
        fc = ctypes.c_int(0)
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.hydro_batch_autotune(self.b, path, _stream_handle(stream), ctypes.byref(fc)))
        return bool(fc.value)

    def set_option(self, option: int, value: int):
        self._check(self.lib.hydro_batch_set_option(self.b, int(option), int(value)))

    def get_option(self, option: int) -> int:
        v = ctypes.c_longlong(0)
        self._check(self.lib.hydro_batch_get_option(self.b, int(option), ctypes.byref(v)))
        return v.value

    def sums(self, event: int) -> np.ndarray:
        out = (ctypes.c_double * 6)()
        self._check(self.lib.hydro_batch_sums(self.b, int(event), out))
        return np.array(list(out))

    def get_state(self, event: int):
        t = ctypes.c_double(0)
        st = ctypes.c_int64(0)
        nj = self.njet[event]
        E = (ctypes.c_double * max(1, nj))()
        self._check(self.lib.hydro_batch_get_state(self.b, int(event), ctypes.byref(t), ctypes.byref(st), E, nj))
        return t.value, st.value, np.array(list(E)[:nj])

    def fixups(self) -> int:
        f = ctypes.c_int64(0)
        self._check(self.lib.hydro_batch_diag(self.b, ctypes.byref(f)))
        return f.value

    def close(self):
        if getattr(self, "b", None):
            self.lib.hydro_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_from_workloads(ws, precision: str = "f32", weno: str = "z", device="cuda", limiter: str = "none",
                         flux: str = "weno", musta_k: int = 2) -> Batch:
    """Batch of workloads.Workload events, with their jets."""
    cfgs = [make_config(w.n, w.dx, w.dt, w.t0, w.bc, precision, weno, w.deposit, limiter=limiter, flux=flux,
                        musta_k=musta_k) for w in ws]
    b = Batch(cfgs, [w.prim0 for w in ws], device=device)
    for e, w in enumerate(ws):
        for j in w.jets:
            b.add_jet(e, j.x0, j.dir, j.E0, j.t_start, j.kappa_rad, j.kappa_coll, j.cr_over_cf)
    return b
