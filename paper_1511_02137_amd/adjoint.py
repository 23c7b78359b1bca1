"""Differentiable runs: eps2 of the final state with a hand-written adjoint.

The observable is the energy-weighted anisotropy on the z = 0 plane,
eps2 = sum (y^2 - x^2) e / sum (y^2 + x^2) e, after `steps` SSP-RK3 steps
from an initial state whose energy density e_init is an input; the other
inputs are kappa_rad, kappa_coll of jet 0 (the energy-loss law, Eq. 3) and
its origin (x0, y0).

Forward: hydro_reset from the primitives, the steps (a checkpoint of U and of
the jet energies every `ckpt_every` steps; the last segment's stage states
are kept as it runs, hydro_rk3_step_record), hydro_loss_eps2.  Backward: the
loss seed, the reverse sweep over each segment from the last (the last one
from its kept stage states, hydro_adjoint_recorded, while the workspace still
holds them; the others, and the last one after anything replaced them, by
hydro_adjoint_step, which recomputes them from the segment's checkpoint:
bit for bit the same), then hydro_init_vjp for d/de_init.  Every step runs in libhydro's kernels; this module orders the
calls and keeps the checkpoints (torch tensors in HBM).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from . import hydro as H


@dataclass
class Checkpoint:
    U: object            # torch tensor like Hydro.U
    step: int
    E_jet: np.ndarray
    recorded: int = 0    # forward whose recorded stage states cover this segment (0: none)


@dataclass
class Recorded:
    """Stands for the stage states a forward left in the workspace."""
    generation: int


class Eps2Problem:
    """A workload (workloads.Workload) set up for differentiation: one
    context whose workspace holds the stage states of `ckpt_every` steps, the
    fixed primitives (v, n) on the device, and jet 0's direction, energy and
    start time (its kappas and origin are inputs of forward).

    record=True keeps the stage states of every step in HBM during the
    forward (hydro_rk3_step_record; 3 steps states of U's size) so that the
    backward runs the reverse sweep alone (hydro_adjoint_recorded, bit for bit
    the checkpointed result); a backward then belongs to the latest forward."""

    def __init__(self, workload, precision: str = "f64", ckpt_every: int = 10, device: str = "cuda",
                 record: bool = False):
        import torch
        self.w = workload
        self.steps = int(workload.steps)
        self.record = bool(record)
        self.k = self.steps if self.record else int(ckpt_every)
        self._generation = 0
        self._params = None   # the jet parameters the context holds
        self._live = 0        # forward whose recorded stage states the workspace still holds (0: none)
        self.h = H.from_workload(workload, precision=precision, adjoint_k=self.k, device=device)
        # eps2 depends on e and v only, so the adjoint of N is zero throughout
        self.h.set_option(H.OPT_ADJ_SKIP_N, 1)
        self.prim = torch.tensor(workload.prim0, dtype=torch.float64, device=device)
        self.jet = workload.jets[0]

    def set_params(self, kappa_rad: float, kappa_coll: float, x0: float, y0: float):
        j = self.jet
        self.h.set_jet(0, (x0, y0, j.x0[2]), j.dir, j.E0, j.t_start, kappa_rad, kappa_coll, j.cr_over_cf)
        self._params = (float(kappa_rad), float(kappa_coll), float(x0), float(y0))
        self._live = 0  # hydro_set_jet discards a record

    def forward(self, e_init, kappa_rad: float, kappa_coll: float, x0: float, y0: float):
        """Runs the steps; returns (eps2 device scalar, checkpoints, final U, primitives)."""
        prim = self.prim.clone()
        prim[0] = e_init.detach().to(prim)
        self.set_params(kappa_rad, kappa_coll, x0, y0)
        self.h.reset(prim)
        if self.record:
            self.h.step_record(self.steps)
            self._generation += 1
            return self.h.loss_eps2(), [Recorded(self._generation)], self.h.U.clone(), prim
        # the last segment's stage states are kept as it runs, so that the
        # backward sweeps it without a recompute while they are still there
        self._generation += 1
        self._live = 0
        cks: List[Checkpoint] = []
        s = 0
        while s < self.steps:
            _, step, Ej = self.h.get_state()
            cks.append(Checkpoint(self.h.U.clone(), step, Ej))
            n = min(self.k, self.steps - s)
            if s + n == self.steps:
                self.h.step_record(n)
                cks[-1].recorded = self._generation
                self._live = self._generation
            else:
                self.h.step(n)
            s += n
        eps = self.h.loss_eps2()
        return eps, cks, self.h.U.clone(), prim

    def backward(self, cks: List[Checkpoint], U_final, prim, scale: float = 1.0, params=None):
        """scale * (d eps2/d e_init [device (nz, ny, nx)], d eps2/d jet params
        [device (njet, 5): kappa_rad, kappa_coll, x0, y0, z0]).  The reverse
        sweep recomputes the stage states with the context's current jet;
        params = (kappa_rad, kappa_coll, x0, y0) of the forward being
        differentiated re-applies them first (needed whenever another forward
        ran in between)."""
        import torch
        if self.record:
            if len(cks) != 1 or not isinstance(cks[0], Recorded) or cks[0].generation != self._generation:
                raise RuntimeError("another forward replaced the recorded stage states of this one "
                                   "(record=False keeps checkpoints and allows interleaved forwards)")
        elif params is not None and tuple(float(v) for v in params) != self._params:
            self.set_params(*params)
        lam = torch.empty_like(U_final)
        self.h.loss_eps2(U_final, seed=lam, scale=scale)
        grad = torch.zeros((max(1, self.h.njet), 5), dtype=torch.float64, device=U_final.device)
        if self.record:
            self.h.adjoint_recorded(lam, grad)
        else:
            ends = [c.step for c in cks[1:]] + [self.steps]
            for ck, end in reversed(list(zip(cks, ends))):
                if ck.recorded and ck.recorded == self._live:
                    self.h.adjoint_recorded(lam, grad)
                else:
                    self.h.adjoint_step(ck.U, ck.step, ck.E_jet, end - ck.step, lam, grad)
                    self._live = 0  # the recompute overwrote the record
        gprim = self.h.init_vjp(prim, lam)
        return gprim[0], grad


_FUNCTION = None


def _function():
    global _FUNCTION
    if _FUNCTION is not None:
        return _FUNCTION
    import torch

    class HydroEps2(torch.autograd.Function):
        """eps2(e_init, kappa_rad, kappa_coll, jet_xy; problem)."""

        @staticmethod
        def forward(ctx, e_init, kappa_rad, kappa_coll, jet_xy, problem):
            params = (float(kappa_rad), float(kappa_coll), float(jet_xy[0]), float(jet_xy[1]))
            eps, cks, U_final, prim = problem.forward(e_init, *params)
            ctx.problem, ctx.cks, ctx.U_final, ctx.prim = problem, cks, U_final, prim
            # the problem's context is shared: another forward may set other
            # jet parameters before this backward runs
            ctx.params = params
            ctx.dtypes = (e_init.dtype, kappa_rad.dtype, kappa_coll.dtype, jet_xy.dtype)
            ctx.devices = (e_init.device, kappa_rad.device, kappa_coll.device, jet_xy.device)
            return eps

        @staticmethod
        def backward(ctx, g):
            gde, grad = ctx.problem.backward(ctx.cks, ctx.U_final, ctx.prim, scale=float(g), params=ctx.params)
            dt, dv = ctx.dtypes, ctx.devices
            return (gde.to(device=dv[0], dtype=dt[0]), grad[0, 0].to(device=dv[1], dtype=dt[1]),
                    grad[0, 1].to(device=dv[2], dtype=dt[2]), grad[0, 2:4].to(device=dv[3], dtype=dt[3]), None)

    _FUNCTION = HydroEps2
    return _FUNCTION


def eps2(e_init, kappa_rad, kappa_coll, jet_xy, problem: Eps2Problem):
    """Differentiable eps2.  e_init: (nz, ny, nx) tensor; kappa_rad,
    kappa_coll: 0-d tensors; jet_xy: (2,) tensor (x0, y0 of jet 0)."""
    return _function().apply(e_init, kappa_rad, kappa_coll, jet_xy, problem)
