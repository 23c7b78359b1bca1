#!/usr/bin/env python3
"""Throughput of the jet + ideal-hydro SSP-RK3 step on one MI355X.

A step is one full SSP-RK3 step (three stages of WENO7 x/y/z faces, jet
source, RK combine) plus the FP64 conservation sums, over the paper's shape:
256^3 cells, dx = 0.1 fm, dt = 0.02 fm/c, p = e/3, one jet (synthetic,
seeded inputs; see paper_1511_02137_amd/workloads.py).  The inputs are
resident in HBM before the timed region starts.

Prints one JSON line: whole-job cell-updates/s (cells x stages / s), the
roofline of the dominant kernel from HIP events recorded around every
launch on the launch stream over the timed region, the adjoint/forward time
ratio of the differentiable run (128^3, 100 steps, checkpoints every 10,
FP32 fields) with the error of its initial-field gradient against the FP64
form, the freeze-out pass (spectra and flow harmonics of the evolved
state), the throughput of the 64-event uneven ensemble through the batch
API, and the CPU oracle timed on a bounded slab of the stage workload.

    python bench.py [--steps K] [--warmup W] [--precision f64|f32] [--n 256]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per RK3 stage at 256^3 (% of roofline); adjoint/forward time"

# Algorithmic flops per cell and kernel (adds and multiplies 1, fma 2,
# divide and square root 1), minimal form of the scheme:
#   one WENO7-Z reconstruction: candidates 28, smoothness 92, tau 4,
#   weights 20, sum 3, combination 7, normalisation 1 = 155;
#   per face 10 reconstructions (5 fields x 2 splits) = 1550;
#   flux and Lax-Friedrichs split per cell and axis 25;
#   divergence 10 per axis; conserved->primitive 25 (counted once, x);
#   RK combine 15 (z).
# Flops per reconstruction for the other schemes, same accounting: WENO7-JS
# drops tau (151); linear weights: candidates + combination (35 for WENO7, 20
# for WENO5).  For WENO5-Z/JS the plain formulation (counted operation by
# operation by the oracle's counting scalar: 78 and 71) needs fewer than the
# library's form (85, 83), so the smaller count is used: the algorithmic count
# is never taken above what a plain implementation needs (the test of the
# counts checks this for every scheme).
RECON_FLOPS = {"z": 155, "js": 151, "linear": 35, "z5": 78, "js5": 71, "linear5": 20}


SCHEME_NAMES = {"z": "WENO7-Z", "js": "WENO7-JS", "linear": "WENO7 linear weights", "z5": "WENO5-Z",
                "js5": "WENO5-JS", "linear5": "WENO5 linear weights"}


# MUSTA-FORCE per face and stage: three recoveries with their fluxes (3 x 31),
# the Richtmyer state (20) and the FORCE flux (30); the local update between
# stages (30).
MUSTA_STAGE_FLOPS, MUSTA_UPDATE_FLOPS = 3 * 31 + 20 + 30, 30


def flops_per_cell(weno: str = "z", flux: str = "weno", musta_k: int = 2):
    r = 10 * RECON_FLOPS[weno]
    if flux == "musta":  # reconstructions of the two states, stages, divergence (+ combine in z)
        f = r + MUSTA_STAGE_FLOPS * musta_k + MUSTA_UPDATE_FLOPS * (musta_k - 1) + 10
        return {"xface": f, "ymarch": f, "zmarch": f + 15}
    return {"xface": r + 25 + 10 + 25, "ymarch": r + 25 + 10, "zmarch": r + 25 + 10 + 15}


FLOPS_PER_CELL = flops_per_cell("z")
FLOPS_PER_CELL_UPDATE = sum(FLOPS_PER_CELL.values())  # 4795
# Algorithmic words moved per cell by each kernel (W read + D read/write;
# z: + U^n read in stages 2-3 (2/3 on average) + output write).
BYTES_PER_CELL = {"xface": 10, "ymarch": 15, "zmarch": 5 + 5 + 5 * 2 / 3 + 5}
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}  # MI355X vector FP64 / FP32 (packed)

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (KiB per
# dispatch, scaled by a 1 GiB plain copy: read x2.0, write x1.0), for the
# kernel sources with the given hash (KERNEL_SOURCES); reported as null once
# any of them changes.  Source: profiles/stage_256cube_f64.md.
MEASURED_TRAFFIC = {
    ("zmarch", "f64", "tile", 256, 2): {"kernels_sha256": "e5d3f7c1bedb188c",
                                        "read_bytes": 956126 * 2.0 * 1024, "write_bytes": 655360 * 1.0 * 1024},
}
# The whole stage from the same counters, in fields (one field = one full
# read or write of one of the five state fields) per cell and stage: x faces
# 5 + 5, outflow x faces 0.63 + 0.08, y tiles 10 + 5, z tiles 14.59 + 5, the
# per-step sums 5 / 3; the minimal stage moves 13.33 (10 / 15 / 15).
MEASURED_STAGE_FIELDS = {("f64", "tile", 256, 2): {"kernels_sha256": "e5d3f7c1bedb188c",
                                                   "fields": 10.0 + 0.71 + 15.0 + 19.59 + 5.0 / 3}}
KERNEL_SOURCES = ("hydro_kernels.hip", "hydro_device.hpp", "hydro_internal.hpp")


def kernels_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1511_02137_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cpu_baseline(w, target_s: float):
    """The oracle, one RK3 step on a centred z-slab of the same workload."""
    import numpy as np
    import oracle as O
    nz = w.n[2]

    def run_slab(planes):
        z0 = (nz - planes) // 2
        prim = np.ascontiguousarray(w.prim0[:, z0:z0 + planes])
        pb = O.Problem(n=(w.n[0], w.n[1], planes), dx=w.dx, t0=w.t0, dt=w.dt, bc=w.bc)
        U = O.prim_to_cons(pb, prim)
        jets = [O.Jet(**j.__dict__) for j in w.jets]
        t = time.perf_counter()
        O.run(pb, U, 1, jets)
        return time.perf_counter() - t

    cores = O.threads()
    planes = min(nz, 8)
    t = run_slab(planes)
    if t < 0.5 * target_s and planes < nz:
        planes = min(nz, max(planes + 1, int(planes * target_s / max(t, 1e-3))))
        t = run_slab(planes)
    cells = w.n[0] * w.n[1] * planes
    # the same on one core, on a thinner slab (about a tenth of the time budget)
    O.set_threads(1)
    p1 = max(1, min(planes, int(planes * 0.1 * target_s / max(t * cores, 1e-3))))
    t1 = run_slab(p1)
    O.set_threads(cores)
    # the whole 32^3 x 10-step small event on all cores
    from paper_1511_02137_amd import workloads as W
    ws = W.small_event(1)
    pbs = O.Problem(n=ws.n, dx=ws.dx, t0=ws.t0, dt=ws.dt, bc=ws.bc)
    Us = O.prim_to_cons(pbs, ws.prim0)
    ts = time.perf_counter()
    O.run(pbs, Us, ws.steps, [O.Jet(**j.__dict__) for j in ws.jets])
    ts = time.perf_counter() - ts
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": cells * 3 / t,
        "unit": "cell-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "one RK3 step (3 stages) of the central %dx%dx%d z-slab of the %s workload, outflow, "
                  "%.1f s wall" % (w.n[0], w.n[1], planes, w.name, t),
        "single_core_value": w.n[0] * w.n[1] * p1 * 3 / t1,
        "single_core_sample": "the central %dx%dx%d z-slab, one step, %.1f s wall" % (w.n[0], w.n[1], p1, t1),
        "small_event_run_s": ts,
        "small_event_run": "%s, %d steps, all cores" % (ws.name, ws.steps),
        "host_cpu": model, "host_logical_cpus": os.cpu_count(),
    }


def precision_check(n: int, steps: int):
    """FP32 form against the FP64 form of the same run (paper shape, one jet):
    relative L2 of e and |v| after `steps` steps (primitives in FP64)."""
    import torch
    from paper_1511_02137_amd import hydro as H
    from paper_1511_02137_amd import workloads as W
    w = W.paper_event(2, n=(n,) * 3)
    prims = {}
    for prec in ("f64", "f32"):
        h = H.from_workload(w, precision=prec)
        h.step(steps)
        p = h.primitives().double()
        prims[prec] = (p[0], torch.sqrt(p[1] ** 2 + p[2] ** 2 + p[3] ** 2))
        h.close()
        del h
    out = {"workload": "%s, %d steps, FP32 form against FP64" % (w.name, steps)}
    for k, name in ((0, "e"), (1, "abs_v")):
        a, b = prims["f32"][k], prims["f64"][k]
        out["rel_l2_" + name] = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    return out


# Algorithmic flops of one reconstruction's adjoint (WENO7-Z; add and
# multiply 1, fma 2): the forward recomputed (155, as in FLOPS_PER_CELL) and
# the reverse sweep (122: the partials of the normalised sum in the weights
# and candidates 6, through the Z weights to tau and the indicators 34, the
# indicators to the nested differences 34, the candidates to the first
# differences 24, the transposed differences to the seven points 24).
ADJ_FLOPS_RECON = 155 + 122


def adjoint_ratio(precision: str, n: int, steps: int, ckpt: int, repeats: int = 3):
    """Differentiable run (workloads.gradient_event): forward = reset, the
    steps with a checkpoint every `ckpt` steps (the last segment's stage
    states kept as it runs), eps2; backward = loss seed, reverse sweep over
    every segment (recomputing the stage states of all but the last),
    initial state VJP.  Best of `repeats` after one untimed pass,
    GPU-synchronised."""
    import torch
    from paper_1511_02137_amd import adjoint as A
    from paper_1511_02137_amd import workloads as W
    w = W.gradient_event(n=(n,) * 3, steps=steps)
    pb = A.Eps2Problem(w, precision=precision, ckpt_every=ckpt)
    j = w.jets[0]
    e0 = torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda")
    tf, tb = [], []
    for r in range(repeats + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eps, cks, Uf, prim = pb.forward(e0, j.kappa_rad, j.kappa_coll, j.x0[0], j.x0[1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ge, gj = pb.backward(cks, Uf, prim)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r:
            tf.append(t1 - t0)
            tb.append(t2 - t1)
    eps, cks, Uf, prim = pb.forward(e0, j.kappa_rad, j.kappa_coll, j.x0[0], j.x0[1])
    pb.h.profile(True)
    pb.backward(cks, Uf, prim)
    torch.cuda.synchronize()
    prof = pb.h.profile_read()
    pb.h.profile(False)
    g = gj[0].tolist()
    ge_run = ge.double()
    pb.h.close()
    # error of the initial-field gradient: against the FP64 form (everywhere,
    # and at least 16 cells inside the outflow faces, where it is well
    # conditioned), and along a smooth bump on the jet's path
    p64 = A.Eps2Problem(w, precision="f64", ckpt_every=ckpt)
    eps64, cks64, Uf64, prim64 = p64.forward(e0, j.kappa_rad, j.kappa_coll, j.x0[0], j.x0[1])
    ge64, gj64 = p64.backward(cks64, Uf64, prim64)
    p64.h.close()
    nz, ny, nx = ge64.shape
    iz, iy, ix = torch.meshgrid(torch.arange(nz, device="cuda"), torch.arange(ny, device="cuda"),
                                torch.arange(nx, device="cuda"), indexing="ij")
    dist = torch.minimum(torch.minimum(torch.minimum(ix, nx - 1 - ix), torch.minimum(iy, ny - 1 - iy)),
                         torch.minimum(iz, nz - 1 - iz))
    inner = dist >= 16
    cz = [(torch.arange(m, device="cuda", dtype=torch.float64) - 0.5 * (m - 1)) * 0.1 for m in (nz, ny, nx)]
    zz, yy, xx = torch.meshgrid(*cz, indexing="ij")
    blob = torch.exp(-((xx + 1.0) ** 2 + yy ** 2 + zz ** 2) / (2 * 0.5 ** 2))
    rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    d32, d64 = float((ge_run * blob).sum()), float((ge64 * blob).sum())
    einit = {"rel_l2_vs_f64": rel(ge_run, ge64),
             "rel_l2_vs_f64_inner": rel(ge_run[inner], ge64[inner]),
             "inner": ">= 16 cells from every outflow face (well conditioned; the gradient next to the faces "
                      "moves by ~7e-6 in FP64 under a 1e-14 change of e_init)",
             "blob_direction_rel_vs_f64": abs(d32 - d64) / abs(d64),
             "blob_direction": "exp(-|x - (-1, 0, 0)|^2 / (2 * 0.5^2)), x in fm",
             "f64_blob_derivative": d64}
    # the same run with every step's stage states kept in HBM during the
    # forward (hydro_rk3_step_record), so that the backward is the reverse
    # sweep alone (hydro_adjoint_recorded); its gradients are those above bit
    # for bit
    pr = A.Eps2Problem(w, precision=precision, record=True)
    rf, rb = [], []
    for r in range(repeats + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eps_r, rec, Uf_r, prim_r = pr.forward(e0, j.kappa_rad, j.kappa_coll, j.x0[0], j.x0[1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ge_r, gj_r = pr.backward(rec, Uf_r, prim_r)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r:
            rf.append(t1 - t0)
            rb.append(t2 - t1)
    recorded = {"forward_ms": 1e3 * min(rf), "backward_ms": 1e3 * min(rb), "ratio": min(rb) / min(rf),
                "stage_states_gb": 3 * steps * 5 * float(n) ** 3 * (4 if precision == "f32" else 8) / 1e9,
                "gradients_bitwise_equal": bool(torch.equal(ge_r, ge) and torch.equal(gj_r, gj))}
    pr.h.close()
    # the line adjoints' arithmetic rate: reverse-WENO flops of a launch
    # (ADJ_FLOPS_RECON per reconstruction, 4 fields (N's adjoint is zero for
    # eps2 and skipped) x 2 splits per cell) over the mean time of the line and
    # boundary-face adjoint launches of one axis (HIP events)
    t_adj, n_adj = prof.get("adjoint", (0.0, 0))
    flops_launch = float(n) ** 3 * 4 * 2 * ADJ_FLOPS_RECON
    adj_tf = flops_launch / (t_adj / n_adj * 1e-3) / 1e12 if n_adj else 0.0
    peak = PEAK_TFLOPS[precision]
    out = {"workload": "%s: %d^3, %d steps, checkpoint every %d, %s fields, FP64 parameter gradients"
                       % (w.name, n, steps, ckpt, precision),
           "forward_ms": 1e3 * min(tf), "backward_ms": 1e3 * min(tb), "ratio": min(tb) / min(tf),
           "backward_kernels_ms": {k: t for k, (t, c) in prof.items() if c},
           "line_adjoint_roofline": {"bound": "alu", "kernel": "line adjoints (one launch per axis and stage)",
                                     "flops_per_cell": 4 * 2 * ADJ_FLOPS_RECON,
                                     "ms_per_launch": t_adj / n_adj if n_adj else None,
                                     "achieved": adj_tf, "peak": peak, "unit": "TFLOP/s", "frac": adj_tf / peak},
           "eps2": float(eps.item()),
           "grad": {"kappa_rad": g[0], "kappa_coll": g[1], "x0": g[2], "y0": g[3]},
           "e_init_grad": einit,
           "recorded_stage_states": recorded}
    return out


# Algorithmic flops of the freeze-out pass (adds and multiplies 1, fma 2,
# divide, square root, exp and pow 1): per cell the recovery (25), T(e) (4),
# gamma and the weights (8); per cell and azimuth D = 1 - vx cos - vy sin (4)
# and the p_T-integrated term w/(gamma D)^3 added in (cube 2, divide 1, fma 2);
# per cell, azimuth and p_T the exponent (2), exp (1), the fma (2).
FO_FLOPS_CELL, FO_FLOPS_PHI, FO_FLOPS_PT = 37, 9, 5


def freezeout_timing(precision: str, n: int, steps: int, n_phi: int, pts, repeats: int = 5):
    """hydro_freezeout on the paper event after `steps` steps: mean time of
    the spectra + harmonics launches (HIP events on the launch stream) and
    the ALU fraction of the algorithmic flops; v_2 and v_3 of the
    p_T-integrated row."""
    import torch
    from paper_1511_02137_amd import hydro as H
    from paper_1511_02137_amd import workloads as W
    w = W.paper_event(2, n=(n,) * 3)
    h = H.from_workload(w, precision=precision)
    h.step(steps)
    h.freezeout(n_phi=n_phi, pt=pts, n_harm=8)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(repeats):
        spec, harm = h.freezeout(n_phi=n_phi, pt=pts, n_harm=8)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / repeats
    nc = n ** 3
    flops = nc * (FO_FLOPS_CELL + n_phi * (FO_FLOPS_PHI + FO_FLOPS_PT * len(pts)))
    hm = harm.cpu().numpy()
    out = {"workload": "%s after %d steps, %s fields: Cooper-Frye on the fixed-time surface, massless Boltzmann "
                       "particles at y = 0, %d azimuths, p_T-integrated + %d p_T values"
                       % (w.name, steps, precision, n_phi, len(pts)),
           "ms": ms, "achieved_tflops": flops / (ms * 1e-3) / 1e12, "peak": PEAK_TFLOPS["f64"],
           "alu_frac": flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["f64"],
           "dNdy": float(hm[0, 0, 0]),
           "v2": float(np.hypot(*hm[0, 2])), "v3": float(np.hypot(*hm[0, 3]))}
    h.close()
    return out


def batch_throughput(precision: str, steps: int, warmup: int, cache, limiter: str = "pp"):
    """The uneven ensemble (workloads.ensemble: 64 events, edges 64/96/128,
    0-3 jets) advanced by the batch API: autotuned launch shapes, one graph
    replay per step; cell-updates/s over `steps` steps.  The positivity-
    preserving limiter is on by default: without it the NGP deposits drive
    stage states of 32 of the events out of the admissible set (recovery
    fix-ups) within the 50 steps."""
    import torch
    from paper_1511_02137_amd import hydro as H
    from paper_1511_02137_amd import workloads as W
    ws = W.ensemble(steps=steps)
    b = H.batch_from_workloads(ws, precision=precision, limiter=limiter)
    from_cache = b.autotune(cache)
    b.run(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    b.run(steps)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    cells = sum(w.n[0] * w.n[1] * w.n[2] for w in ws)
    value = cells * 3 * steps / (ms * 1e-3)
    out = {"workload": "ensemble of %d events, edges {64, 96, 128} per axis, 0-3 jets, %s fields, %d steps, "
                       "one graph replay per step%s" % (len(ws), precision, steps,
                                                        ", positivity limiter" if limiter == "pp" else ""),
           "cells": cells, "ms_per_step": ms / steps, "value": value,
           "unit": "cell-updates/s", "limiter": limiter,
           "alu_frac": FLOPS_PER_CELL_UPDATE * value / 1e12 / PEAK_TFLOPS[precision],
           "blocks_per_axis": [b.get_option(a) for a in (0, 1, 2)],
           "x_form": "rows" if b.get_option(H.BOPT_X_ROWS) else "tiles",
           "tuned_from_cache": from_cache, "fixups": b.fixups()}
    b.close()
    return out


def log_run(h, steps: int, path: str) -> int:
    """Steps h one at a time and appends one JSON line per step to path: the
    step's FP64 sums (hydro_step_sums), ledger, jet energies, fix-up count and
    per-kernel-class times (HIP events); each step sits in a roctx range
    ("hydro step <n>") for rocprofv3's marker trace.  Untimed diagnostics, not
    a benchmark.  Returns the number of lines written."""
    import torch
    h.profile(True)
    with open(path, "a") as f:
        for _ in range(steps):
            n = h.get_state()[1]
            torch.cuda.nvtx.range_push("hydro step %d" % n)
            h.step(1)
            torch.cuda.nvtx.range_pop()
            ss = h.step_sums()
            t, step, Ej = h.get_state()
            prof = h.profile_read()
            f.write(json.dumps({"step": step, "t": t, "sums": [float(v) for v in ss[:5]], "ledger": float(ss[5]),
                                "E_jet": [float(v) for v in Ej], "fixups": h.fixups(),
                                "kernels_ms": {k: ms for k, (ms, c) in prof.items() if c}}) + "\n")
    h.profile(False)
    return steps


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--yz", choices=["tile", "march"], default="tile", help="y/z face kernels")
    ap.add_argument("--x", choices=["row", "tile"], default="row", help="x face kernel")
    ap.add_argument("--tile-order", type=int, default=2, choices=[0, 1, 2, 3],
                    help="workgroup order of the y/z LDS tiles (HYDRO_OPT_TILE_ORDER)")
    ap.add_argument("--limiter", choices=["none", "pp"], default="none",
                    help="face-flux limiter of the stage run (pp: positivity-preserving)")
    ap.add_argument("--flux", choices=["weno", "musta"], default="weno",
                    help="face fluxes of the stage run: WENO of the LF split fluxes, or MUSTA-FORCE")
    ap.add_argument("--musta-k", type=int, default=2, help="MUSTA-FORCE stages")
    ap.add_argument("--weno", choices=sorted(RECON_FLOPS), default="z",
                    help="reconstruction: WENO7 (z, js, linear) or WENO5 (z5, js5, linear5)")
    ap.add_argument("--adjoint-n", type=int, default=128, help="grid edge of the differentiable run (0: skip)")
    ap.add_argument("--adjoint-steps", type=int, default=100)
    ap.add_argument("--adjoint-ckpt", type=int, default=10)
    ap.add_argument("--adjoint-precision", choices=["f64", "f32"], default="f32")
    ap.add_argument("--batch-steps", type=int, default=50, help="steps of the ensemble run (0: skip)")
    ap.add_argument("--precision-steps", type=int, default=10,
                    help="steps of the FP32-against-FP64 check at the stage shape (0: skip)")
    ap.add_argument("--freezeout-steps", type=int, default=10,
                    help="steps of the paper event before the timed freeze-out (0: skip)")
    ap.add_argument("--batch-precision", choices=["f64", "f32"], default="f32")
    ap.add_argument("--batch-limiter", choices=["none", "pp"], default="pp",
                    help="face-flux limiter of the ensemble run")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file of the ensemble run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB 10 times (scale for the HBM counters)")
    ap.add_argument("--log", default=None,
                    help="only run --steps steps of the stage workload one at a time, appending one JSON line "
                         "per step (sums, ledger, jet energies, fix-ups, kernel times) to this file")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the stage update is built and measured on a single MI355X "
              "(multi-GPU domain decomposition is designed, not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1511_02137_amd import hydro as H
    from paper_1511_02137_amd import workloads as W

    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": a.numel() * 8, "calibrate_copy_bytes_written": b.numel() * 8,
                          "launches": 10}))
        return

    w = W.paper_event(2, n=(args.n,) * 3)
    h = H.from_workload(w, precision=args.precision, weno=args.weno, limiter=args.limiter, flux=args.flux,
                        musta_k=args.musta_k)
    fpc = flops_per_cell(args.weno, args.flux, args.musta_k)  # the limiter's own arithmetic is not counted
    fpc_update = sum(fpc.values())
    h.set_option(H.OPT_YZ_KERNEL, 0 if args.yz == "tile" else 1)
    h.set_option(H.OPT_X_KERNEL, 0 if args.x == "row" else 1)
    h.set_option(H.OPT_TILE_ORDER, args.tile_order)
    nc = w.n[0] * w.n[1] * w.n[2]
    if args.log:
        log_run(h, args.steps, args.log)
        h.close()
        print("logged %d steps of %s to %s" % (args.steps, w.name, args.log), file=sys.stderr)
        return

    h.step(args.warmup)
    torch.cuda.synchronize()

    h.profile(True)
    start = torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    start.record()
    for i in range(args.steps):
        h.step(1)
        marks[i].record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(marks[-1])
    per_step = sorted([start.elapsed_time(marks[0])] +
                      [marks[i - 1].elapsed_time(marks[i]) for i in range(1, args.steps)])
    median_ms = per_step[len(per_step) // 2]
    prof = h.profile_read()
    h.profile(False)
    fix = h.fixups()

    value = nc * 3 * args.steps / (ms * 1e-3)
    per_kernel = {k: {"ms_per_launch": (t / n if n else 0.0), "launches": n} for k, (t, n) in prof.items()}
    dom = max(fpc, key=lambda k: prof[k][0])
    t_launch = prof[dom][0] / prof[dom][1]
    achieved = fpc[dom] * nc / (t_launch * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    traffic = None
    rec = (MEASURED_TRAFFIC.get((dom, args.precision, args.yz, args.n, args.tile_order))
           if args.weno == "z" and args.limiter == "none" and args.flux == "weno" else None)
    if rec is not None and kernels_sha256() == rec["kernels_sha256"]:
        traffic = rec["read_bytes"] + rec["write_bytes"]
    srec = (MEASURED_STAGE_FIELDS.get((args.precision, args.yz, args.n, args.tile_order))
            if args.weno == "z" and args.limiter == "none" and args.flux == "weno" else None)
    stage_traffic = None
    if srec is not None and kernels_sha256() == srec["kernels_sha256"]:
        stage_traffic = {"fields_per_cell_stage": srec["fields"], "algorithmic_fields": 40.0 / 3,
                         "ratio": srec["fields"] / (40.0 / 3),
                         "bytes_per_stage": srec["fields"] * nc * (8 if args.precision == "f64" else 4)}
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic,
                "algorithmic_bytes": BYTES_PER_CELL[dom] * (8 if args.precision == "f64" else 4) * nc,
                "flops_per_cell": fpc[dom]}
    step_frac = fpc_update * value / 1e12 / peak

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "median_ms_per_step": median_ms,
        "value_without_sums": nc * 3 * args.steps / ((ms - prof["sums"][0]) * 1e-3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "%s: %d^3 cells, dx 0.1 fm, dt 0.02 fm/c, p = e/3, %s + LF split%s, "
                               "SSP-RK3, 1 jet (NGP), outflow" % (
                                   w.name, args.n, SCHEME_NAMES[args.weno],
                                   (" + positivity limiter" if args.limiter == "pp" else "") +
                                   (" (MUSTA-FORCE fluxes, %d stages, of the WENO states)" % args.musta_k
                                    if args.flux == "musta" else "")),
                   "grid": list(w.n), "precision": args.precision, "jets": len(w.jets), "yz_kernel": args.yz,
                   "x_kernel": args.x, "tile_order": args.tile_order, "weno": args.weno, "limiter": args.limiter, "flux": args.flux,
                   "musta_k": args.musta_k if args.flux == "musta" else None},
        "roofline": roofline,
        "step_alu_frac": step_frac,
        "stage_traffic": stage_traffic,
        "flops_per_cell_update": fpc_update,
        "kernels": per_kernel,
        "fixups": fix,
    }
    print("timed %d steps: %.3f ms/step, %.3e cell-updates/s" % (args.steps, ms / args.steps, value),
          file=sys.stderr, flush=True)
    h.close()
    if args.precision_steps > 0:
        out["precision_check"] = precision_check(args.n, args.precision_steps)
    if args.adjoint_n > 0:
        out["adjoint"] = adjoint_ratio(args.adjoint_precision, args.adjoint_n, args.adjoint_steps, args.adjoint_ckpt)
        print("adjoint/forward %.2f (stage states kept in HBM: %.2f)"
              % (out["adjoint"]["ratio"], out["adjoint"]["recorded_stage_states"]["ratio"]), file=sys.stderr, flush=True)
    if args.freezeout_steps > 0:
        out["freezeout"] = freezeout_timing(args.precision, args.n, args.freezeout_steps, 64,
                                            [0.5, 1.0, 1.5, 2.0, 3.0])
        print("freeze-out %.3f ms" % out["freezeout"]["ms"], file=sys.stderr, flush=True)
    if args.batch_steps > 0:
        out["batch"] = batch_throughput(args.batch_precision, args.batch_steps, 2, args.tune_cache,
                                        args.batch_limiter)
        print("batch %.3e cell-updates/s" % out["batch"]["value"], file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
