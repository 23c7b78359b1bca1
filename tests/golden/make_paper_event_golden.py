"""Writes tests/golden/paper_event_256.json from the oracle alone: the 256^3
FP64 run shaped like the paper's (Fig. 3 caption: dx = 0.1 fm, dt = 0.02 fm/c,
p = e/3; t = 1 -> 3.4 fm/c, 120 SSP-RK3 steps; workloads.paper_event, seed 2).

At steps 1, 10, 40 and 120 it stores the FP64 sums of U dV, the ledger, the
jet energy, the fix-up count and all five conserved fields at a fixed set of
sampled cells (uniform over the grid, along the jet's path, and next to the
outflow faces).  It also runs the same event from initial energy densities
changed by a relative 1e-15 (seeded, uniform in [-1, 1]) and stores, per
checkpoint, how far that moves the fields (relative to max |E| for E and M,
max N for N; over the whole grid and over the sampled cells): the scale below
which two correct implementations that round differently cannot be told
apart after that many steps.

    python tests/golden/make_paper_event_golden.py    # ~1 h on 8 cores
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1511_02137_amd import workloads as W  # noqa: E402

CHECKPOINTS = (1, 10, 40, 120)


def sample_cells(w, seed=20260):
    """(z, y, x) indices: 160 uniform, 64 along the jet path, 96 within four
    cells of an outflow face."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = w.n
    cells = set()
    while len(cells) < 160:
        cells.add((int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))))
    j = w.jets[0]
    for k in range(64):
        t = w.t0 + (w.steps * w.dt) * k / 63.0
        p = [j.x0[d] + j.dir[d] * (t - j.t_start) for d in range(3)]
        idx = [int(np.clip(np.floor(p[d] / w.dx[d] + w.n[d] / 2.0), 0, w.n[d] - 1)) for d in range(3)]
        off = rng.integers(-2, 3, size=3)
        cells.add(tuple(int(np.clip(idx[2 - a] + off[a], 0, (nz, ny, nx)[a] - 1)) for a in range(3)))
    nb = 0
    while nb < 96:
        c = [int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))]
        a = int(rng.integers(3))
        size = (nz, ny, nx)[a]
        c[a] = int(rng.integers(4)) if rng.random() < 0.5 else size - 1 - int(rng.integers(4))
        if tuple(c) not in cells:
            cells.add(tuple(c))
            nb += 1
    return sorted(cells)


def rel_change(A, B, cells=None):
    """Per field max |A - B|, E and M over max |B_E|, N over max |B_N|."""
    scale = [np.abs(B[0]).max()] * 4 + [np.abs(B[4]).max()]
    if cells is not None:
        z, y, x = (np.array(v) for v in zip(*cells))
        A = A[:, z, y, x]
        B = B[:, z, y, x]
    return [float(np.abs(A[f] - B[f]).max() / scale[f]) for f in range(5)]


def main():
    w = W.paper_event(2)
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, bc=tuple(w.bc), deposit=w.deposit)
    jets = [O.Jet(**j.__dict__) for j in w.jets]
    cells = sample_cells(w)
    z, y, x = (np.array(v) for v in zip(*cells))
    rng = np.random.default_rng(7)
    prim_p = w.prim0.copy()
    prim_p[0] *= 1.0 + 1e-15 * rng.uniform(-1.0, 1.0, size=prim_p[0].shape)
    st = O.RunState(U=O.prim_to_cons(pb, w.prim0), Ejet=np.array([j.E0 for j in jets]))
    sp = O.RunState(U=O.prim_to_cons(pb, prim_p), Ejet=np.array([j.E0 for j in jets]))
    out = {"workload": w.name, "seed": 2, "steps": w.steps, "n": list(w.n), "dx": list(w.dx), "dt": w.dt,
           "t0": w.t0, "jet0": {k: (list(v) if isinstance(v, tuple) else v) for k, v in w.jets[0].__dict__.items()},
           "method": "oracle FP64 run (oracle/hydro_oracle.cpp)", "perturbation": "e_init * (1 + 1e-15 u), u ~ U(-1, 1), "
           "numpy default_rng(7)", "cells_zyx": [list(c) for c in cells], "checkpoints": []}
    done = 0
    t_all = time.time()
    for k in CHECKPOINTS:
        t = time.time()
        st = O.run(pb, st.U, k - done, jets, step0=done, Ejet=st.Ejet, ledger=st.ledger)
        st_fix = st.fixups
        sp = O.run(pb, sp.U, k - done, jets, step0=done, Ejet=sp.Ejet, ledger=sp.ledger)
        done = k
        ck = {"step": k, "sums": [float(v) for v in O.sums(pb, st.U)], "ledger": st.ledger,
              "E_jet": [float(v) for v in st.Ejet], "fixups": int(st_fix),
              "max_abs_E": float(np.abs(st.U[0]).max()), "max_abs_N": float(np.abs(st.U[4]).max()),
              "values": st.U[:, z, y, x].T.tolist(),
              "response_grid": rel_change(sp.U, st.U), "response_cells": rel_change(sp.U, st.U, cells),
              "response_sums": [float(v) for v in (O.sums(pb, sp.U) - O.sums(pb, st.U))],
              "response_ledger": sp.ledger - st.ledger}
        out["checkpoints"].append(ck)
        print("step %d: %.0f s, response grid %s cells %s" % (k, time.time() - t, ck["response_grid"],
                                                              ck["response_cells"]), flush=True)
        with open(os.path.join(HERE, "paper_event_256.json"), "w") as f:
            json.dump(out, f, indent=0)
    print("total %.0f s" % (time.time() - t_all), flush=True)


if __name__ == "__main__":
    main()
