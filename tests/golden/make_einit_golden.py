"""Writes tests/golden/gradient_event_128_einit.json from the oracle alone:
directional derivatives of eps2 with respect to the initial energy density
of the 128^3, 100-step differentiable event (workloads.gradient_event) along
two smooth directions, by the complex-step method (h = 1e-30):

  "fireball": d e_init = e_init - 1e-3 (the Gaussian ellipsoid itself);
  "blob":     d e_init = exp(-|x - (-1, 0, 0) fm|^2 / (2 (0.5 fm)^2)), a bump
              on the jet's path next to the z = 0 plane.

For each it also stores the derivative at an initial state changed by a
relative 1e-14 (seeded, uniform in [-1, 1]): how much the derivative itself
moves under a change of rounding size, the bar for comparing any two correct
implementations.

    python tests/golden/make_einit_golden.py     # ~40 min on 8 cores
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


def directions(w):
    nx, ny, nz = w.n
    c = [(np.arange(n) - 0.5 * (n - 1)) * w.dx[d] for d, n in enumerate(w.n)]
    z, y, x = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    return {"fireball": w.prim0[0] - 1e-3,
            "blob": np.exp(-((x + 1.0) ** 2 + y ** 2 + z ** 2) / (2 * 0.5 ** 2))}


def main():
    w = W.gradient_event()
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, bc=tuple(w.bc), deposit=w.deposit)
    jets = [O.Jet(**j.__dict__) for j in w.jets]
    prim_p = w.prim0.copy()
    prim_p[0] *= 1.0 + 1e-14 * np.random.default_rng(11).uniform(-1.0, 1.0, size=prim_p[0].shape)
    out = {"workload": w.name, "steps": w.steps, "deposit": w.deposit, "method": "oracle complex step, h = 1e-30",
           "perturbation": "e_init * (1 + 1e-14 u), u ~ U(-1, 1), numpy default_rng(11)",
           "directions": {"fireball": "e_init - 1e-3",
                          "blob": "exp(-|x - (-1, 0, 0)|^2 / (2 * 0.5^2)), x in fm"},
           "grad": {}, "grad_perturbed": {}}
    for name, d in directions(w).items():
        for key, prim in (("grad", w.prim0), ("grad_perturbed", prim_p)):
            t = time.time()
            v, g = O.eps2_complex_step(pb, prim, w.steps, jets, "e_init", de=d)
            out[key][name] = g
            if key == "grad":
                out["eps2"] = v
            print(name, key, repr(g), "%.0f s" % (time.time() - t), flush=True)
            with open(os.path.join(HERE, "gradient_event_128_einit.json"), "w") as f:
                json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
