"""Writes tests/golden/gradient_event_128.json: eps2 and its complex-step
derivatives with respect to kappa_rad, kappa_coll, x0, y0 of the 128^3,
100-step differentiable event (workloads.gradient_event), from the oracle only.

    python tests/golden/make_gradient_golden.py      # ~10 min per parameter on 8 cores
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1511_02137_amd import workloads as W  # noqa: E402


def main():
    w = W.gradient_event()
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, bc=tuple(w.bc), deposit=w.deposit)
    jets = [O.Jet(**j.__dict__) for j in w.jets]
    out = {"workload": w.name, "steps": w.steps, "deposit": w.deposit, "method": "oracle complex step, h = 1e-30",
           "jet0": {k: v for k, v in w.jets[0].__dict__.items()}, "grad": {}}
    for which in ("kappa_rad", "kappa_coll", "x0", "y0"):
        t = time.time()
        v, d = O.eps2_complex_step(pb, w.prim0, w.steps, jets, which)
        out["eps2"] = v
        out["grad"][which] = d
        print(which, repr(v), repr(d), "%.0f s" % (time.time() - t), flush=True)
    with open(os.path.join(HERE, "gradient_event_128.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
