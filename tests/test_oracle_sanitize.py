"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(oracle/build_oracle.py --sanitize, host code only) runs clean through small
cases of every entry point: prim->cons, cons->prim with fix-ups, runs of
WENO7-Z/JS, WENO5, the limiter, MUSTA-FORCE, NGP and Gaussian jets, a
1 x 1 x 12 grid, periodic boxes, eps2 and its complex step, the
Jacobian-vector product and the freeze-out.  The child process preloads the
ASan runtime; any report makes it exit non-zero."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import oracle as O
from paper_1511_02137_amd import workloads as W
w = W.small_event(1, n=(10, 9, 8), steps=2)
jets = [O.Jet(**j.__dict__) for j in w.jets]
for kw in (dict(), dict(weno="js"), dict(weno="z5"), dict(limiter="pp"), dict(flux="musta", musta_k=2),
           dict(bc=("periodic",) * 3), dict(deposit="gauss")):
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, **kw)
    U = O.prim_to_cons(pb, w.prim0)
    st = O.run(pb, U, 2, jets)
    O.cons_to_prim(pb, st.U)
    O.rhs(pb, st.U, 1.0, jets)
    O.sums(pb, st.U)
    O.eps2(pb, st.U)
pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, deposit="gauss")
O.eps2_complex_step(pb, w.prim0, 1, jets, "x0")
U = O.prim_to_cons(pb, w.prim0)
O.jvp(pb, U, np.ones_like(U) * 1e-3, 1, jets)
O.freezeout(pb, U, n_phi=16, pt=[0.5, 1.0], T_min=0.1, n_harm=4)
bad = U.copy(); bad[0, 2, 2, 2] = -1.0; bad[1, 3, 3, 3] = 2.0 * bad[0, 3, 3, 3]
print("fixups", O.cons_to_prim(pb, bad)[1])
one = O.Problem(n=(1, 1, 12), dx=(0.1, 0.1, 0.1))
prim = np.zeros((5, 12, 1, 1)); prim[0] = np.linspace(1, 3, 12)[:, None, None]; prim[4] = 0.5
O.run(one, O.prim_to_cons(one, prim), 2)
print("sanitized oracle: clean")
"""


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    from oracle import build_oracle
    try:
        lib = build_oracle.build(force=True, sanitize=True)
    except (subprocess.CalledProcessError, OSError) as e:
        pytest.fail("sanitized build failed: %s" % e)
    env = dict(os.environ)
    env["LD_PRELOAD"] = build_oracle.asan_runtime()
    env["HYDRO_ORACLE_LIB"] = lib
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle: clean" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
