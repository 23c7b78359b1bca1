"""hydro_sums_noalloc (the entry point for callers that cannot allocate)
against hydro_sums, through the C ABI: two calls in a row on different
contexts, the second on a smaller grid, each bit for bit equal to
hydro_sums of the same state, plus the argument checks."""
import ctypes

import numpy as np
import pytest

from paper_1511_02137_amd import hydro as H
from paper_1511_02137_amd import workloads as W

pytestmark = pytest.mark.gpu


def _event(n, precision, steps):
    w = W.small_event(1, n=n, steps=steps)
    h = H.from_workload(w, precision=precision)
    h.step(steps)
    return h


def test_sums_noalloc_matches_sums_on_two_calls_second_smaller():
    import torch
    big = _event((40, 36, 30), "f64", 3)
    small = _event((20, 18, 16), "f32", 2)
    for h in (big, small):
        out = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
        print("hydro_sums_noalloc on %s %s" % (tuple(h.cfg.n), "f32" if h.cfg.precision else "f64"), flush=True)
        h.sums_noalloc(out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = h.sums()
        assert np.array_equal(got, ref), (got, ref)
        assert got[5] > 0.0  # the jet has deposited energy
    big.close()
    small.close()


def test_sums_noalloc_rejects_host_output_and_null():
    import torch
    h = _event((20, 18, 16), "f64", 1)
    lib = h.lib
    host = (ctypes.c_double * 6)()
    assert lib.hydro_sums_noalloc(h.ctx, h.U.data_ptr(), ctypes.cast(host, ctypes.c_void_p), None) == H.HYDRO_EINVAL
    out = torch.zeros(6, dtype=torch.float64, device="cuda")
    assert lib.hydro_sums_noalloc(h.ctx, None, out.data_ptr(), None) == H.HYDRO_EINVAL
    assert lib.hydro_sums_noalloc(None, h.U.data_ptr(), out.data_ptr(), None) == H.HYDRO_EINVAL
    h.close()
