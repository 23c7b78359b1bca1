"""GPU freeze-out (hydro_freezeout: Cooper-Frye on the fixed-time surface,
massless Boltzmann particles, rapidity 0, azimuthal spectra and flow
harmonics) against the oracle's on the same state.

Both sides take the state's values (FP64, or the FP32 form's values widened
exactly) and do all arithmetic in FP64; they differ only in summation order
and in the last bit of a few library functions (cos/sin, exp, 1/D), so the
bar is 1e-12 relative per output (spectra, dN/dy) and 1e-12 absolute for the
normalised harmonics.
"""
import numpy as np
import pytest

import oracle as O
from paper_1511_02137_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1511_02137_amd import hydro as H
    H.load_library()


def H():
    from paper_1511_02137_amd import hydro
    return hydro


def compare(h, w, n_phi, pt, T_min=0.0, dof=1.0, n_harm=8):
    spec, harm = h.freezeout(n_phi=n_phi, pt=pt, T_min=T_min, dof=dof, n_harm=n_harm)
    torch.cuda.synchronize()
    spec, harm = spec.cpu().numpy(), harm.cpu().numpy()
    U = h.U.cpu().numpy().astype(np.float64)
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt)
    rs, rh, _ = O.freezeout(pb, U, n_phi=n_phi, pt=pt, T_min=T_min, dof=dof, n_harm=n_harm)
    err_s = np.abs(spec - rs).max(axis=1) / np.abs(rs).max(axis=1)
    err_y = np.abs(harm[:, 0, 0] - rh[:, 0, 0]) / np.abs(rh[:, 0, 0])
    err_h = np.abs(harm[:, 1:] - rh[:, 1:]).max() if n_harm else 0.0
    print("n %s n_phi %d n_pt %d T_min %g: spectra %.2e dN/dy %.2e harmonics %.2e" % (
        w.n, n_phi, len(pt), T_min, err_s.max(), err_y.max(), err_h), flush=True)
    assert np.all(err_s <= 1e-12), err_s
    assert np.all(err_y <= 1e-12), err_y
    assert err_h <= 1e-12
    assert harm[:, 0, 1].max() == 0.0
    return spec, harm, rh


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_small_event_after_its_run(precision):
    w = W.small_event(1)
    print("small event", w.n, precision, flush=True)
    h = H().from_workload(w, precision=precision)
    h.step(w.steps)
    compare(h, w, 64, [0.5, 1.0, 2.0, 3.0])
    compare(h, w, 64, [0.5, 1.0, 2.0, 3.0], T_min=0.15, dof=16.0)
    h.close()


@pytest.mark.parametrize("n_phi,pt,n_harm", [
    # n_phi <= 256: lanes own azimuths, 256 // n_phi groups split the cells
    (1, [], 0),                      # one azimuth: 256 groups
    (3, [0.7], 1),                   # 85 groups, lane 255 idle
    (48, [0.4, 2.2], 12),            # 5 groups, lanes 240..255 idle
    (256, [], 32),                   # one group
    (100, [0.3, 0.9, 1.5], 20),      # 2 groups, lanes 200..255 idle
    (64, list(np.linspace(0.2, 4.0, 15)), 31),  # the most rows, 1024 outputs
    # n_phi > 256: lanes own outputs (row, azimuth), up to four each
    (300, [0.5, 1.5], 8),            # 900 outputs: four per lane, the last partly owned
    (1024, [], 16),                  # the most azimuths
])
def test_output_shapes_and_ragged_grids(n_phi, pt, n_harm):
    w = W.small_event(1, n=(21, 18, 13), steps=3)  # 4914 cells: not a multiple of 256
    print("ragged", w.n, n_phi, len(pt), n_harm, flush=True)
    h = H().from_workload(w)
    h.step(w.steps)
    compare(h, w, n_phi, pt, n_harm=n_harm)
    h.close()


def test_paper_shape_after_steps():
    """The 256^3 paper event after 20 steps: all 16.7 M cells, 32 outputs,
    against the oracle on the downloaded state."""
    w = W.paper_event(2)
    print("paper event 256^3, 20 steps", flush=True)
    h = H().from_workload(w)
    h.step(20)
    spec, harm, rh = compare(h, w, 16, [1.0], n_harm=7)
    print("v2 (cos, sin) per row", harm[:, 2].tolist(), flush=True)
    h.close()


def test_repeatable_and_reading_only():
    w = W.small_event(1, n=(24, 20, 16), steps=2)
    h = H().from_workload(w, precision="f32")
    h.step(2)
    U0 = h.U.clone()
    f0 = h.fixups()
    a = [t.cpu().numpy() for t in h.freezeout(n_phi=40, pt=[0.5, 1.5], n_harm=9)]
    b = [t.cpu().numpy() for t in h.freezeout(n_phi=40, pt=[0.5, 1.5], n_harm=9)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert torch.equal(U0, h.U) and h.fixups() == f0
    h.close()


def test_no_particles_above_every_cell():
    """T_min above every cell's temperature: zero spectra, dN/dy and v_n
    (0, not 0/0), as in the oracle."""
    w = W.small_event(1, n=(12, 12, 12), steps=1)
    h = H().from_workload(w)
    spec, harm = h.freezeout(n_phi=16, pt=[1.0, 2.0], T_min=100.0, n_harm=4)
    spec, harm = spec.cpu().numpy(), harm.cpu().numpy()
    assert np.all(spec == 0.0) and np.all(harm == 0.0)
    h.close()


def test_argument_checks():
    w = W.small_event(1, n=(12, 12, 12), steps=1)
    h = H().from_workload(w)
    bad = [dict(n_phi=0), dict(n_phi=64, pt=[1.0] * 16), dict(n_phi=128, pt=[1.0] * 8),
           dict(n_phi=16, n_harm=8), dict(n_phi=64, n_harm=33), dict(pt=[0.0]), dict(pt=[-1.0]),
           dict(dof=0.0), dict(T_min=-0.1)]
    for kw in bad:
        with pytest.raises(H().HydroError) as ei:
            h.freezeout(**kw)
        assert ei.value.code == H().HYDRO_EINVAL, kw
    h.close()
