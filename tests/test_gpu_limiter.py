"""GPU positivity-preserving flux limiter (HYDRO_LIMITER_PP) against the
oracle's, on the events that need it, and across launch shapes and batches.

Bars: FP64 relative L-infinity 1e-12 of the oracle on the peripheral jet; no
recovery fix-ups and E - |M| > 0, N > 0 everywhere; kernel variants and
batches bitwise equal.  Near vacuum the limited map amplifies rounding: in
the oracle itself a 1e-15 relative change of the initial state of the
vacuum Riemann problem moves E by ~5e-12 (unlimited: ~1e-14), and a change
of FP32 rounding size (6e-8) moves the peripheral jet's e and |v| by ~1e-5
and ~4e-5 (relative L2).  There the bar is three times the oracle's own
response to such a change, measured in the test: FP64 max(1e-12, 3 x the
1e-15 response); FP32 form against FP64: 3 x the 6e-8 response.
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


def oracle_run(w, steps, bc=None, weno="z", limiter="pp"):
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, bc=tuple(bc or w.bc), weno=weno, deposit=w.deposit,
                   limiter=limiter)
    return O.run(pb, O.prim_to_cons(pb, w.prim0), steps, [O.Jet(**j.__dict__) for j in w.jets])


def gpu_run(w, steps, precision="f64", bc=None, weno="z", limiter="pp", opts=None):
    h = H().from_workload(w, precision=precision, weno=weno, bc=bc, limiter=limiter)
    for k, v in (opts or {}).items():
        h.set_option(k, v)
    h.step(steps)
    torch.cuda.synchronize()
    out = h.U.cpu().numpy().astype(np.float64), h.fixups(), h.get_state()
    h.close()
    return out


def rel_linf(a, b):
    Emax = np.abs(b[0]).max()
    return np.array([np.abs(a[f] - b[f]).max() / (Emax if f in (1, 2, 3) else np.abs(b[f]).max())
                     for f in range(5)])


def oracle_response(w, steps, rel, seed=0):
    """Relative change of the oracle's limited run (per field, L-infinity as
    rel_linf, and L2 of e and |v|) after a random relative change `rel` of
    the initial conserved state."""
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, bc=tuple(w.bc), deposit=w.deposit, limiter="pp")
    U0 = O.prim_to_cons(pb, w.prim0)
    jets = [O.Jet(**j.__dict__) for j in w.jets]
    a = O.run(pb, U0, steps, jets).U
    rng = np.random.default_rng(seed)
    b = O.run(pb, U0 * (1.0 + rel * rng.uniform(-1.0, 1.0, U0.shape)), steps, jets).U
    (ea, va), (eb, vb) = prim_ev(a), prim_ev(b)
    return rel_linf(b, a), (np.linalg.norm(eb - ea) / np.linalg.norm(ea), np.linalg.norm(vb - va) / np.linalg.norm(va))


def prim_ev(U):
    M = np.sqrt(U[1] ** 2 + U[2] ** 2 + U[3] ** 2)
    e = 3 * (U[0] ** 2 - M ** 2) / (U[0] + np.sqrt(4 * U[0] ** 2 - 3 * M ** 2))
    return e, M / (U[0] + e / 3)


def admissible(U):
    g = U[0] - np.sqrt(U[1] ** 2 + U[2] ** 2 + U[3] ** 2)
    return g.min() > 0 and U[4].min() > 0


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
@pytest.mark.parametrize("weno", ["z", "z5"])
def test_peripheral_jet_matches_oracle(bc, weno):
    w = W.peripheral_jet_event()
    print("peripheral jet", w.n, bc, weno, flush=True)
    st = oracle_run(w, w.steps, bc=(bc,) * 3, weno=weno)
    assert st.fixups == 0
    U, fx, (_, step, Ej) = gpu_run(w, w.steps, bc=(bc,) * 3, weno=weno)
    err = rel_linf(U, st.U)
    print("rel Linf", err, flush=True)
    assert np.all(err <= 1e-12), err
    assert fx == 0 and admissible(U)
    assert step == w.steps and Ej[0] == pytest.approx(st.Ejet[0], rel=1e-12)


def test_unlimited_gpu_run_needs_the_limiter():
    w = W.peripheral_jet_event()
    U, fx, _ = gpu_run(w, w.steps, limiter="none")
    assert fx > 0 or not admissible(U)


def test_unlimited_run_through_the_fixup_branch_matches_oracle():
    """The unlimited scheme on the peripheral jet: from step 23 on, stage
    states next to the deposit leave the admissible set and both recoveries
    take the fix-up branch (M rescaled to the speed cap).  The GPU follows the
    oracle through it.  Bar per field: max(1e-12, 4 x the oracle's own
    response to a 1e-15 relative change of the initial e, measured here):
    the N field next to the deposit is that sensitive (response ~5e-13 of
    max N from step 24 on), and the GPU's rounding differs from the oracle's
    in each of the 90 stages, not once.  Observed: E 3.0e-13, N 1.38e-12
    (3.0 x its response).  (The fix-up counts differ by design: the GPU
    counts every recovery of a halo point, the oracle each cell once.)"""
    w = W.peripheral_jet_event()
    print("peripheral jet, unlimited, FP64", w.n, w.steps, flush=True)
    st = oracle_run(w, w.steps, limiter="none")
    assert st.fixups > 0
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, bc=tuple(w.bc), deposit=w.deposit)
    prim = w.prim0.copy()
    prim[0] *= 1.0 + 1e-15 * np.random.default_rng(7).uniform(-1.0, 1.0, prim[0].shape)
    sp = O.run(pb, O.prim_to_cons(pb, prim), w.steps, [O.Jet(**j.__dict__) for j in w.jets])
    bar = np.maximum(1e-12, 4.0 * rel_linf(sp.U, st.U))
    U, fx, (_, step, Ej) = gpu_run(w, w.steps, limiter="none")
    err = rel_linf(U, st.U)
    print("rel Linf", err, "bar", bar, "fix-ups gpu", fx, "oracle", st.fixups, flush=True)
    assert fx > 0
    assert np.all(err <= bar), (err, bar)
    assert Ej[0] == pytest.approx(st.Ejet[0], rel=1e-12)


@pytest.mark.parametrize("n,njets,precision", [((256, 256, 256), 1, "f64"), ((256, 256, 256), 3, "f32"),
                                               ((512, 512, 512), 3, "f32")])
def test_fp32_event_needs_no_fixups_with_the_limiter(n, njets, precision):
    """The small event's initial state on the large grids with 1-3 jets, the
    full run (256^3: 120 steps; 512^3: 60).  Unlimited, the NGP deposit (a
    light-like spike into one cell every step) drives stage states next to it
    out of the admissible set after 14-33 steps (fix-ups > 0, measured); with
    the positivity-preserving limiter, the reading used for this workload,
    there is none, and every cell of the final state is admissible."""
    w = W.fp32_event(3, n=n, njets=njets)
    print("fp32_event", n, njets, precision, w.steps, flush=True)
    h = H().from_workload(w, precision=precision, limiter="pp")
    h.step(w.steps)
    torch.cuda.synchronize()
    assert h.fixups() == 0
    E = h.U[0].double()
    M = torch.sqrt(h.U[1].double() ** 2 + h.U[2].double() ** 2 + h.U[3].double() ** 2)
    assert float((E - M).min()) > 0 and float(h.U[4].min()) > 0
    h.close()
    hu = H().from_workload(w, precision=precision, limiter="none")
    hu.step(w.steps)
    print("unlimited fix-ups", hu.fixups(), flush=True)
    assert hu.fixups() > 0
    hu.close()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_vacuum_riemann_matches_oracle(axis):
    # e_R = 1e-7: the unlimited scheme leaves E < |M| and N < 0 (oracle);
    # limited states stay far from the recovery's speed cap
    w = W.vacuum_riemann(N=120, axis=axis, e_right=1e-7)
    print("vacuum riemann axis", axis, w.n, w.steps, flush=True)
    st = oracle_run(w, w.steps)
    assert st.fixups == 0
    U, fx, _ = gpu_run(w, w.steps)
    err = rel_linf(U, st.U)
    bar = np.maximum(1e-12, 3.0 * oracle_response(w, w.steps, 1e-15)[0])
    print("rel Linf", err, "bar", bar, flush=True)
    assert np.all(err <= bar), (err, bar)
    assert fx == 0 and admissible(U)


def test_launch_shapes_are_bitwise():
    w = W.peripheral_jet_event(n=(37, 21, 18), steps=12)
    H_ = H()
    ref, _, _ = gpu_run(w, w.steps)
    for opts in ({H_.OPT_X_KERNEL: 1}, {H_.OPT_YZ_KERNEL: 1}, {H_.OPT_YZ_KERNEL: 1, H_.OPT_MARCH_SEG: 5}):
        U, _, _ = gpu_run(w, w.steps, opts=opts)
        assert np.array_equal(U, ref), opts
    for bc in (("periodic", "outflow", "periodic"),):
        a, _, _ = gpu_run(w, w.steps, bc=bc)
        b, _, _ = gpu_run(w, w.steps, bc=bc, opts={H_.OPT_X_KERNEL: 1})
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_matches_single_events(precision):
    ws = [W.peripheral_jet_event(), W.peripheral_jet_event(n=(20, 26, 18), steps=30),
          W.peripheral_jet_event(mirror=True)]
    b = H().batch_from_workloads(ws, precision=precision, limiter="pp")
    b.run(20)
    torch.cuda.synchronize()
    for e, w in enumerate(ws):
        U, fx, _ = gpu_run(w, 20, precision=precision)
        assert np.array_equal(b.U[e].cpu().numpy().astype(np.float64), U), e
    assert b.fixups() == 0
    b.close()


def test_mirror_image_is_bitwise():
    a, _, _ = gpu_run(W.peripheral_jet_event(), 30)
    b, _, _ = gpu_run(W.peripheral_jet_event(mirror=True), 30)
    b = b[:, :, :, ::-1].copy()
    b[1] = -b[1]
    assert np.array_equal(a, b)


def test_smooth_event_unchanged_bitwise():
    w = W.small_event(n=(33, 20, 18), steps=5, with_jet=False)
    a, _, _ = gpu_run(w, 5, limiter="none")
    b, _, _ = gpu_run(w, 5, limiter="pp")
    assert np.array_equal(a, b)


def test_fp32_form():
    w = W.peripheral_jet_event()
    U32, fx, _ = gpu_run(w, w.steps, precision="f32")
    U64, _, _ = gpu_run(w, w.steps)
    assert fx == 0 and admissible(U32)
    e32, v32 = prim_ev(U32)
    e64, v64 = prim_ev(U64)
    l2e = np.linalg.norm(e32 - e64) / np.linalg.norm(e64)
    l2v = np.linalg.norm(v32 - v64) / np.linalg.norm(v64)
    _, (re_, rv) = oracle_response(w, w.steps, 2.0 ** -24)
    print("fp32 rel L2 e %.2e |v| %.2e; oracle response e %.2e |v| %.2e" % (l2e, l2v, re_, rv), flush=True)
    assert l2e <= 3.0 * re_ and l2v <= 3.0 * rv


def test_adjoint_refuses_the_limiter():
    cfg = H().make_config((16, 16, 16), limiter="pp")
    assert H().workspace_bytes(cfg, 2) == 0
    assert H().workspace_bytes(cfg, 0) > 0
    with pytest.raises(H().HydroError):
        H().Hydro(cfg, W.uniform_prim((16, 16, 16)), adjoint_k=2)
