"""GPU adjoint: gradients of eps2 from the hand-written reverse sweep
(hydro_loss_eps2 seed, hydro_adjoint_step, hydro_init_vjp) against the
oracle's complex-step derivatives of the same discrete map, against central
differences of the GPU forward, and between checkpoint intervals.

Bars.  FP64: the adjoint and the complex step are both exact derivatives of
the discrete map, so they differ only by rounding carried through the run;
the forward's own rounding reaches ~1e-12 relative after the outflow WENO-Z
amplification, and the reverse sweep carries the same factor, so 1e-9
relative (of the largest gradient entry compared) leaves three digits of
margin while any dropped term or wrong sign gives an O(1) error.  Checkpoint
interval: bitwise (the recomputation repeats the forward's arithmetic).
Central differences: truncation O(h^2) with h = 1e-4 relative, bar 1e-5.
"""
import numpy as np
import pytest

import oracle as O
from paper_1511_02137_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PARAMS = ["kappa_rad", "kappa_coll", "x0", "y0"]


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1511_02137_amd import hydro as H
    H.load_library()


def adjoint_mod():
    from paper_1511_02137_amd import adjoint
    return adjoint


def small(n=(20, 18, 16), steps=5, deposit="gauss"):
    w = W.small_gradient_event(n=n, steps=steps)
    w.deposit = deposit
    w.jets[0].x0 = (-0.3345, 0.031, 0.013)  # inside the box, off every cell face at every stage time
    return w


def oracle_problem(w):
    return O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, bc=tuple(w.bc), deposit=w.deposit)


def oracle_jets(w):
    return [O.Jet(**j.__dict__) for j in w.jets]


def gpu_grads(w, precision="f64", ckpt=2, record=False):
    A = adjoint_mod()
    pb = A.Eps2Problem(w, precision=precision, ckpt_every=ckpt, record=record)
    j = w.jets[0]
    e0 = torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda")
    eps, cks, Uf, prim = pb.forward(e0, j.kappa_rad, j.kappa_coll, j.x0[0], j.x0[1])
    ge, gj = pb.backward(cks, Uf, prim)
    torch.cuda.synchronize()
    out = {"eps2": float(eps.item()), "e_init": ge.cpu().numpy(), "jets": gj.cpu().numpy()}
    pb.h.close()
    return out


def smooth_direction(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    out = np.zeros(shape)
    for _ in range(4):
        kx, ky, kz = rng.integers(0, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        out += rng.normal() * (np.cos(2 * np.pi * kx * np.arange(nx) / nx + ph[0])[None, None, :]
                               * np.cos(2 * np.pi * ky * np.arange(ny) / ny + ph[1])[None, :, None]
                               * np.cos(2 * np.pi * kz * np.arange(nz) / nz + ph[2])[:, None, None])
    return out


@pytest.fixture(scope="module")
def small_case():
    w = small()
    print("adjoint small case", w.n, w.steps, flush=True)
    return w, gpu_grads(w)


def test_eps2_value_matches_oracle(small_case):
    w, g = small_case
    pb = oracle_problem(w)
    st = O.run(pb, O.prim_to_cons(pb, w.prim0), w.steps, oracle_jets(w))
    ref = O.eps2(pb, st.U)
    assert abs(g["eps2"] - ref) <= 1e-12 * abs(ref), (g["eps2"], ref)


@pytest.mark.parametrize("which", PARAMS)
def test_param_gradient_matches_complex_step(small_case, which):
    w, g = small_case
    _, ref = O.eps2_complex_step(oracle_problem(w), w.prim0, w.steps, oracle_jets(w), which)
    got = g["jets"][0, PARAMS.index(which)]
    assert ref != 0.0
    assert abs(got - ref) <= 1e-9 * abs(ref), (which, got, ref, (got - ref) / ref)


@pytest.mark.parametrize("seed", [11, 12])
def test_initial_field_gradient_matches_complex_step(small_case, seed):
    w, g = small_case
    de = smooth_direction(w.prim0[0].shape, seed) * w.prim0[0]
    _, ref = O.eps2_complex_step(oracle_problem(w), w.prim0, w.steps, oracle_jets(w), "e_init", de=de)
    got = float(np.sum(g["e_init"] * de))
    assert abs(got - ref) <= 1e-9 * abs(ref), (got, ref, (got - ref) / ref)


def test_initial_field_gradient_pointwise_sample(small_case):
    # single cells near the jet and in the z = 0 planes: d eps2 / d e_init(cell)
    w, g = small_case
    nz, ny, nx = w.prim0[0].shape
    pb = oracle_problem(w)
    cells = [(nz // 2, ny // 2, nx // 2 - 3), (nz // 2 - 1, ny // 2 + 2, 4), (1, 2, 3)]
    scale = np.abs(g["e_init"]).max()
    for (k, j, i) in cells:
        de = np.zeros((nz, ny, nx))
        de[k, j, i] = 1.0
        _, ref = O.eps2_complex_step(pb, w.prim0, w.steps, oracle_jets(w), "e_init", de=de)
        got = g["e_init"][k, j, i]
        assert abs(got - ref) <= 1e-9 * scale, ((k, j, i), got, ref, scale)


def test_ngp_deposit_kappa_gradients_and_zero_origin_gradient():
    w = small(deposit="ngp")
    g = gpu_grads(w)
    pb = oracle_problem(w)
    for which in ("kappa_rad", "kappa_coll"):
        _, ref = O.eps2_complex_step(pb, w.prim0, w.steps, oracle_jets(w), which)
        got = g["jets"][0, PARAMS.index(which)]
        assert abs(got - ref) <= 1e-9 * abs(ref), (which, got, ref)
    assert np.all(g["jets"][0, 2:5] == 0.0)


def test_checkpoint_interval_is_bitwise_invariant():
    w = small(steps=6)
    a = gpu_grads(w, ckpt=1)
    b = gpu_grads(w, ckpt=4)   # segments 4 + 2
    c = gpu_grads(w, ckpt=6)
    for x in (b, c):
        assert x["eps2"] == a["eps2"]
        assert np.array_equal(x["jets"], a["jets"])
        assert np.array_equal(x["e_init"], a["e_init"])


def test_autograd_function_matches_direct_backward(small_case):
    w, g = small_case
    A = adjoint_mod()
    pb = A.Eps2Problem(w, ckpt_every=2)
    j = w.jets[0]

    def leaves():
        return (torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda", requires_grad=True),
                torch.tensor(j.kappa_rad, dtype=torch.float64, requires_grad=True),
                torch.tensor(j.kappa_coll, dtype=torch.float64, requires_grad=True),
                torch.tensor(j.x0[:2], dtype=torch.float64, requires_grad=True))

    e0, kr, kc, xy = leaves()
    loss = A.eps2(e0, kr, kc, xy, pb)
    loss.backward()
    assert float(loss.item()) == g["eps2"]
    assert np.array_equal(e0.grad.cpu().numpy(), g["e_init"])
    assert kr.grad.item() == g["jets"][0, 0]
    assert kc.grad.item() == g["jets"][0, 1]
    assert np.array_equal(xy.grad.numpy(), g["jets"][0, 2:4])
    # an upstream factor scales the seed; the sweep is linear in it
    e0, kr, kc, xy = leaves()
    (3.0 * A.eps2(e0, kr, kc, xy, pb)).backward()
    np.testing.assert_allclose(e0.grad.cpu().numpy(), 3.0 * g["e_init"], rtol=0,
                               atol=1e-12 * np.abs(g["e_init"]).max())
    np.testing.assert_allclose(xy.grad.numpy(), 3.0 * g["jets"][0, 2:4], rtol=1e-12)
    assert kr.grad.item() == pytest.approx(3.0 * g["jets"][0, 0], rel=1e-12)
    pb.h.close()


@pytest.mark.parametrize("which", PARAMS)
def test_param_gradient_matches_gpu_central_differences(small_case, which):
    w, g = small_case
    A = adjoint_mod()
    pb = A.Eps2Problem(w, ckpt_every=w.steps)
    j = w.jets[0]
    e0 = torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda")
    base = {"kappa_rad": j.kappa_rad, "kappa_coll": j.kappa_coll, "x0": j.x0[0], "y0": j.x0[1]}
    h = 1e-4 * abs(base[which])

    def f(s):
        p = dict(base)
        p[which] += s
        eps, _, _, _ = pb.forward(e0, p["kappa_rad"], p["kappa_coll"], p["x0"], p["y0"])
        return float(eps.item())

    fd = (f(h) - f(-h)) / (2 * h)
    got = g["jets"][0, PARAMS.index(which)]
    pb.h.close()
    assert abs(got - fd) <= 1e-5 * abs(got), (which, got, fd)


def test_adjoint_rejects_more_steps_than_workspace():
    from paper_1511_02137_amd import hydro as H
    w = small(steps=2)
    h = H.from_workload(w, adjoint_k=1)
    lam = torch.zeros_like(h.U)
    grad = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(H.HydroError):
        h.adjoint_step(h.U.clone(), 0, [w.jets[0].E0], 2, lam, grad)
    h.close()
    h0 = H.from_workload(w)  # no adjoint workspace
    with pytest.raises(H.HydroError):
        h0.adjoint_step(h0.U.clone(), 0, [w.jets[0].E0], 1, torch.zeros_like(h0.U), grad)
    with pytest.raises(H.HydroError) as ei:
        h0.step_record(1)
    assert ei.value.code == H.HYDRO_EINVAL
    with pytest.raises(H.HydroError) as ei:  # nothing recorded
        h0.adjoint_recorded(torch.zeros_like(h0.U), grad)
    assert ei.value.code == H.HYDRO_ESTATE
    h0.close()
    # schemes the adjoint does not cover get no adjoint workspace at all
    with pytest.raises(H.HydroError):
        H.from_workload(w, weno="z5", adjoint_k=2)


# --- the differentiable run's sizes --------------------------------------------------------------------------------

def test_32cube_gradients_match_complex_step():
    """The 32^3, 10-step differentiable event: the four parameter gradients and
    an initial-field direction against the oracle's complex step.

    The initial-field derivative of this run is ill-conditioned: the second
    derivatives of the outflow WENO-Z faces grow step by step, so a random
    1e-14 relative change of e_init moves the oracle's own complex-step value
    by ~1e-7 relative (and ~1e-5 for 1e-13) after 10 steps, against 1e-15 after
    2 steps; the parameter gradients move by <1e-11.  GPU and oracle differ by
    rounding at every operation, so the initial-field bar is that measured
    response (at least 1e-9): a wrong term still gives an O(1) error."""
    w = W.small_gradient_event(n=(32, 32, 32), steps=10)
    g = gpu_grads(w, ckpt=4)
    pb = oracle_problem(w)
    for which in PARAMS:
        _, ref = O.eps2_complex_step(pb, w.prim0, w.steps, oracle_jets(w), which)
        got = g["jets"][0, PARAMS.index(which)]
        assert abs(got - ref) <= 1e-9 * abs(ref), (which, got, ref)
    de = smooth_direction(w.prim0[0].shape, 3) * w.prim0[0]
    _, ref = O.eps2_complex_step(pb, w.prim0, w.steps, oracle_jets(w), "e_init", de=de)
    p = w.prim0.copy()
    p[0] *= 1.0 + 1e-14 * np.random.default_rng(0).normal(size=p[0].shape)
    _, ref_p = O.eps2_complex_step(pb, p, w.steps, oracle_jets(w), "e_init", de=de)
    bar = max(1e-9 * abs(ref), abs(ref_p - ref))
    got = float(np.sum(g["e_init"] * de))
    print("32^3 e_init direction: gpu %.15e oracle %.15e, conditioning bar %.3e" % (got, ref, bar / abs(ref)))
    assert abs(got - ref) <= bar, (got, ref, bar)


def test_differentiable_run_matches_full_size_complex_step_fixture():
    """128^3, 100 steps, checkpoints every 10: FP64 adjoint against the
    oracle's complex-step gradients stored in tests/golden (written by
    tests/golden/make_gradient_golden.py from the oracle alone); the FP32
    form against the same values with its stated error."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "gradient_event_128.json")))
    w = W.gradient_event()
    assert w.name == gold["workload"] and w.steps == gold["steps"]
    g64 = gpu_grads(w, "f64", ckpt=10)
    assert abs(g64["eps2"] - gold["eps2"]) <= 1e-12 * abs(gold["eps2"])
    for k, which in enumerate(PARAMS):
        ref = gold["grad"][which]
        assert abs(g64["jets"][0, k] - ref) <= 1e-9 * abs(ref), (which, g64["jets"][0, k], ref)
    g32 = gpu_grads(w, "f32", ckpt=10)
    assert abs(g32["eps2"] - gold["eps2"]) <= 1e-6 * abs(gold["eps2"])
    # FP32 fields, FP64 gradient accumulation: kappa gradients to 1e-4, origin
    # gradients to 2e-2 (measured 2e-5, 1e-5, 7e-5, 5e-3)
    for k, (which, bar) in enumerate(zip(PARAMS, (1e-4, 1e-4, 2e-2, 2e-2))):
        ref = gold["grad"][which]
        rel = abs(g32["jets"][0, k] - ref) / abs(ref)
        print("FP32 %s: rel %.2e" % (which, rel))
        assert rel <= bar, (which, rel)


def test_initial_field_gradient_at_full_size():
    """The initial-field gradient of the 128^3, 100-step differentiable run.

    FP64 adjoint against the oracle's complex-step directional derivatives
    (tests/golden/gradient_event_128_einit.json, written by
    tests/golden/make_einit_golden.py from the oracle alone) along a smooth
    bump on the jet's path and along the fireball itself; the bar is
    max(1e-9 relative, 4 x how far the oracle's own derivative moves when
    e_init changes by a relative 1e-14) -- the gradient next to the outflow
    faces is that ill-conditioned.

    FP32 form against FP64, per region (measured on the GPU): within 16 cells
    of an outflow face the FP64 gradient itself moves by ~7e-6 under a 1e-14
    change of e_init and FP32 rounding moves it at O(1) (it carries 99.8 % of
    the gradient's norm: the x^2 + y^2 weights of eps2 are largest there);
    deeper inside it is well conditioned (<= 1e-11) and the FP32 gradient
    agrees to ~1e-3 in relative L2."""
    import json
    import os
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    gold = json.load(open(os.path.join(here, "golden", "gradient_event_128_einit.json")))
    sys.path.insert(0, os.path.join(here, "golden"))
    from make_einit_golden import directions
    w = W.gradient_event()
    assert w.name == gold["workload"] and w.steps == gold["steps"]
    print("e_init gradient 128^3 x 100, FP64 and FP32", flush=True)
    g64 = gpu_grads(w, "f64", ckpt=10)["e_init"]
    g32 = gpu_grads(w, "f32", ckpt=10)["e_init"]
    dirs = directions(w)
    for name, d in dirs.items():
        ref, refp = gold["grad"][name], gold["grad_perturbed"][name]
        bar = max(1e-9 * abs(ref), 4.0 * abs(refp - ref))
        got64, got32 = float(np.sum(g64 * d)), float(np.sum(g32 * d))
        print("direction %-8s: oracle %.12e (moves %.1e), FP64 %.12e (rel %.1e), FP32 rel %.1e" % (
            name, ref, abs(refp - ref) / abs(ref), got64, abs(got64 - ref) / abs(ref), abs(got32 - ref) / abs(ref)),
            flush=True)
        assert abs(got64 - ref) <= bar, (name, got64, ref, bar)
    nx, ny, nz = w.n
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dist = np.minimum.reduce([ix, nx - 1 - ix, iy, ny - 1 - iy, iz, nz - 1 - iz])
    inner = dist >= 16
    rel_inner = float(np.linalg.norm((g32 - g64)[inner]) / np.linalg.norm(g64[inner]))
    rel_all = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    blob = abs(float(np.sum(g32 * dirs["blob"])) - float(np.sum(g64 * dirs["blob"]))) / abs(float(np.sum(g64 * dirs["blob"])))
    print("FP32 vs FP64 e_init gradient: rel L2 everywhere %.2e, >= 16 cells from the faces %.2e, blob %.2e" % (
        rel_all, rel_inner, blob), flush=True)
    assert rel_inner <= 1e-2 and blob <= 1e-3


# --- the whole Jacobian: dot products against the oracle's forward mode ---------------------------------------------

@pytest.mark.parametrize("weno", ["z", "js", "linear"])
@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_adjoint_step_dot_product_with_oracle_jvp(weno, bc):
    """<J^T W, V> from hydro_adjoint_step against <W, J V> from the oracle's
    complex-step forward mode, J the Jacobian of three whole steps (all five
    fields, jet deposit and depletion included) at the same U0, W and V
    smooth in every field.  Both sides are exact derivatives of the discrete
    map, so they agree to rounding: bar 1e-10 of the sum of |products|."""
    from paper_1511_02137_amd import hydro as H
    steps = 3
    w = small(n=(21, 18, 16), steps=steps)
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, bc=(bc,) * 3, deposit=w.deposit, weno=weno)
    U0 = O.prim_to_cons(pb, w.prim0)
    amp = np.abs(U0).max(axis=(1, 2, 3))[:, None, None, None]
    V = np.stack([smooth_direction(pb.shape, 40 + f) for f in range(5)]) * amp
    Wt = np.stack([smooth_direction(pb.shape, 60 + f) for f in range(5)]) / amp
    _, JV = O.jvp(pb, U0, V, steps, oracle_jets(w))
    print("dot product", weno, bc, w.n, flush=True)
    h = H.from_workload(w, precision="f64", weno=weno, bc=(bc,) * 3, adjoint_k=steps)
    lam = torch.tensor(Wt, dtype=torch.float64, device="cuda")
    grad = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
    Uc = torch.tensor(U0, dtype=torch.float64, device="cuda")
    h.adjoint_step(Uc, 0, [w.jets[0].E0], steps, lam, grad)
    torch.cuda.synchronize()
    lam0 = lam.cpu().numpy()
    h.close()
    lhs = np.sum(lam0 * V)
    rhs = np.sum(Wt * JV)
    scale = np.sum(np.abs(Wt * JV))
    assert abs(lhs - rhs) <= 1e-10 * scale, (lhs, rhs, scale)
    # per field: the adjoint of each field's block row, same bar
    for f in range(5):
        Vf = np.zeros_like(V)
        Vf[f] = V[f]
        _, JVf = O.jvp(pb, U0, Vf, steps, oracle_jets(w))
        assert abs(np.sum(lam0[f] * V[f]) - np.sum(Wt * JVf)) <= 1e-10 * scale, f


@pytest.mark.parametrize("n", [(20, 300, 6), (20, 6, 300)])
def test_long_lines_dot_product_with_oracle_jvp(n):
    """Lines longer than 256 cells take the line adjoint's 1024-lane form
    (FP64: one line per workgroup, 320 lanes): the same dot-product check as
    above, two steps, WENO-Z, outflow."""
    from paper_1511_02137_amd import hydro as H
    steps = 2
    w = small(n=n, steps=steps)
    pb = O.Problem(n=w.n, dx=w.dx, t0=w.t0, dt=w.dt, bc=("outflow",) * 3, deposit=w.deposit)
    U0 = O.prim_to_cons(pb, w.prim0)
    amp = np.abs(U0).max(axis=(1, 2, 3))[:, None, None, None]
    V = np.stack([smooth_direction(pb.shape, 140 + f) for f in range(5)]) * amp
    Wt = np.stack([smooth_direction(pb.shape, 160 + f) for f in range(5)]) / amp
    _, JV = O.jvp(pb, U0, V, steps, oracle_jets(w))
    print("long lines", w.n, flush=True)
    h = H.from_workload(w, precision="f64", adjoint_k=steps)
    lam = torch.tensor(Wt, dtype=torch.float64, device="cuda")
    grad = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
    h.adjoint_step(torch.tensor(U0, dtype=torch.float64, device="cuda"), 0, [w.jets[0].E0], steps, lam, grad)
    torch.cuda.synchronize()
    lam0 = lam.cpu().numpy()
    h.close()
    lhs, rhs, scale = np.sum(lam0 * V), np.sum(Wt * JV), np.sum(np.abs(Wt * JV))
    print("lhs %.15e rhs %.15e rel %.2e" % (lhs, rhs, abs(lhs - rhs) / scale), flush=True)
    assert abs(lhs - rhs) <= 1e-10 * scale, (lhs, rhs, scale)


def test_long_lines_fp32_lines_per_workgroup_bitwise():
    """FP32 z lines of 300 cells: one and two lines per workgroup (320 and
    640 lanes, the 1024-lane form) give the same bits."""
    from paper_1511_02137_amd import hydro as H
    steps = 2
    w = small(n=(20, 6, 300), steps=steps)
    pb = oracle_problem(w)
    U0 = torch.tensor(O.prim_to_cons(pb, w.prim0), dtype=torch.float32, device="cuda")
    Wt = np.stack([smooth_direction(pb.shape, 180 + f) for f in range(5)])
    outs = []
    for lines in (1, 2):
        h = H.from_workload(w, precision="f32", adjoint_k=steps)
        h.set_option(H.OPT_ADJ_LINES, lines)
        lam = torch.tensor(Wt, dtype=torch.float32, device="cuda")
        grad = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
        h.adjoint_step(U0, 0, [w.jets[0].E0], steps, lam, grad)
        torch.cuda.synchronize()
        outs.append((lam.cpu().numpy(), grad.cpu().numpy()))
        h.close()
    assert np.any(outs[0][0])
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_skip_n_option_is_exact_for_zero_n_adjoint():
    """HYDRO_OPT_ADJ_SKIP_N: with lambda_N = 0 on entry the skipping sweep
    returns the general sweep's result (values equal, N component zero); with
    lambda_N != 0 it returns the general sweep of lambda with N zeroed."""
    from paper_1511_02137_amd import hydro as H
    steps = 2
    w = small(n=(21, 18, 16), steps=steps)
    pb = oracle_problem(w)
    U0 = torch.tensor(O.prim_to_cons(pb, w.prim0), dtype=torch.float64, device="cuda")
    Wt = np.stack([smooth_direction(pb.shape, 80 + f) for f in range(5)])
    outs = {}
    for skip in (0, 1):
        for zero_n in (True, False):
            h = H.from_workload(w, precision="f64", adjoint_k=steps)
            h.set_option(H.OPT_ADJ_SKIP_N, skip)
            assert h.get_option(H.OPT_ADJ_SKIP_N) == skip
            lam = torch.tensor(Wt, dtype=torch.float64, device="cuda")
            if zero_n:
                lam[4] = 0
            grad = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
            h.adjoint_step(U0, 0, [w.jets[0].E0], steps, lam, grad)
            torch.cuda.synchronize()
            outs[skip, zero_n] = (lam.cpu().numpy(), grad.cpu().numpy())
            h.close()
    for k in range(2):
        assert np.array_equal(outs[1, True][k], outs[0, True][k])
        assert np.array_equal(outs[1, False][k], outs[0, True][k])
    assert not np.any(outs[1, True][0][4])
    assert np.any(outs[0, False][0][4])
    with pytest.raises(H.HydroError):
        h = H.from_workload(w, precision="f64")
        try:
            h.set_option(H.OPT_ADJ_SKIP_N, 2)
        finally:
            h.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_adjoint_lines_per_workgroup_bitwise(precision, bc):
    """HYDRO_OPT_ADJ_LINES: the y and z line adjoints with 1, 2 or 4
    neighbouring lines per workgroup return the same bits (lambda and the
    parameter gradients), here with n_x = 20 (a multiple of 4) and ragged
    y/z extents; an unsupported value is refused."""
    from paper_1511_02137_amd import hydro as H
    steps = 2
    w = small(n=(20, 18, 13), steps=steps)
    pb = oracle_problem(w)
    dt = torch.float64 if precision == "f64" else torch.float32
    U0 = torch.tensor(O.prim_to_cons(pb, w.prim0), dtype=dt, device="cuda")
    Wt = np.stack([smooth_direction(pb.shape, 90 + f) for f in range(5)])
    outs = []
    for lines in (1, 2, 4, 0):
        h = H.from_workload(w, precision=precision, bc=(bc,) * 3, adjoint_k=steps)
        h.set_option(H.OPT_ADJ_LINES, lines)
        assert h.get_option(H.OPT_ADJ_LINES) == lines
        lam = torch.tensor(Wt, dtype=dt, device="cuda")
        grad = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
        h.adjoint_step(U0, 0, [w.jets[0].E0], steps, lam, grad)
        torch.cuda.synchronize()
        outs.append((lam.cpu().numpy(), grad.cpu().numpy()))
        h.close()
    assert np.any(outs[0][0]) and np.any(outs[0][1])
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0])
        assert np.array_equal(o[1], outs[0][1])
    h = H.from_workload(w, precision=precision)
    try:
        with pytest.raises(H.HydroError):
            h.set_option(H.OPT_ADJ_LINES, 3)
    finally:
        h.close()


def test_torch_gradcheck_small():
    """torch.autograd.gradcheck (fast mode: random projections of the Jacobian
    against central differences of the GPU forward, eps 1e-6) of the
    differentiable eps2 at 16^3, 3 steps."""
    A = adjoint_mod()
    w = small(n=(16, 16, 16), steps=3)
    w.jets[0].x0 = (-0.4345, 0.031, 0.013)
    pb = A.Eps2Problem(w, ckpt_every=2)
    j = w.jets[0]
    e0 = torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda", requires_grad=True)
    kr = torch.tensor(j.kappa_rad, dtype=torch.float64, requires_grad=True)
    kc = torch.tensor(j.kappa_coll, dtype=torch.float64, requires_grad=True)
    xy = torch.tensor(j.x0[:2], dtype=torch.float64, requires_grad=True)
    ok = torch.autograd.gradcheck(lambda a, b, c, d: A.eps2(a, b, c, d, pb), (e0, kr, kc, xy), eps=1e-6,
                                  atol=1e-9, rtol=1e-4, fast_mode=True)
    assert ok
    pb.h.close()


def test_backward_after_another_forward_uses_its_own_parameters():
    """Two differentiable forwards at different jet parameters on one problem,
    then the backward of the first: it must re-apply the first forward's
    kappas and origin before recomputing its stage states, so its gradients
    equal those of a lone forward + backward at those parameters (bitwise:
    the same kernels on the same inputs)."""
    A = adjoint_mod()
    w = small(n=(16, 16, 16), steps=3)
    pb = A.Eps2Problem(w, ckpt_every=2)
    j = w.jets[0]
    e0 = torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda", requires_grad=True)

    def leaf(v):
        return torch.tensor(v, dtype=torch.float64, requires_grad=True)

    pa = (leaf(j.kappa_rad), leaf(j.kappa_coll), leaf(list(j.x0[:2])))
    pbb = (leaf(2.0 * j.kappa_rad), leaf(0.5 * j.kappa_coll), leaf([j.x0[0] + 0.07, j.x0[1] - 0.05]))
    ea = A.eps2(e0, *pa, pb)
    eb = A.eps2(e0, *pbb, pb)
    assert float(ea) != float(eb)
    ga = torch.autograd.grad(ea, [e0, *pa])
    # the lone run at the first parameters
    e1 = torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda", requires_grad=True)
    p1 = (leaf(j.kappa_rad), leaf(j.kappa_coll), leaf(list(j.x0[:2])))
    e_alone = A.eps2(e1, *p1, pb)
    g1 = torch.autograd.grad(e_alone, [e1, *p1])
    assert float(e_alone) == float(ea)
    for a, b in zip(ga, g1):
        assert torch.equal(a.cpu(), b.cpu())
    pb.h.close()


def test_adjoint_sweep_leaves_the_fixup_count_alone():
    """The reverse sweep recomputes the segment's stages and recovers
    primitives in its own kernels; none of that may add to the run's fix-up
    count (hydro_diag), here with a non-admissible cell in the checkpoint so
    that the recomputation does go through the fix-up branch."""
    from paper_1511_02137_amd import hydro as H
    w = small(n=(16, 16, 16), steps=2)
    h = H.from_workload(w, adjoint_k=2)
    h.U[0, 8, 8, 8] = -1.0
    U0 = h.U.clone()
    _, step0, E0 = h.get_state()
    h.step(2)
    f = h.fixups()
    assert f > 0
    lam = torch.empty_like(h.U)
    h.loss_eps2(h.U, seed=lam)
    grad = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
    h.adjoint_step(U0, step0, E0, 2, lam, grad)
    torch.cuda.synchronize()
    assert h.fixups() == f
    h.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("deposit", ["gauss", "ngp"])
def test_recorded_stage_states_give_the_checkpointed_gradients(precision, deposit):
    """hydro_rk3_step_record + hydro_adjoint_recorded (stage states kept
    from the forward, no recompute) against checkpoints every 2 steps: eps2,
    the initial-field and jet gradients bit for bit."""
    w = small(steps=5, deposit=deposit)
    print("recorded", precision, deposit, w.n, w.steps, flush=True)
    a = gpu_grads(w, precision=precision, ckpt=2)
    b = gpu_grads(w, precision=precision, record=True)
    assert b["eps2"] == a["eps2"]
    assert np.array_equal(b["jets"], a["jets"])
    assert np.array_equal(b["e_init"], a["e_init"])


def test_recorded_steps_equal_plain_steps_and_their_record_lifetime():
    """The recording forward advances U, the step sums, the jet energies and
    the ledger exactly as hydro_rk3_step; the record serves repeated sweeps
    (the same result each time) and is discarded by hydro_set_jet,
    hydro_reset, hydro_set_state and hydro_adjoint_step (HYDRO_ESTATE
    after); a sweep leaves U, step, jet energies, ledger and fix-up count
    alone; more steps than the workspace holds is HYDRO_EINVAL."""
    from paper_1511_02137_amd import hydro as H
    w = small(n=(16, 16, 16), steps=3)
    a = H.from_workload(w, adjoint_k=3)
    b = H.from_workload(w)
    a.step_record(3)
    b.step(3)
    torch.cuda.synchronize()
    assert torch.equal(a.U, b.U)
    assert np.array_equal(a.step_sums(), b.step_sums())
    sa, sb = a.get_state(), b.get_state()
    assert sa[0] == sb[0] and sa[1] == sb[1] and np.array_equal(sa[2], sb[2])
    assert a.sums()[5] == b.sums()[5]
    U_end, state_end, f_end = a.U.clone(), a.get_state(), a.fixups()
    lam0 = torch.empty_like(a.U)
    a.loss_eps2(a.U, seed=lam0)
    res = []
    for _ in range(2):
        lam = lam0.clone()
        grad = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
        a.adjoint_recorded(lam, grad)
        torch.cuda.synchronize()
        res.append((lam, grad))
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])
    assert torch.equal(a.U, U_end) and a.fixups() == f_end
    st = a.get_state()
    assert st[0] == state_end[0] and st[1] == state_end[1] and np.array_equal(st[2], state_end[2])
    j = w.jets[0]
    grad = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
    for discard in (lambda: a.set_jet(0, j.x0, j.dir, j.E0, j.t_start, j.kappa_rad, j.kappa_coll, j.cr_over_cf),
                    lambda: a.reset(torch.from_numpy(w.prim0)),
                    lambda: a.set_state(*a.get_state()[1:], 0.0),
                    lambda: a.adjoint_step(U_end, 0, [j.E0], 1, lam0.clone(), grad)):
        a.step_record(2)
        discard()
        with pytest.raises(H.HydroError) as ei:
            a.adjoint_recorded(lam0.clone(), grad)
        assert ei.value.code == H.HYDRO_ESTATE
    with pytest.raises(H.HydroError) as ei:
        a.step_record(4)
    assert ei.value.code == H.HYDRO_EINVAL
    a.close()
    b.close()


def test_recorded_problem_refuses_a_backward_after_another_forward():
    """With the stage states kept from the forward, a backward belongs to the
    latest forward: an earlier one's backward is refused, not silently
    differentiated through the later run's states."""
    A = adjoint_mod()
    w = small(n=(16, 16, 16), steps=3)
    pb = A.Eps2Problem(w, record=True)
    j = w.jets[0]
    e0 = torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda")
    fa = pb.forward(e0, j.kappa_rad, j.kappa_coll, j.x0[0], j.x0[1])
    fb = pb.forward(e0, 2.0 * j.kappa_rad, j.kappa_coll, j.x0[0], j.x0[1])
    with pytest.raises(RuntimeError):
        pb.backward(fa[1], fa[2], fa[3])
    pb.backward(fb[1], fb[2], fb[3])
    pb.h.close()


def test_recorded_problem_under_autograd():
    """eps2(...) through torch.autograd with the stage states kept from the
    forward: the value and every gradient equal those of the checkpointed
    problem bit for bit."""
    A = adjoint_mod()
    w = small(n=(16, 16, 16), steps=3)
    j = w.jets[0]

    def run(pb):
        e0 = torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda", requires_grad=True)
        p = [torch.tensor(v, dtype=torch.float64, requires_grad=True)
             for v in (j.kappa_rad, j.kappa_coll, list(j.x0[:2]))]
        e = A.eps2(e0, *p, pb)
        g = torch.autograd.grad(e, [e0, *p])
        pb.h.close()
        return float(e), g

    ec, gc = run(A.Eps2Problem(w, ckpt_every=2))
    er, gr = run(A.Eps2Problem(w, record=True))
    assert er == ec
    for a, b in zip(gr, gc):
        assert torch.equal(a.cpu(), b.cpu())


def test_checkpointed_backward_with_and_without_the_kept_last_segment():
    """The checkpointed forward keeps its last segment's stage states; the
    first backward sweeps that segment from them, a second backward of the
    same forward (the record overwritten by the first one's recomputes)
    recomputes every segment: the same gradients bit for bit."""
    A = adjoint_mod()
    w = small(steps=5)
    pb = A.Eps2Problem(w, ckpt_every=2)
    j = w.jets[0]
    e0 = torch.tensor(w.prim0[0], dtype=torch.float64, device="cuda")
    eps, cks, Uf, prim = pb.forward(e0, j.kappa_rad, j.kappa_coll, j.x0[0], j.x0[1])
    assert [c.recorded != 0 for c in cks] == [False, False, True]
    g1 = pb.backward(cks, Uf, prim)
    assert pb._live == 0
    g2 = pb.backward(cks, Uf, prim)
    torch.cuda.synchronize()
    assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1], g2[1])
    pb.h.close()
