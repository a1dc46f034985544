"""GPU parity of the grid energies (Poisson image editing, optical flow, ARAP
warp) against the FP64 oracle, through the C ABI.

Tolerances: FP64 operator products (J^T F, diag, J^T J p) agree to 1e-12 of
their largest entry; FP64 PCG iterates to 1e-9 (or 100x the oracle's own spread
between two valid evaluation orders, never above 1e-6: cases where CG has lost
orthogonality are not compared); FP64 GN and
LM cost traces to 1e-9 relative; mixed precision to 1e-4 relative final cost.
Sizes span several 64 x 16 tiles and end in ragged partial tiles.
"""
import numpy as np
import pytest

import oracle as o
import workloads as w
from tests.gpu_util import pcg_tol, f32_inputs, make_problem, relmax, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _poisson(W, H, seed=5):
    d = w.poisson_edit(W, H, seed=seed)
    rng = np.random.default_rng(seed)
    act = d["mask"] == 0
    x = np.where(act[None], d["x0"] + 0.1 * rng.normal(size=d["x0"].shape), d["x0"])
    return d, x


def _flow(W, H, seed=4):
    d = w.optical_flow(W, H, seed=seed)
    rng = np.random.default_rng(seed)
    x = d["flow_true"] * 0.7 + 0.3 * rng.normal(size=d["x0"].shape)
    return d, x


def _warp(W, H, seed=3):
    d = w.arap_warp(W, H, seed=seed, n_constraints=max(2, W * H // 64), margin=2, mask="random")
    rng = np.random.default_rng(seed)
    x = d["x0"] + np.concatenate([rng.normal(0, 0.5, (2, H, W)), rng.normal(0, 0.2, (1, H, W))])
    return d, np.where((d["mask"] == 0)[None], x, d["x0"])


# Shape-from-shading cases use distinct focal lengths and centre coordinates and
# nine distinct non-zero lighting coefficients, so that a swapped intrinsic, a
# swapped normal component or a wrong lighting derivative changes the result.
SFS_LIGHT = (0.5, 0.07, -0.3, 0.04, 0.03, -0.02, 0.05, 0.06, -0.04)


def _sfs_general(W, H, seed=2, **kw):
    return w.shape_from_shading(W, H, seed=seed, focal=(0.95 * W, 1.1 * W),
                                center=((W - 1) / 2 + 1.3, (H - 1) / 2 - 0.7), lighting=SFS_LIGHT, **kw)


def _sfs(W, H, seed=2):
    d = _sfs_general(W, H, seed=seed, invalid="hole" if W > 20 else "none", edge_zero_frac=0.1)
    rng = np.random.default_rng(seed)
    x = d["x0"] + 1e-4 * rng.normal(size=d["x0"].shape)
    return d, np.where((d["D"] > 0)[None], x, d["x0"])


MAKERS = {"poisson": _poisson, "flow": _flow, "warp": _warp, "sfs": _sfs}
SIZES = [(9, 7), (97, 41), (130, 70)]
CASES = [(k, W, H) for k in MAKERS for (W, H) in SIZES]


@pytest.mark.parametrize("kind,W,H", CASES)
def test_operators_fp64(kind, W, H):
    d, x = MAKERS[kind](W, H)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    assert abs(prob.cost(xt) - lin.E) <= 1e-12 * lin.E
    assert abs(prob.linearize(xt) - lin.E) <= 1e-12 * lin.E
    b, dg = prob.eval_jtf()
    assert relmax(to_np(b), lin.jtf()) < 1e-12
    assert relmax(to_np(dg), lin.diag) < 1e-12
    rng = np.random.default_rng(1)
    p = rng.normal(size=lin.diag.size) * lin.active
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p))), lin.apply(p)) < 1e-12
    D = lin.damping()
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p), lam=0.21)), lin.apply(p, 0.21, D)) < 1e-12


@pytest.mark.parametrize("kind,W,H", CASES)
@pytest.mark.parametrize("variant", ["fused", "split"])
def test_pcg_fp64(kind, W, H, variant):
    d, x = MAKERS[kind](W, H)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    prob.linearize(xt)
    A = (lin.JT @ lin.J).tocsr()
    for precond in (True, False):
        # without the preconditioner the 9 x 7 grids lose orthogonality past
        # about 15 iterations (iterates then depend on rounding order)
        Ls = (1, 9, 30) if (precond or W * H > 100) else (1, 9, 12)
        for L in Ls:
            ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(precond), L)
            ref2, _ = o.pcg(lambda v: A @ v, lin.jtf(), lin.minv(precond), L)
            tol = pcg_tol(ref, ref2)
            got = to_np(prob.pcg(L, use_precond=precond, variant=variant))
            assert relmax(got, ref) < tol, (precond, L, tol)


@pytest.mark.parametrize("kind", list(MAKERS))
@pytest.mark.parametrize("variant", ["fused", "split"])
def test_gn_fp64(kind, variant):
    d, _ = MAKERS[kind](97, 41)
    e = o.make_energy(d)
    xo, costs = o.gauss_newton(e, d["x0"], 3, 15)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=3, pcg_iters=15, pcg_variant=variant)
    assert np.allclose(rep["cost_trace"], costs, rtol=1e-9, atol=0)
    assert relmax(to_np(xt) - d["x0"].ravel(), xo - d["x0"].ravel()) < 1e-8


@pytest.mark.parametrize("kind", list(MAKERS))
def test_gn_mixed(kind):
    K = 4
    if kind == "sfs":
        d = _sfs_general(130, 70)
    else:
        d, _ = MAKERS[kind](130, 70)
    e = o.make_energy(d)
    xo, costs = o.gauss_newton(e, d["x0"], K, 20)
    if kind == "sfs":
        # The smoothness residuals of shape from shading are switched on and off
        # by a threshold (0.01) on neighbouring depth differences (Fig. 26),
        # evaluated at each linearisation point.  FP32 and FP64 iterates select
        # the same residuals only if no difference that enters the test lies
        # near the threshold: checked at every outer iteration of the oracle.
        assert sfs_mask_margin(e, d["x0"], K, 20) > 1e-4
    prob = make_problem(d, "mixed")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=K, pcg_iters=20)
    assert abs(rep["cost_final"] - costs[-1]) <= 1e-4 * costs[-1]


def sfs_mask_margin(e, x0, K, L):
    """Smallest distance to the 0.01 threshold of a neighbouring depth
    difference that enters the smoothness test, over the K linearisation points
    of the oracle's GN K x L from x0."""
    x = np.asarray(x0, float).ravel().copy()
    worst = np.inf
    for _ in range(K):
        X = x.reshape(e.H, e.W)
        c = X[1:-1, 1:-1]
        for nb in (X[1:-1, 2:], X[1:-1, :-2], X[2:, 1:-1], X[:-2, 1:-1]):
            worst = min(worst, float(np.min(np.abs(np.abs(c - nb) - 0.01))))
        lin = o.Linearization(e, x)
        delta, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), L)
        x = x + delta
    return worst


# FP32 operator tolerances (relative to the largest entry): a product sums a few
# dozen FP32 terms (unit roundoff 6e-8); shape from shading forms its shading
# derivatives from depth differences about 300x smaller than the depth itself,
# which costs that factor in relative accuracy.
MIXED_OP_TOL = {"poisson": 1e-5, "flow": 1e-5, "warp": 1e-5, "sfs": 1e-3}


@pytest.mark.parametrize("kind", list(MAKERS))
def test_operators_mixed(kind):
    """Mixed precision: the FP64 cost of FP32 values is exact, and the FP32
    products agree with the FP64 oracle on the same FP32-rounded inputs."""
    d, x = MAKERS[kind](97, 41)
    d32 = f32_inputs(d)
    x32 = np.asarray(x, np.float32).astype(np.float64)
    e = o.make_energy(d32)
    lin = o.Linearization(e, x32)
    prob = make_problem(d, "mixed")
    xt = to_dev(prob, x32)
    assert abs(prob.cost(xt) - lin.E) <= 1e-12 * lin.E
    assert abs(prob.linearize(xt) - lin.E) <= 1e-12 * lin.E
    tol = MIXED_OP_TOL[kind]
    b, dg = prob.eval_jtf()
    errs = [relmax(to_np(b), lin.jtf()), relmax(to_np(dg), lin.diag)]
    p = np.random.default_rng(1).normal(size=lin.diag.size) * lin.active
    p32 = np.asarray(p, np.float32).astype(np.float64)
    errs.append(relmax(to_np(prob.apply_jtj(to_dev(prob, p32))), lin.apply(p32)))
    print(kind, "mixed operator errors", errs)
    assert max(errs) < tol


@pytest.mark.parametrize("kind", list(MAKERS))
def test_lm_fp64(kind):
    d, _ = MAKERS[kind](97, 41)
    e = o.make_energy(d)
    xo, costs, acc = o.levenberg_marquardt(e, d["x0"], 4, 12)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="lm", outer_iters=4, pcg_iters=12)
    assert rep["steps_accepted"] == sum(acc)
    assert np.allclose(rep["cost_trace"][:len(costs)], costs, rtol=1e-9, atol=0)


def test_poisson_one_step_exact():
    """GN reaches the minimiser of the linear Poisson energy in one outer
    iteration given an (effectively) exact inner solve (Sec. 8.1): a second
    iteration no longer lowers the cost."""
    d = w.poisson_edit(40, 24, seed=7)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=2, pcg_iters=400)
    e = o.make_energy(d)
    xo, costs = o.gauss_newton(e, d["x0"], 1, 400)
    assert abs(rep["cost_trace"][1] - costs[1]) <= 1e-10 * costs[1]
    assert abs(rep["cost_trace"][2] - rep["cost_trace"][1]) <= 1e-10 * rep["cost_trace"][1]


@pytest.mark.parametrize("tuning", [dict(strip_rows=1), dict(strip_rows=5), dict(strip_rows=300),
                                    dict(waves_per_simd=1), dict(waves_per_simd=3)])
def test_sfs_fused_launch_shapes(tuning):
    """The shape-from-shading fused kernel walks strips of 58 columns with 3
    halo rows above and 2 below: every strip partition (one-row strips, strips
    taller than the grid, ragged last strips) gives the oracle's PCG iterates,
    plain and with LM damping."""
    d, x = _sfs(190, 83)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    prob.set_tuning(**tuning)
    xt = to_dev(prob, x)
    prob.linearize(xt)
    JTJ = (lin.JT @ lin.J).tocsr()
    for lam in (0.0, 0.3):
        D = lin.damping() if lam else np.zeros(lin.diag.size)
        Mi = lin.minv(True, lam, D) if lam else lin.minv(True)
        ref, _ = o.pcg(lambda v: lin.apply(v, lam, D) if lam else lin.apply(v), lin.jtf(), Mi, 14)
        # the oracle's own spread between two evaluation orders bounds what can agree
        ref2, _ = o.pcg(lambda v: JTJ @ v + lam * D * v, lin.jtf(), Mi, 14)
        tol = pcg_tol(ref, ref2)
        got = to_np(prob.pcg(14, lam=lam, variant="fused"))
        assert relmax(got, ref) < tol, (tuning, lam, tol)


@pytest.mark.parametrize("kind", ["poisson", "flow", "warp"])
@pytest.mark.parametrize("rows", [1, 2, 3])
def test_short_strips(kind, rows):
    """The one- to three-row strips the tuning table gives small grids: FP64
    PCG iterates match the oracle's (1e-9, as every launch shape), and a mixed
    precision GN 4 x 20 in those strips reaches the oracle's cost within the
    mixed-precision bar of 1e-4 (as test_gn_mixed in the library's own shape)."""
    d, x = MAKERS[kind](130, 70)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), 20)
    prob = make_problem(d, "fp64", tuning=None)
    prob.set_tuning(strip_rows=rows)
    assert prob.get_tuning()["strip_rows"] == rows
    prob.linearize(to_dev(prob, x))
    assert relmax(to_np(prob.pcg(20, variant="fused")), ref) < 1e-9
    _, costs = o.gauss_newton(e, d["x0"], 4, 20)
    p32 = make_problem(d, "mixed", tuning=None)
    p32.set_tuning(strip_rows=rows)
    rep = p32.solve(to_dev(p32, d["x0"]), method="gn", outer_iters=4, pcg_iters=20)
    assert abs(rep["cost_final"] - costs[-1]) <= 1e-4 * costs[-1]
