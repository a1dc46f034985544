"""GPU parity of the ARAP image-warping path against the FP64 oracle.

Every comparison calls through the C ABI (libopt.so) and checks element by
element against the oracle on the same seeded inputs.  FP64 operator products
must agree to 1e-12 of their largest entry (rounding order only); FP64 solves to
1e-9 relative cost; the mixed-precision path (FP32 bulk, FP64 reductions) to
1e-4 relative final cost.
"""
import numpy as np
import pytest

import oracle as o
import workloads as w
from tests.gpu_util import f32_inputs, make_problem, pcg_tol, relmax, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8, "none"), (37, 29, "random"), (70, 65, "hole")]


def _case(W, H, mask, seed=3):
    d = w.arap_warp(W, H, seed=seed, n_constraints=max(2, W * H // 64), margin=2, mask=mask)
    rng = np.random.default_rng(seed)
    x = d["x0"] + np.concatenate([rng.normal(0, 0.5, (2, H, W)), rng.normal(0, 0.2, (1, H, W))])
    act = (d["mask"] == 0)
    x = np.where(act[None], x, d["x0"])
    return d, x


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("W,H,mask", SHAPES)
def test_cost_linearize_jtf_diag(W, H, mask):
    d, x = _case(W, H, mask)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    assert abs(prob.cost(xt) - lin.E) <= 1e-12 * lin.E
    assert abs(prob.linearize(xt) - lin.E) <= 1e-12 * lin.E
    b, dg = prob.eval_jtf()
    assert relmax(to_np(b), lin.jtf()) < 1e-12
    assert relmax(to_np(dg), lin.diag) < 1e-12


@pytest.mark.parametrize("W,H,mask", SHAPES)
def test_jtjp_random(W, H, mask):
    d, x = _case(W, H, mask)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    prob.linearize(to_dev(prob, x))
    rng = np.random.default_rng(7)
    p = rng.normal(size=lin.diag.size) * lin.active
    q = to_np(prob.apply_jtj(to_dev(prob, p)))
    assert relmax(q, lin.apply(p)) < 1e-12
    D = lin.damping()
    q2 = to_np(prob.apply_jtj(to_dev(prob, p), lam=0.37))
    assert relmax(q2, lin.apply(p, 0.37, D)) < 1e-12


def test_dense_jtj_8x8():
    """The matrix-free product applied to every unit vector reproduces the dense
    J^T J of the oracle's explicit Jacobian."""
    d, x = _case(8, 8, "random", seed=5)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    A = (lin.J.T @ lin.J).toarray()
    prob = make_problem(d, "fp64")
    prob.linearize(to_dev(prob, x))
    N = A.shape[0]
    cols = []
    for k in range(N):
        ek = np.zeros(N)
        ek[k] = 1.0
        cols.append(to_np(prob.apply_jtj(to_dev(prob, ek))))
    G = np.stack(cols, 1)
    act = lin.active
    assert np.abs(G - A)[np.ix_(act, act)].max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("W,H,mask", SHAPES)
@pytest.mark.parametrize("precond", [True, False])
@pytest.mark.parametrize("variant", ["fused", "split"])
def test_pcg(W, H, mask, precond, variant):
    d, x = _case(W, H, mask)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    prob.linearize(xt)
    A = (lin.JT @ lin.J).tocsr()
    # odd and even counts end d's paired updates both ways; without the
    # preconditioner the 8 x 8 lattice loses orthogonality past about 20
    # iterations (its iterates then depend on rounding order), so it stops at 15
    Ls = (1, 7, 8, 25) if (precond or W * H > 100) else (1, 7, 8, 15)
    for L in Ls:
        ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(precond), L)
        ref2, _ = o.pcg(lambda v: A @ v, lin.jtf(), lin.minv(precond), L)
        tol = pcg_tol(ref, ref2)
        got = to_np(prob.pcg(L, use_precond=precond, variant=variant))
        assert relmax(got, ref) < tol, (L, tol)


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_gn_config1_fp64(variant):
    """ARAP warp 64x64, FP64, GN 5 x 20, Jacobi: the parity configuration."""
    d = w.arap_warp(64, 64, seed=1)
    e = o.make_energy(d)
    xo, costs = o.gauss_newton(e, d["x0"], 5, 20)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=5, pcg_iters=20, pcg_variant=variant)
    assert np.allclose(rep["cost_trace"], costs, rtol=1e-9, atol=0)
    assert relmax(to_np(xt) - d["x0"].ravel(), xo - d["x0"].ravel()) < 1e-8


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_gn_mixed_precision(variant):
    d = w.arap_warp(64, 64, seed=1)
    e = o.make_energy(d)
    xo, costs = o.gauss_newton(e, d["x0"], 5, 20)
    prob = make_problem(d, "mixed")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=5, pcg_iters=20, pcg_variant=variant)
    assert abs(rep["cost_final"] - costs[-1]) <= 1e-4 * costs[-1]
    assert relmax(to_np(xt) - d["x0"].ravel(), xo - d["x0"].ravel()) < 1e-3


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_lm_fp64(variant):
    d = w.arap_warp(40, 33, seed=4, n_constraints=12, sigma=4.0, margin=3, mask="random")
    e = o.make_energy(d)
    xo, costs, acc = o.levenberg_marquardt(e, d["x0"], 6, 15)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="lm", outer_iters=6, pcg_iters=15, pcg_variant=variant)
    assert rep["steps_accepted"] == sum(acc)
    assert np.allclose(rep["cost_trace"][:len(costs)], costs, rtol=1e-9, atol=0)
    assert relmax(to_np(xt) - d["x0"].ravel(), xo - d["x0"].ravel()) < 1e-8


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_deterministic(variant):
    d = w.arap_warp(150, 130, seed=2, mask="hole")
    outs = []
    for _ in range(2):
        prob = make_problem(d, "mixed")
        xt = to_dev(prob, d["x0"])
        rep = prob.solve(xt, method="gn", outer_iters=3, pcg_iters=10, pcg_variant=variant)
        outs.append((rep["cost_trace"], to_np(xt)))
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1])


def test_excluded_unknowns_unchanged():
    d = w.arap_warp(37, 29, seed=3, mask="random")
    prob = make_problem(d, "mixed")
    xt = to_dev(prob, d["x0"])
    prob.solve(xt, method="gn", outer_iters=2, pcg_iters=10)
    x = to_np(xt).reshape(3, -1)
    ex = (d["mask"] != 0).ravel()
    assert np.array_equal(x[:, ex], d["x0"].reshape(3, -1)[:, ex].astype(np.float32))


def test_lm_damped_pcg_matches_oracle():
    d, x = _case(70, 65, "hole")
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    prob.linearize(xt)
    lam = 0.3
    D = lin.damping()
    ref, _ = o.pcg(lambda v: lin.apply(v, lam, D), lin.jtf(), lin.minv(True, lam, D), 12)
    for variant in ("fused", "split"):
        got = to_np(prob.pcg(12, lam=lam, variant=variant))
        assert relmax(got, ref) < 1e-9, variant


def test_full_size_operators_mixed():
    """1024 x 1024 (the benchmark size): J^T F, diag and J^T J p in FP32 against
    the FP64 oracle, and one GN iteration of 10 PCG steps."""
    d = w.arap_warp(1024, 1024, seed=2)
    e = o.make_energy(d)
    rng = np.random.default_rng(0)
    x = d["x0"] + np.concatenate([rng.normal(0, 0.3, (2, 1024, 1024)), rng.normal(0, 0.05, (1, 1024, 1024))])
    lin = o.Linearization(e, x)
    prob = make_problem(d, "mixed")
    xt = to_dev(prob, x)
    assert abs(prob.linearize(xt) - lin.E) <= 1e-6 * lin.E
    b, dg = prob.eval_jtf()
    assert relmax(to_np(b), lin.jtf()) < 1e-5
    assert relmax(to_np(dg), lin.diag) < 1e-6
    p = rng.normal(size=lin.diag.size)
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p))), lin.apply(p)) < 1e-5
    xo, costs = o.gauss_newton(e, d["x0"], 1, 10)
    x0t = to_dev(prob, d["x0"])
    rep = prob.solve(x0t, method="gn", outer_iters=1, pcg_iters=10)
    assert abs(rep["cost_final"] - costs[-1]) <= 1e-4 * costs[-1]


def test_zero_iterations_and_tiny_grid():
    d = w.arap_warp(1, 1, seed=1, n_constraints=1, margin=0)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=0, pcg_iters=0)
    assert rep["cost_final"] == o.cost(o.make_energy(d), d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=2, pcg_iters=3)
    xo, costs = o.gauss_newton(o.make_energy(d), d["x0"], 2, 3)
    assert np.allclose(rep["cost_trace"], costs, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("tuning", [dict(strip_rows=1), dict(strip_rows=2), dict(strip_rows=4), dict(strip_rows=7),
                                    dict(strip_rows=200),
                                    dict(waves_per_simd=1), dict(waves_per_simd=3)])
def test_launch_shapes_agree(tuning):
    """Every strip partition of the fused kernel gives the oracle's PCG iterates
    (strips walk in alternating directions and end in ragged partial strips)."""
    d, x = _case(130, 97, "random")
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), 20)
    prob = make_problem(d, "fp64")
    prob.set_tuning(**tuning)
    t = prob.get_tuning()
    assert t["strip_rows"] >= 1 and t["waves_per_simd"] >= 1
    if tuning.get("strip_rows"):
        assert t["strip_rows"] == min(tuning["strip_rows"], 97)
    xt = to_dev(prob, x)
    prob.linearize(xt)
    got = to_np(prob.pcg(20, variant="fused"))
    assert relmax(got, ref) < 1e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("pcg_iters", [1, 2, 3, 6])
def test_pcg_exact_stop_keeps_last_update(precision, pcg_iters):
    """Isolated active pixels with fit terms only: J^T J is w_fit I on their
    positions (the angles have no term), so Jacobi-PCG reaches the exact Newton
    step after one iteration, and with dyadic data every product and sum is
    exact.  The second iteration then finds gamma = delta = 0 and stops; the
    step of the first iteration must still reach d, so one GN iteration puts
    every constrained pixel on its target (cost 0), as the oracle does."""
    W, H = 18, 14
    d = w.arap_warp(W, H, seed=1, n_constraints=1, margin=0, w_fit=4.0, w_reg=1.0)
    i, j = np.meshgrid(np.arange(W), np.arange(H))
    act = (i % 2 == 0) & (j % 2 == 0)
    d["mask"] = np.where(act, 0, 1).astype(np.uint8)
    rng = np.random.default_rng(4)
    C = -np.ones((2, H, W))
    tgt = act & (rng.random((H, W)) < 0.7)
    off = rng.integers(0, 4, size=(2, H, W)).astype(np.float64)
    C[:, tgt] = d["U"][:, tgt] + off[:, tgt]
    d["C"] = C
    e = o.make_energy(d)
    xo, costs = o.gauss_newton(e, d["x0"], 1, pcg_iters)
    assert costs[-1] == 0.0 and costs[0] > 0.0
    prob = make_problem(d, precision)
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=1, pcg_iters=pcg_iters)
    assert rep["cost_trace"][0] == costs[0]
    assert rep["cost_final"] == 0.0
    assert np.array_equal(to_np(xt).reshape(3, H, W), np.asarray(xo).reshape(3, H, W))


def test_fused_beyond_256mb_vectors_matches_split():
    """FP64 warp on 3400 x 3400 sites: each internal vector is 277 MB and the
    state 370 MB, past the 2^28-byte offsets of a whole-vector raw buffer, so
    the fused form runs its instantiation with buffers based at each strip's
    first row.  Its PCG iterates must equal the split (textbook) form's, which
    is parity-tested against the oracle at smaller sizes, to the FP64
    tolerance."""
    d = w.arap_warp(3400, 3400, seed=12)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    prob.linearize(xt)
    fused = to_np(prob.pcg(12, variant="fused"))
    split = to_np(prob.pcg(12, variant="split"))
    assert relmax(fused, split) < 1e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_large_grid_form_matches_oracle(precision, lam):
    """The fused kernel's large-grid form (every buffer based at the strip's
    first row; in FP32 held to two waves per SIMD, with register spills), forced
    on a small grid, gives the oracle's PCG iterates, undamped and with LM
    damping, for odd and even iteration counts.  FP64 to the PCG tolerance;
    FP32 against the FP64 oracle on the same FP32-rounded inputs, and against
    the regular form."""
    d, x = _case(70, 65, "hole")
    if precision == "mixed":
        d = f32_inputs(d)
        x = np.asarray(x, np.float32).astype(np.float64)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    D = lin.damping()
    prob = make_problem(d, precision)
    prob.set_tuning(large_grid_form=1)
    assert prob.get_tuning().get("large_grid_form") == 1
    reg = make_problem(d, precision)
    xt = to_dev(prob, x)
    prob.linearize(xt)
    xr = to_dev(reg, x)
    reg.linearize(xr)
    A = (lin.JT @ lin.J).tocsr()
    Ls = (1, 7, 8, 25) if precision == "fp64" else (1, 7, 8)
    for L in Ls:
        Mi = lin.minv(True, lam, D) if lam else lin.minv(True)
        ref, _ = o.pcg(lambda v: lin.apply(v, lam, D) if lam else lin.apply(v), lin.jtf(), Mi, L)
        got = to_np(prob.pcg(L, lam=lam, variant="fused"))
        if precision == "fp64":
            ref2, _ = o.pcg(lambda v: A @ v + lam * D * v, lin.jtf(), Mi, L)
            assert relmax(got, ref) < pcg_tol(ref, ref2), L
        else:
            assert relmax(got, ref) < 2e-4, (L, relmax(got, ref))
            assert relmax(got, to_np(reg.pcg(L, lam=lam, variant="fused"))) < 1e-5, L


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_grid_form_solves(precision):
    """GN and LM solves in the large-grid form agree with the oracle (FP64: cost
    traces to 1e-9; mixed: final cost to 1e-4 and the same accepted steps)."""
    d = w.arap_warp(64, 64, seed=1)
    e = o.make_energy(d)
    xo, costs = o.gauss_newton(e, d["x0"], 5, 20)
    xl, costs_l, acc = o.levenberg_marquardt(e, d["x0"], 5, 20)
    prob = make_problem(d, precision)
    prob.set_tuning(large_grid_form=1)
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=5, pcg_iters=20)
    xt2 = to_dev(prob, d["x0"])
    rep_l = prob.solve(xt2, method="lm", outer_iters=5, pcg_iters=20)
    assert rep_l["steps_accepted"] == sum(acc)
    if precision == "fp64":
        assert np.allclose(rep["cost_trace"], costs, rtol=1e-9, atol=0)
        assert np.allclose(rep_l["cost_trace"][:len(costs_l)], costs_l, rtol=1e-9, atol=0)
    else:
        assert abs(rep["cost_final"] - costs[-1]) <= 1e-4 * costs[-1]
        assert abs(rep_l["cost_final"] - costs_l[-1]) <= 1e-4 * costs_l[-1]


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_lm_step_control_closed_form(variant):
    """LM step control on a problem whose only residuals are linear (the
    centre pixel of a masked 3 x 3 warp, fit terms only): the gain ratio is 1, so
    every step is taken and the radius triples; from radius 1 the damping is
    lambda = 1, 1/3, 1/9, 1/27 and x - C shrinks by (1/2)(1/4)(1/10)(1/28).
    With an acceptance threshold above 1 every step is rejected, x does not
    move, and from radius 1e-30 the radius (halved, then divided by 4, 8, 16)
    falls below 1e-32 after four iterations."""
    from tests.test_oracle_pins import _one_pixel_warp
    d = _one_pixel_warp()
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="lm", outer_iters=4, pcg_iters=3, lm_radius0=1.0, pcg_variant=variant)
    assert rep["steps_accepted"] == 4 and rep["outer_done"] == 4
    xs = to_np(xt).reshape(3, 3, 3)
    assert np.allclose([xs[0, 1, 1] - 20.0, xs[1, 1, 1] - 30.0], np.array([2.0, -1.5]) / 2240.0,
                       rtol=0, atol=1e-13)
    wf2 = d["params"]["w_fit"] ** 2
    assert rep["cost_final"] == pytest.approx(wf2 * (2.0 ** 2 + 1.5 ** 2) / 2240.0 ** 2, rel=1e-9)
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="lm", outer_iters=5, pcg_iters=3, lm_radius0=1.0, lm_min_rel_decrease=2.0,
                     pcg_variant=variant)
    assert rep["steps_accepted"] == 0 and rep["outer_done"] == 5
    assert np.array_equal(to_np(xt), d["x0"].ravel())
    rep = prob.solve(xt, method="lm", outer_iters=10, pcg_iters=3, lm_radius0=1e-30, lm_radius_min=1e-32,
                     lm_min_rel_decrease=2.0, pcg_variant=variant)
    assert rep["outer_done"] == 4 and rep["steps_accepted"] == 0
