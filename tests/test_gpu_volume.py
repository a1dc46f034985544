"""GPU parity of volumetric ARAP (3D grid, Fig. 31, A.2.5) against the FP64
oracle, and against the mesh energy's graph path on the voxel lattice's edge
list (the same residuals; implicit vs explicit connectivity in 3D).

Tolerances as for the other energies: FP64 operators 1e-12 of their largest
entry, FP64 PCG the oracle-spread rule, FP64 GN/LM cost traces 1e-9 relative,
mixed-precision operators 1e-5 on FP32-rounded inputs and mixed LM 1e-4
relative final cost (5% handles: well conditioned)."""
import numpy as np
import pytest
import torch

import oracle as o
import workloads as w
from tests.gpu_util import pcg_tol, f32_inputs, make_problem, relmax, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _volume(W, H, D, seed=3, handle_frac=0.05, sigma=0.5, scale=0.2):
    d = w.arap_volume(W, H, D, seed=seed, handle_frac=handle_frac, sigma=sigma)
    rng = np.random.default_rng(seed)
    x = d["x0"] + scale * rng.normal(size=d["x0"].shape)
    return d, x


def _as_mesh(d):
    return dict(energy="arap_mesh", V=d["W"] * d["H"] * d["D"], edges=w.lattice_edges(d["W"], d["H"], d["D"]),
                U=d["U"], C=d["C"], x0=d["x0"], params=d["params"])


@pytest.mark.parametrize("dims", [(4, 3, 2), (17, 13, 11)])
def test_operators_fp64(dims):
    d, x = _volume(*dims)
    lin = o.Linearization(o.make_energy(d), x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    assert abs(prob.cost(xt) - lin.E) <= 1e-12 * lin.E
    assert abs(prob.linearize(xt) - lin.E) <= 1e-12 * lin.E
    b, dg = prob.eval_jtf()
    assert relmax(to_np(b), lin.jtf()) < 1e-12
    assert relmax(to_np(dg), lin.diag) < 1e-12
    p = np.random.default_rng(2).normal(size=lin.diag.size)
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p))), lin.apply(p)) < 1e-12
    D = lin.damping()
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p), lam=0.4)), lin.apply(p, 0.4, D)) < 1e-12


def test_dense_jtj_small_block():
    d, x = _volume(3, 2, 2, seed=5)
    lin = o.Linearization(o.make_energy(d), x)
    A = (lin.J.T @ lin.J).toarray()
    prob = make_problem(d, "fp64")
    prob.linearize(to_dev(prob, x))
    N = A.shape[0]
    G = np.stack([to_np(prob.apply_jtj(to_dev(prob, np.eye(N)[k]))) for k in range(N)], 1)
    assert np.abs(G - A).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_pcg_fp64(variant):
    d, x = _volume(9, 8, 7)
    lin = o.Linearization(o.make_energy(d), x)
    prob = make_problem(d, "fp64")
    prob.linearize(to_dev(prob, x))
    A = (lin.JT @ lin.J).tocsr()
    for L in (1, 10, 25):
        ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), L)
        ref2, _ = o.pcg(lambda v: A @ v, lin.jtf(), lin.minv(True), L)
        tol = pcg_tol(ref, ref2)
        assert relmax(to_np(prob.pcg(L, variant=variant)), ref) < tol, L


def test_lm_fp64():
    d = w.arap_volume(8, 7, 6, seed=3, handle_frac=0.05, sigma=0.5)
    xo, costs, acc = o.levenberg_marquardt(o.make_energy(d), d["x0"], 5, 20)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="lm", outer_iters=5, pcg_iters=20)
    assert rep["steps_accepted"] == sum(acc)
    assert np.allclose(rep["cost_trace"][:len(costs)], costs, rtol=1e-9, atol=0)
    assert relmax(to_np(xt) - d["x0"].ravel(), xo - d["x0"].ravel()) < 1e-8


def test_gn_fp64():
    d = w.arap_volume(7, 6, 5, seed=4, handle_frac=0.05, sigma=0.3)
    xo, costs = o.gauss_newton(o.make_energy(d), d["x0"], 3, 15)
    prob = make_problem(d, "fp64")
    rep = prob.solve(to_dev(prob, d["x0"]), method="gn", outer_iters=3, pcg_iters=15)
    assert np.allclose(rep["cost_trace"], costs, rtol=1e-9, atol=0)


def test_operators_mixed():
    d, x = _volume(12, 10, 9)
    d32 = f32_inputs(d)
    x32 = np.asarray(x, np.float32).astype(np.float64)
    lin = o.Linearization(o.make_energy(d32), x32)
    prob = make_problem(d, "mixed")
    xt = to_dev(prob, x32)
    assert abs(prob.cost(xt) - lin.E) <= 1e-12 * lin.E
    assert abs(prob.linearize(xt) - lin.E) <= 1e-12 * lin.E
    b, dg = prob.eval_jtf()
    p32 = np.asarray(np.random.default_rng(2).normal(size=lin.diag.size), np.float32).astype(np.float64)
    errs = [relmax(to_np(b), lin.jtf()), relmax(to_np(dg), lin.diag),
            relmax(to_np(prob.apply_jtj(to_dev(prob, p32))), lin.apply(p32))]
    assert max(errs) < 1e-5, errs


def test_lm_mixed():
    d = w.arap_volume(10, 9, 8, seed=6, handle_frac=0.05, sigma=0.5)
    d32 = f32_inputs(d)
    xo, costs, acc = o.levenberg_marquardt(o.make_energy(d32), d32["x0"], 4, 30)
    prob = make_problem(d, "mixed")
    xt = to_dev(prob, d32["x0"])
    rep = prob.solve(xt, method="lm", outer_iters=4, pcg_iters=30)
    assert rep["steps_accepted"] == sum(acc)
    assert abs(rep["cost_final"] - costs[-1]) <= 1e-4 * costs[-1]


def test_volume_equals_mesh_path_on_the_lattice():
    """Implicit (3D stencil) and explicit (lattice edge list through the graph
    path) connectivity: the same residuals, so the same operators and solves."""
    d, x = _volume(11, 9, 7, seed=8)
    pv = make_problem(d, "fp64")
    pm = make_problem(_as_mesh(d), "fp64")
    xv, xm = to_dev(pv, x), to_dev(pm, x)
    assert abs(pv.linearize(xv) - pm.linearize(xm)) <= 1e-12 * pm.cost(xm)
    bv, dv = pv.eval_jtf()
    bm, dm = pm.eval_jtf()
    assert relmax(to_np(bv), to_np(bm)) < 1e-12 and relmax(to_np(dv), to_np(dm)) < 1e-12
    rv = pv.solve(xv, method="lm", outer_iters=3, pcg_iters=15)
    rm = pm.solve(xm, method="lm", outer_iters=3, pcg_iters=15)
    assert np.allclose(rv["cost_trace"], rm["cost_trace"], rtol=1e-9, atol=0)
    assert rv["steps_accepted"] == rm["steps_accepted"]


def test_bad_domain_rejected():
    import paper_1604_06525_amd as pkg
    d, _ = _volume(4, 4, 4)
    dd = dict(d)
    dd.pop("D")
    # the volume energy on a 2D grid descriptor is refused
    U = torch.zeros(3 * 16, dtype=torch.float64, device="cuda")
    with pytest.raises(pkg.OptError) as ei:
        pkg.Problem("arap_volume", [U, U], [10.0, 1.0], precision="fp64", width=4, height=4, tuning=None)
    assert ei.value.code == pkg.OPT_EUNSUPPORTED
