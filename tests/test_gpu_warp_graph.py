"""ARAP image warping with explicit connectivity (the graph form) against the
grid form and the grid oracle.

With the 4-neighbour edges of the pixel lattice (each pair once, both
orientations evaluated) the graph energy has exactly the grid energy's
residuals, so its cost, J^T F, diag(J^T J), products, PCG iterates and GN/LM
solves must match the FP64 oracle of the grid energy (Sec. 7, the implicit vs
explicit connectivity comparison of Fig. 18)."""
import numpy as np
import pytest
import oracle as o
import workloads as w
from workloads.mesh import grid_edges
from tests.gpu_util import make_problem, relmax, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _graph_problem(d, precision):
    """The warp of `d` as a graph: vertex j*W+i, the lattice's 4-neighbour edges."""
    return make_problem(dict(d, V=d["W"] * d["H"], edges=grid_edges(d["W"], d["H"])), precision)


def _case(W, H, mask, seed=3):
    d = w.arap_warp(W, H, seed=seed, n_constraints=max(2, W * H // 64), margin=2, mask=mask)
    rng = np.random.default_rng(seed)
    x = d["x0"] + np.concatenate([rng.normal(0, 0.5, (2, H, W)), rng.normal(0, 0.2, (1, H, W))])
    return d, np.where((d["mask"] == 0)[None], x, d["x0"])


@pytest.mark.parametrize("W,H,mask", [(9, 7, "none"), (37, 29, "random"), (70, 65, "hole")])
def test_graph_form_operators(W, H, mask):
    d, x = _case(W, H, mask)
    lin = o.Linearization(o.make_energy(d), x)
    prob = _graph_problem(d, "fp64")
    xt = to_dev(prob, x)
    assert abs(prob.cost(xt) - lin.E) <= 1e-12 * lin.E
    assert abs(prob.linearize(xt) - lin.E) <= 1e-12 * lin.E
    b, dg = prob.eval_jtf()
    assert relmax(to_np(b), lin.jtf()) < 1e-12
    assert relmax(to_np(dg), lin.diag) < 1e-12
    p = np.random.default_rng(1).normal(size=lin.diag.size) * lin.active
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p))), lin.apply(p)) < 1e-12
    D = lin.damping()
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p), lam=0.21)), lin.apply(p, 0.21, D)) < 1e-12
    ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), 12)
    assert relmax(to_np(prob.pcg(12)), ref) < 1e-9


def test_graph_form_solves_match_grid_form():
    d, _ = _case(64, 48, "random")
    e = o.make_energy(d)
    xo, costs = o.gauss_newton(e, d["x0"], 3, 20)
    for precision, tol in (("fp64", 1e-9), ("mixed", 1e-4)):
        g = _graph_problem(d, precision)
        xg = to_dev(g, d["x0"])
        rg = g.solve(xg, method="gn", outer_iters=3, pcg_iters=20)
        grid = make_problem(d, precision)
        xd = to_dev(grid, d["x0"])
        rd = grid.solve(xd, method="gn", outer_iters=3, pcg_iters=20)
        assert abs(rg["cost_final"] - costs[-1]) <= tol * costs[-1], precision
        assert abs(rd["cost_final"] - costs[-1]) <= tol * costs[-1], precision
    xl, lcosts, acc = o.levenberg_marquardt(e, d["x0"], 3, 12)
    g = _graph_problem(d, "fp64")
    xg = to_dev(g, d["x0"])
    rep = g.solve(xg, method="lm", outer_iters=3, pcg_iters=12)
    assert rep["steps_accepted"] == sum(acc)
    assert np.allclose(rep["cost_trace"][:len(lcosts)], lcosts, rtol=1e-9, atol=0)
