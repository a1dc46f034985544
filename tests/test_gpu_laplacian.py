"""The Laplacian energy (Figs. 3 and 5) on the GPU: operators against the FP64
oracle, the one-step exactness of Gauss-Newton on this linear energy against
the closed form (w_f^2 I + w_r^2 D^T D) x = w_f^2 A solved by scipy, and the
grid form against the graph form on the lattice's edge list.

Tolerances: FP64 operators 1e-12 of their largest entry; one GN step with
N inner iterations reaches the closed form to 1e-9; mixed precision 1e-4
relative cost."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

import oracle as o
import workloads as w
from tests.gpu_util import f32_inputs, make_problem, pcg_tol, relmax, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _grad_ops(W, H):
    """Forward differences to the right and down neighbour (built directly, not
    by the oracle)."""
    def d1(n):
        return sp.diags([np.ones(n - 1), -np.ones(n - 1)], [0, 1], shape=(n - 1, n))
    return sp.kron(sp.eye(H), d1(W)), sp.kron(d1(H), sp.eye(W))


@pytest.mark.parametrize("W,H", [(9, 7), (70, 53)])
def test_grid_operators_fp64(W, H):
    d = w.laplacian_grid(W, H, seed=2)
    x = np.random.default_rng(1).normal(size=W * H)
    lin = o.Linearization(o.make_energy(d), x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    assert abs(prob.cost(xt) - lin.E) <= 1e-12 * lin.E
    assert abs(prob.linearize(xt) - lin.E) <= 1e-12 * lin.E
    b, dg = prob.eval_jtf()
    assert relmax(to_np(b), lin.jtf()) < 1e-12 and relmax(to_np(dg), lin.diag) < 1e-12
    p = np.random.default_rng(3).normal(size=W * H)
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p))), lin.apply(p)) < 1e-12


def test_graph_operators_fp64():
    d = w.laplacian_mesh(3, seed=2)
    x = np.random.default_rng(1).normal(size=d["x0"].size)
    lin = o.Linearization(o.make_energy(d), x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    assert abs(prob.cost(xt) - lin.E) <= 1e-12 * lin.E
    prob.linearize(xt)
    b, dg = prob.eval_jtf()
    assert relmax(to_np(b), lin.jtf()) < 1e-12 and relmax(to_np(dg), lin.diag) < 1e-12
    p = np.random.default_rng(3).normal(size=x.size)
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p))), lin.apply(p)) < 1e-12


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_one_gn_step_reaches_closed_form(variant):
    W, H = 16, 12
    d = w.laplacian_grid(W, H, seed=3)
    wf, wr = d["params"]["w_fit"], d["params"]["w_reg"]
    Dh, Dv = _grad_ops(W, H)
    M = (wf ** 2) * sp.eye(W * H) + (wr ** 2) * (Dh.T @ Dh + Dv.T @ Dv)
    x_star = spla.spsolve(M.tocsc(), (wf ** 2) * d["A"].ravel())
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    prob.solve(xt, method="gn", outer_iters=1, pcg_iters=W * H, pcg_variant=variant)
    assert np.abs(to_np(xt) - x_star).max() < 1e-9 * max(1.0, np.abs(x_star).max())


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_pcg_fp64(variant):
    W, H = 40, 31
    d = w.laplacian_grid(W, H, seed=5)
    x = np.random.default_rng(4).normal(size=W * H)
    lin = o.Linearization(o.make_energy(d), x)
    prob = make_problem(d, "fp64")
    prob.linearize(to_dev(prob, x))
    A = (lin.JT @ lin.J).tocsr()
    for L in (1, 7, 20):
        ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), L)
        ref2, _ = o.pcg(lambda v: A @ v, lin.jtf(), lin.minv(True), L)
        assert relmax(to_np(prob.pcg(L, variant=variant)), ref) < pcg_tol(ref, ref2), L


def test_grid_equals_graph_on_the_lattice():
    W, H = 23, 17
    dg = w.laplacian_grid(W, H, seed=6)
    A3 = np.repeat(dg["A"].reshape(1, -1), 3, 0)
    dm = dict(energy="laplacian_graph", V=W * H, edges=w.grid_edges(W, H), A=A3, x0=np.zeros((3, W * H)),
              params=dg["params"])
    pg, pm = make_problem(dg, "fp64"), make_problem(dm, "fp64")
    xg, xm = to_dev(pg, dg["x0"]), to_dev(pm, dm["x0"])
    rg = pg.solve(xg, method="gn", outer_iters=2, pcg_iters=25, pcg_variant="split")
    rm = pm.solve(xm, method="gn", outer_iters=2, pcg_iters=25)
    assert np.allclose(rm["cost_trace"], 3 * np.asarray(rg["cost_trace"]), rtol=1e-10, atol=0)
    for c in range(3):
        assert relmax(to_np(xm).reshape(3, -1)[c], to_np(xg)) < 1e-10


def test_gn_mixed():
    d = w.laplacian_grid(96, 80, seed=7)
    d32 = f32_inputs(d)
    xo, costs = o.gauss_newton(o.make_energy(d32), d32["x0"], 2, 30)
    prob = make_problem(d, "mixed")
    rep = prob.solve(to_dev(prob, d32["x0"]), method="gn", outer_iters=2, pcg_iters=30)
    assert abs(rep["cost_final"] - costs[-1]) <= 1e-4 * costs[-1]
