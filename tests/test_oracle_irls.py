"""Pins of the oracle's l_p smoothing energy and its IRLS loop (Sec. 7, variants
of GN/LM), each against something other than the oracle's own formulas:

* the weight at a hand-computed point, and w = 1 at p = 2;
* p = 2: IRLS is Gauss-Newton on the Laplacian energy (the same iterates; the
  objective differs by eps^2 per edge);
* the frozen-weight operator J^T J and J^T F against the weighted graph
  Laplacian w_fit^2 I + w_reg^2 D^T diag(w) D built here from forward
  differences (not from the oracle's Jacobian);
* with exact inner solves, IRLS is a majorise-minimise method for p <= 2: the
  objective never increases, and the fixed point is a stationary point of the
  objective (its gradient by central differences vanishes): this pins the
  factor p/2 of the weight, without which the fixed point minimises another
  function;
* the oracle's IRLS with enough PCG iterations reproduces those exact steps.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as o
import workloads as w


def _diff_ops(W, H):
    """Forward differences to the right and down neighbour, rows only where the
    neighbour exists (site id j*W + i)."""
    def d1(n):
        return sp.diags([np.ones(n - 1), -np.ones(n - 1)], [0, 1], shape=(n - 1, n))
    return sp.kron(sp.eye(H), d1(W)).tocsr(), sp.kron(d1(H), sp.eye(W)).tocsr()


def _weights_on_edges(e, W, H):
    """The frozen weights in the row order of _diff_ops."""
    return e.wh[:, :W - 1].ravel(), e.wv[:H - 1, :].ravel()


def test_weight_values():
    e = o.LpSmoothGrid(3, 2, np.zeros((2, 3)), 1.0, 1.0, 1.0, 0.1)
    assert abs(e.weight(0.3) - 0.5 / np.sqrt(0.1)) < 1e-15
    e2 = o.LpSmoothGrid(3, 2, np.zeros((2, 3)), 1.0, 1.0, 2.0, 0.1)
    assert np.all(e2.weight(np.array([0.0, 0.3, -5.0])) == 1.0)


def test_p2_is_the_laplacian():
    d = w.lp_smooth(11, 8, seed=2, p=2.0, eps=0.05)
    e = o.make_energy(d)
    lap = o.LaplacianGrid(d["W"], d["H"], d["A"], d["params"]["w_fit"], d["params"]["w_reg"])
    x1, objs = o.irls(e, d["x0"], 4, 30)
    x2, costs = o.gauss_newton(lap, d["x0"], 4, 30)
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x2).max()
    n_edges = (d["W"] - 1) * d["H"] + d["W"] * (d["H"] - 1)
    assert np.allclose(np.asarray(objs) - 0.05 ** 2 * n_edges, costs, rtol=1e-12, atol=0)


@pytest.mark.parametrize("p", [1.0, 0.7])
def test_frozen_operator_is_the_weighted_laplacian(p):
    W, H = 9, 7
    d = w.lp_smooth(W, H, seed=3, p=p, eps=0.02)
    e = o.make_energy(d)
    x = d["x0"].ravel() + 0.05 * np.random.default_rng(1).normal(size=W * H)
    e.freeze(x)
    lin = o.Linearization(e, x)
    Dh, Dv = _diff_ops(W, H)
    wh, wv = _weights_on_edges(e, W, H)
    wf, wr = d["params"]["w_fit"], d["params"]["w_reg"]
    M = wf ** 2 * sp.eye(W * H) + wr ** 2 * (Dh.T @ sp.diags(wh) @ Dh + Dv.T @ sp.diags(wv) @ Dv)
    v = np.random.default_rng(2).normal(size=W * H)
    assert np.abs(lin.apply(v) - M @ v).max() <= 1e-13 * np.abs(M @ v).max()
    b = -(wf ** 2 * (x - d["A"].ravel()) + wr ** 2 * (Dh.T @ (wh * (Dh @ x)) + Dv.T @ (wv * (Dv @ x))))
    assert np.abs(lin.jtf() - b).max() <= 1e-13 * np.abs(b).max()
    assert np.abs(lin.diag - M.diagonal()).max() <= 1e-13 * M.diagonal().max()


def _exact_irls(e, d, x0, iters):
    """IRLS with every weighted least-squares step solved exactly (sparse LU)."""
    W, H = d["W"], d["H"]
    Dh, Dv = _diff_ops(W, H)
    wf, wr = d["params"]["w_fit"], d["params"]["w_reg"]
    A = d["A"].ravel()
    x = x0.copy()
    objs, xs = [e.objective(x)], [x.copy()]
    for _ in range(iters):
        e.freeze(x)
        wh, wv = _weights_on_edges(e, W, H)
        M = wf ** 2 * sp.eye(W * H) + wr ** 2 * (Dh.T @ sp.diags(wh) @ Dh + Dv.T @ sp.diags(wv) @ Dv)
        x = spla.spsolve(M.tocsc(), wf ** 2 * A)
        objs.append(e.objective(x))
        xs.append(x.copy())
    return xs, objs


def _grad_fd(e, x, h=1e-6):
    g = np.zeros_like(x)
    for k in range(x.size):
        xp, xm = x.copy(), x.copy()
        xp[k] += h
        xm[k] -= h
        g[k] = (e.objective(xp) - e.objective(xm)) / (2 * h)
    return g


@pytest.mark.parametrize("p", [1.0, 1.5])
def test_exact_irls_descends_to_a_stationary_point(p):
    d = w.lp_smooth(8, 6, seed=4, p=p, eps=0.05)
    e = o.make_energy(d)
    x0 = d["x0"].ravel()
    xs, objs = _exact_irls(e, d, x0, 120)
    assert all(b <= a * (1 + 1e-14) for a, b in zip(objs, objs[1:])), objs[:10]
    g0 = np.linalg.norm(_grad_fd(e, x0))
    gK = np.linalg.norm(_grad_fd(e, xs[-1]))
    assert gK <= 1e-6 * g0, (gK, g0)


def test_oracle_irls_matches_exact_steps():
    d = w.lp_smooth(8, 6, seed=5, p=1.0, eps=0.05)
    e = o.make_energy(d)
    xs, objs = _exact_irls(e, d, d["x0"].ravel(), 5)
    x, objs2 = o.irls(e, d["x0"], 5, 200)
    assert np.abs(x - xs[-1]).max() <= 1e-9 * np.abs(xs[-1]).max()
    assert np.allclose(objs2, objs, rtol=1e-10, atol=0)
