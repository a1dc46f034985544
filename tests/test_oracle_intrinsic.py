"""Pins of the oracle's intrinsic image decomposition (A.2.4, Fig. 33) and its
IRLS solve (Sec. 7), each against something other than the oracle's own
formulas:

* the weight at a hand-computed point, and w = 1 at p = 2;
* the frozen operator J^T J, J^T F and the diagonal against w_fit^2 F^T F +
  2 w_a^2 sum_c D^T diag(w) D (reflectance) + 2 w_s^2 D^T D (shading), built
  here from forward-difference and fit matrices (each edge is a residual at both
  of its ends, hence the 2);
* the objective is invariant along the decomposition's null direction (all
  reflectance channels down by t, the shading up by t), and so are the frozen
  weights;
* with exact inner solves (minimum-norm least squares) IRLS never raises the
  objective for p <= 2 and ends at a stationary point of it (central-difference
  gradient), which fails without the factor p/2 of the weight; at p = 2 one exact
  step reaches the minimiser;
* the oracle's IRLS with PCG run to convergence reaches the same objectives as
  those exact steps (its iterates may differ along the null direction only).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as o
import workloads as w


def _diff_ops(W, H):
    def d1(n):
        return sp.diags([np.ones(n - 1), -np.ones(n - 1)], [0, 1], shape=(n - 1, n))
    return sp.kron(sp.eye(H), d1(W)).tocsr(), sp.kron(d1(H), sp.eye(W)).tocsr()


def _operator(e, d):
    """(M, b) of the frozen problem at e's weights, channel-major unknowns."""
    W, H = d["W"], d["H"]
    n = W * H
    p = d["params"]
    Dh, Dv = _diff_ops(W, H)
    wh, wv = e.wh[:, :W - 1].ravel(), e.wv[:H - 1, :].ravel()
    Lr = 2 * p["w_a"] ** 2 * (Dh.T @ sp.diags(wh) @ Dh + Dv.T @ sp.diags(wv) @ Dv)
    Ls = 2 * p["w_s"] ** 2 * (Dh.T @ Dh + Dv.T @ Dv)
    I = sp.eye(n)
    F = sp.bmat([[I, None, None, I], [None, I, None, I], [None, None, I, I]])  # r_c + s
    Z = sp.csr_matrix((n, n))
    Lap = sp.bmat([[Lr, Z, Z, Z], [Z, Lr, Z, Z], [Z, Z, Lr, Z], [Z, Z, Z, Ls]])
    M = (p["w_fit"] ** 2 * (F.T @ F) + Lap).tocsr()
    rhs = p["w_fit"] ** 2 * (F.T @ d["I"].ravel())
    return M, rhs


def test_weight_values():
    e = o.IntrinsicImage(3, 2, np.zeros((3, 2, 3)), 1.0, 1.0, 1.0, 1.0, 0.1)
    assert abs(e.weight(0.09) - 0.5 / np.sqrt(0.1)) < 1e-15
    e2 = o.IntrinsicImage(3, 2, np.zeros((3, 2, 3)), 1.0, 1.0, 1.0, 2.0, 0.1)
    assert np.all(e2.weight(np.array([0.0, 0.3, 5.0])) == 1.0)


@pytest.mark.parametrize("p", [0.8, 1.5])
def test_frozen_operator_is_the_weighted_laplacian(p):
    W, H = 9, 7
    d = w.intrinsic_image(W, H, seed=3, p=p, eps=0.02)
    e = o.make_energy(d)
    x = d["x0"].ravel() + 0.05 * np.random.default_rng(1).normal(size=4 * W * H)
    e.freeze(x)
    lin = o.Linearization(e, x)
    M, rhs = _operator(e, d)
    v = np.random.default_rng(2).normal(size=4 * W * H)
    assert np.abs(lin.apply(v) - M @ v).max() <= 1e-13 * np.abs(M @ v).max()
    b = rhs - M @ x
    assert np.abs(lin.jtf() - b).max() <= 1e-12 * np.abs(b).max()
    assert np.abs(lin.diag - M.diagonal()).max() <= 1e-13 * M.diagonal().max()


def test_null_direction():
    d = w.intrinsic_image(8, 6, seed=4)
    e = o.make_energy(d)
    x = d["x0"] + 0.1 * np.random.default_rng(3).normal(size=d["x0"].shape)
    shift = np.concatenate([-np.ones((3, 6, 8)), np.ones((1, 6, 8))]) * 0.37
    assert abs(e.objective(x + shift) - e.objective(x)) <= 1e-12 * e.objective(x)
    e.freeze(x)
    wh, wv = e.wh.copy(), e.wv.copy()
    e.freeze(x + shift)
    assert np.allclose(e.wh, wh, rtol=1e-12, atol=0) and np.allclose(e.wv, wv, rtol=1e-12, atol=0)


def _exact_irls(e, d, x0, iters):
    x = np.asarray(x0, float).ravel().copy()
    objs, xs = [e.objective(x)], [x.copy()]
    for _ in range(iters):
        e.freeze(x)
        M, rhs = _operator(e, d)
        x = np.linalg.lstsq(M.toarray(), rhs, rcond=None)[0]
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


@pytest.mark.parametrize("p", [0.8, 1.5])
def test_exact_irls_descends_to_a_stationary_point(p):
    d = w.intrinsic_image(6, 5, seed=5, p=p, eps=0.05)
    e = o.make_energy(d)
    x0 = d["x0"].ravel()
    xs, objs = _exact_irls(e, d, x0, 150)
    assert all(b <= a * (1 + 1e-13) for a, b in zip(objs, objs[1:])), objs[:10]
    g0 = np.linalg.norm(_grad_fd(e, x0))
    gK = np.linalg.norm(_grad_fd(e, xs[-1]))
    assert gK <= 1e-6 * g0, (gK, g0)


def test_p2_one_exact_step_is_the_minimiser():
    d = w.intrinsic_image(6, 5, seed=6, p=2.0, eps=0.05)
    e = o.make_energy(d)
    xs, _ = _exact_irls(e, d, d["x0"].ravel(), 1)
    assert np.linalg.norm(_grad_fd(e, xs[1])) <= 1e-7 * np.linalg.norm(_grad_fd(e, xs[0]))


def test_oracle_irls_matches_exact_steps():
    d = w.intrinsic_image(7, 6, seed=7, p=1.0, eps=0.05)
    e = o.make_energy(d)
    xs, objs = _exact_irls(e, d, d["x0"].ravel(), 4)
    # the normal equations are semidefinite (the null direction): PCG from 0
    # converges by about 80 iterations at this size, and long past convergence
    # rounding drives it along the null direction, so the comparison stops there
    x, objs2 = o.irls(e, d["x0"], 4, 80)
    assert np.allclose(objs2, objs, rtol=1e-9, atol=0)
    # the iterates differ at most along the null direction
    dx = (x - xs[-1]).reshape(4, -1)
    t = dx[3].mean()
    assert np.abs(dx[3] - t).max() <= 1e-7 and np.abs(dx[:3] + t).max() <= 1e-7
