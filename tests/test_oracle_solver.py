"""Pins of the oracle's PCG, GN and LM against library routines and the
guarantees the paper states."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as o
import workloads as w


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.normal(size=(n, n))
    return B @ B.T + n * np.eye(n) * 0.05


def test_pcg_matches_scipy_cg_iterates():
    d = w.arap_warp(12, 10, seed=2, n_constraints=8, margin=2)
    e = o.make_energy(d)
    lin = o.Linearization(e, d["x0"])
    A = (lin.JT @ lin.J).tocsr()
    b = lin.jtf()
    minv = lin.minv(True)
    for L in (1, 3, 10, 25):
        ours, _ = o.pcg(lin.apply, b, minv, L)
        ref, info = spla.cg(A, b, x0=np.zeros_like(b), rtol=0.0, atol=0.0, maxiter=L,
                            M=sp.diags(minv))
        assert np.linalg.norm(ours - ref) <= 1e-10 * np.linalg.norm(ref)


def test_pcg_full_length_equals_dense_solve():
    n = 12
    A = _spd(n, 1)
    b = np.random.default_rng(2).normal(size=n)
    minv = 1.0 / np.diag(A)
    x, info = o.pcg(lambda p: A @ p, b, minv, 3 * n)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)


def test_pcg_zero_rhs_stops():
    A = _spd(5, 3)
    x, info = o.pcg(lambda p: A @ p, np.zeros(5), np.ones(5), 10)
    assert info.stopped and info.iterations == 0 and not x.any()


def test_gn_decreases_warp_cost():
    d = w.arap_warp(32, 32, seed=1)
    e = o.make_energy(d)
    x, costs = o.gauss_newton(e, d["x0"], 4, 20)
    assert costs[-1] < 0.1 * costs[0]


def test_lm_monotone_and_rejections_keep_x():
    d = w.arap_warp(16, 16, seed=3, n_constraints=6, sigma=4.0, margin=3)
    e = o.make_energy(d)
    x, costs, acc = o.levenberg_marquardt(e, d["x0"], 8, 10)
    for k, a in enumerate(acc):
        if a:
            assert costs[k + 1] < costs[k]
        else:
            assert costs[k + 1] == costs[k]
    # a demanding acceptance threshold forces rejections; x must stay put
    prm = o.LMParams(min_rel_decrease=0.999999)
    x2, costs2, acc2 = o.levenberg_marquardt(e, d["x0"], 4, 10, prm)
    assert not all(acc2)
    if not any(acc2):
        assert np.array_equal(x2, d["x0"].ravel())


def test_lm_tiny_damping_equals_gn_step():
    d = w.arap_warp(16, 16, seed=3, n_constraints=6, margin=3)
    e = o.make_energy(d)
    xg, _ = o.gauss_newton(e, d["x0"], 1, 15)
    xl, _, acc = o.levenberg_marquardt(e, d["x0"], 1, 15, o.LMParams(radius0=1e16))
    assert acc[0]
    step = xg - d["x0"].ravel()
    assert np.linalg.norm(xl - xg) <= 1e-9 * np.linalg.norm(step)


def test_lm_mesh_converges():
    d = w.arap_mesh(2, seed=3, handle_frac=0.05, sigma=0.1)
    e = o.make_energy(d)
    x, costs, acc = o.levenberg_marquardt(e, d["x0"], 6, 20)
    assert costs[-1] < costs[0]
    assert any(acc)
