"""Closed forms, exact invariants and a hand-solved fixture for the oracle."""
import json
import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as o
import workloads as w
from oracle.energies import euler_rotate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_warp_rest_state_zero_energy():
    d = w.arap_warp(16, 12, seed=1, n_constraints=10, margin=2)
    d["C"] = np.where(d["C"] >= 0, d["U"], -1.0)
    e = o.make_energy(d)
    assert o.cost(e, d["x0"]) == 0.0


def test_warp_rigid_motion_zero_energy():
    d = w.arap_warp(16, 12, seed=1, n_constraints=10, margin=2, mask="random")
    th, t = 0.7, np.array([3.0, -2.0])
    U = d["U"]
    O = np.stack([np.cos(th) * U[0] - np.sin(th) * U[1] + t[0],
                  np.sin(th) * U[0] + np.cos(th) * U[1] + t[1]])
    # targets non-negative so the fit terms stay valid
    O = O + 40.0
    d["C"] = np.where(d["C"] >= 0, O, -1.0)
    x = np.concatenate([O, np.full((1,) + O.shape[1:], th)])
    assert o.cost(o.make_energy(d), x) < 1e-20


def test_warp_diagonal_closed_form():
    # interior pixel of a unit lattice: 4 rotation residuals with |dU| = 1 each,
    # 8 offset residuals touching it (4 own + 4 of the neighbours) of weight w_reg
    d = w.arap_warp(9, 9, seed=1, n_constraints=1, margin=4)
    e = o.make_energy(d)
    lin = o.Linearization(e, d["x0"] + 0.1 * np.random.default_rng(0).normal(size=d["x0"].shape))
    wf, wr = d["params"]["w_fit"], d["params"]["w_reg"]
    n = 81
    diag = lin.diag.reshape(3, 9, 9)
    fit = (d["C"][0] >= 0)
    assert np.allclose(diag[2, 1:-1, 1:-1], 4 * wr ** 2, rtol=1e-14)
    assert np.allclose(diag[0, 1:-1, 1:-1], 8 * wr ** 2 + wf ** 2 * fit[1:-1, 1:-1], rtol=1e-14)
    # a corner pixel has two neighbours
    assert np.isclose(diag[2, 0, 0], 2 * wr ** 2) and np.isclose(diag[1, 0, 0], 4 * wr ** 2)
    assert lin.diag.size == 3 * n


def test_mesh_rest_and_rigid_zero_energy():
    d = w.arap_mesh(2, seed=3, handle_frac=0.05)
    d["C"] = np.where(d["C"] > -1e6, d["U"], d["C"])
    e = o.make_energy(d)
    assert o.cost(e, d["x0"]) == 0.0
    a0 = np.array([0.3, -0.5, 1.1])
    A = np.repeat(a0[:, None], d["V"], 1)
    O = euler_rotate(A, d["U"]) + np.array([[0.5], [-1.0], [2.0]])
    d["C"] = np.where(d["C"] > -1e6, O, d["C"])
    x = np.concatenate([O, A])
    assert o.cost(o.make_energy(d), x) < 1e-24


def test_euler_rotation_is_zyx_product():
    a = np.array([0.3, -0.5, 1.1])
    cx, sx, cy, sy, cz, sz = np.cos(a[0]), np.sin(a[0]), np.cos(a[1]), np.sin(a[1]), np.cos(a[2]), np.sin(a[2])
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    d = np.array([0.2, 0.7, -1.3])
    assert np.allclose(euler_rotate(a[:, None], d[:, None])[:, 0], Rz @ Ry @ Rx @ d, atol=1e-15)


def test_poisson_identity_zero_energy():
    d = w.poisson_edit(12, 10, seed=5)
    d["T"] = d["base"].copy()
    assert o.cost(o.make_energy(d), d["x0"]) == 0.0


def test_flow_identical_frames_zero_energy():
    d = w.optical_flow(16, 12, seed=4)
    d["Ihat"] = d["I"].copy()
    assert o.cost(o.make_energy(d), d["x0"]) == 0.0


def test_sfs_constant_depth_flat_light_zero_energy():
    # Constant depth d: n = (0, 0, -d^2/(f_x f_y)) normalises to (0,0,-1), whose
    # brightness is L1 - L3 + 2 L7 = 0.5 + 0.3 + 0.1 = 0.9 for the lighting used.
    W, H = 10, 9
    d = w.shape_from_shading(W, H, seed=1)
    depth = 1.7
    d["D"] = np.full((H, W), depth)
    d["Im"] = np.full((H, W), 0.9)
    e = o.make_energy(d)
    x = np.full((1, H, W), depth)
    assert o.cost(e, x) < 1e-24
    F = e.residuals(x)
    # the shading terms vanish and every smoothness term is active in the interior
    assert e.smooth_valid(x[0])[1:-1, 1:-1].all()
    assert np.abs(F).max() < 1e-12


def _grad_ops(W, H):
    """Forward-difference operators with zero rows dropped at the far edge."""
    def d1(n):
        return sp.diags([np.ones(n - 1), -np.ones(n - 1)], [0, 1], shape=(n - 1, n))
    Dh = sp.kron(sp.eye(H), d1(W))
    Dv = sp.kron(d1(H), sp.eye(W))
    return Dh, Dv


def test_laplacian_grid_closed_form_one_step():
    W, H = 8, 8
    d = w.laplacian_grid(W, H, seed=3)
    e = o.make_energy(d)
    wf, wr = 0.1, 0.9
    Dh, Dv = _grad_ops(W, H)
    A = d["A"].ravel()
    M = (wf ** 2) * sp.eye(W * H) + (wr ** 2) * (Dh.T @ Dh + Dv.T @ Dv)
    x_star = spla.spsolve(M.tocsc(), (wf ** 2) * A)
    # GN with an inner solve of N = 64 PCG iterations reaches the minimiser in one step
    x1, costs = o.gauss_newton(e, d["x0"], 1, W * H)
    assert np.abs(x1 - x_star).max() < 1e-9
    lin = o.Linearization(e, x1)
    assert np.linalg.norm(lin.jtf()) < 1e-10
    x2, _ = o.gauss_newton(e, x1, 1, W * H)
    assert np.abs(x2 - x1).max() < 1e-10


def test_laplacian_graph_equals_grid():
    W, H = 6, 5
    dg = w.laplacian_grid(W, H, seed=4)
    edges = w.grid_edges(W, H)
    A3 = np.repeat(dg["A"].reshape(1, -1), 3, 0)
    eg = o.LaplacianGraph(W * H, edges, A3, 0.1, 0.9)
    ei = o.make_energy(dg)
    x = np.random.default_rng(1).normal(size=W * H)
    Ji = o.jacobian(ei, x).toarray()
    Jg = o.jacobian(eg, np.tile(x, 3)).toarray()
    n = W * H
    assert np.allclose(Jg[:, :n].T @ Jg[:, :n], Ji.T @ Ji, atol=1e-14)
    assert np.isclose(o.cost(eg, np.tile(x, 3)), 3 * o.cost(ei, x), rtol=1e-13)


def test_laplacian_golden_2x1():
    g = json.load(open(os.path.join(GOLDEN, "laplacian_2x1.json")))
    e = o.LaplacianGrid(g["W"], g["H"], np.array(g["A"]).reshape(1, 2), 0.1, 0.9)
    x, costs = o.gauss_newton(e, np.zeros(2), 1, 2)
    assert np.allclose(x, g["x_opt"], atol=1e-13, rtol=0)
    assert abs(costs[-1] - g["E_opt"]) < 1e-15


def test_poisson_one_step_exact_matches_discrete_poisson_equation():
    W, H = 10, 8
    d = w.poisson_edit(W, H, seed=7)
    e = o.make_energy(d)
    act = (d["mask"] == 0).ravel()
    n = W * H
    nact = int(act.sum())
    x1, costs = o.gauss_newton(e, d["x0"], 1, 4 * nact)
    # textbook form: for every free pixel, deg(p) x_p - sum_{free q} x_q
    #   = sum_q (T_p - T_q) + sum_{fixed q} x_q, neighbours q on the grid
    s = np.arange(n).reshape(H, W)
    pairs = np.concatenate([np.stack([s[:, :-1].ravel(), s[:, 1:].ravel()], 1),
                            np.stack([s[:-1].ravel(), s[1:].ravel()], 1)])
    pairs = np.concatenate([pairs, pairs[:, ::-1]])
    Adj = sp.csr_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(n, n))
    deg = np.asarray(Adj.sum(1)).ravel()
    Lap = sp.diags(deg) - Adj
    idx = np.nonzero(act)[0]
    fixed = np.nonzero(~act)[0]
    X0 = d["x0"].reshape(4, n)
    T = d["T"].reshape(4, n)
    for c in range(4):
        rhs = (Lap @ T[c])[idx] - (Lap[idx][:, fixed] @ X0[c, fixed])
        xs = spla.spsolve(Lap[idx][:, idx].tocsc(), rhs)
        assert np.abs(x1.reshape(4, n)[c, idx] - xs).max() < 1e-8
        assert np.array_equal(x1.reshape(4, n)[c, fixed], X0[c, fixed])
    x2, _ = o.gauss_newton(e, x1, 1, 4 * nact)
    assert np.abs(x2 - x1).max() < 1e-8


def test_operator_symmetric_psd():
    d = w.arap_warp(10, 9, seed=2, n_constraints=6, margin=2, mask="random")
    e = o.make_energy(d)
    rng = np.random.default_rng(3)
    lin = o.Linearization(e, d["x0"] + 0.2 * rng.normal(size=d["x0"].shape))
    u, v = rng.normal(size=(2, lin.diag.size))
    assert np.isclose(u @ lin.apply(v), v @ lin.apply(u), rtol=1e-13)
    assert u @ lin.apply(u) >= 0
    # excluded unknowns have empty columns
    act = lin.active
    assert np.all(lin.diag[~act] == 0)
