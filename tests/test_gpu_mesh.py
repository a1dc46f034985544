"""GPU parity of the ARAP mesh (graph domain) path against the FP64 oracle.

The library builds a per-vertex incidence list from the edge list; every product
is a per-vertex gather.  Tolerances as for the grid energies: FP64 operators
1e-12 of their largest entry, FP64 PCG 1e-9, FP64 GN/LM cost traces 1e-9
relative, mixed precision 1e-4 relative final cost.
"""
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


def _mesh(level, seed=3, handle_frac=0.02, sigma=0.1, scale=0.2):
    d = w.arap_mesh(level, seed=seed, handle_frac=handle_frac, sigma=sigma)
    rng = np.random.default_rng(seed)
    x = d["x0"] + scale * rng.normal(size=d["x0"].shape)
    return d, x


@pytest.mark.parametrize("level", [1, 3])
def test_operators_fp64(level):
    d, x = _mesh(level)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
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


def test_dense_jtj_icosphere_level1():
    d, x = _mesh(1, seed=5)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    A = (lin.J.T @ lin.J).toarray()
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    prob.linearize(xt)
    N = A.shape[0]
    G = np.stack([to_np(prob.apply_jtj(to_dev(prob, np.eye(N)[k]))) for k in range(N)], 1)
    assert np.abs(G - A).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_pcg_fp64(variant):
    d, x = _mesh(3)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    prob.linearize(xt)
    A = (lin.JT @ lin.J).tocsr()
    for L in (1, 10, 30):
        ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), L)
        ref2, _ = o.pcg(lambda v: A @ v, lin.jtf(), lin.minv(True), L)
        tol = pcg_tol(ref, ref2)
        got = to_np(prob.pcg(L, variant=variant))
        assert relmax(got, ref) < tol, (L, tol)


def test_lm_fp64():
    d = w.arap_mesh(3, seed=3, handle_frac=0.02, sigma=0.2)
    e = o.make_energy(d)
    xo, costs, acc = o.levenberg_marquardt(e, d["x0"], 5, 20)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="lm", outer_iters=5, pcg_iters=20)
    assert rep["steps_accepted"] == sum(acc)
    assert np.allclose(rep["cost_trace"][:len(costs)], costs, rtol=1e-9, atol=0)
    assert relmax(to_np(xt) - d["x0"].ravel(), xo - d["x0"].ravel()) < 1e-8


def test_gn_fp64():
    d = w.arap_mesh(2, seed=4, handle_frac=0.05)
    e = o.make_energy(d)
    xo, costs = o.gauss_newton(e, d["x0"], 3, 15)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=3, pcg_iters=15)
    assert np.allclose(rep["cost_trace"], costs, rtol=1e-9, atol=0)


@pytest.mark.parametrize("handle_frac,tol", [(0.05, 1e-4), (0.01, 1e-3)])
def test_lm_mixed_level5(handle_frac, tol):
    """LM with 40 PCG iterations, mixed precision, against the FP64 oracle.

    With 5% handles the final cost agrees to 1e-4.  With 1% handles (the
    icosphere configuration's density) the system is so ill-conditioned that 40
    PCG iterations from the first, almost undamped LM step end in a different
    place for any change of FP32 rounding: FP32 emulations of the oracle's PCG
    that differ only in summation order spread by up to 2.2e-4 in final cost
    (5e-6 with 5% handles).  There the bound is 1e-3, and both runs must take
    the same steps."""
    d = w.arap_mesh(5, seed=3, handle_frac=handle_frac)
    e = o.make_energy(d)
    xo, costs, acc = o.levenberg_marquardt(e, d["x0"], 4, 40)
    prob = make_problem(d, "mixed")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="lm", outer_iters=4, pcg_iters=40)
    assert rep["steps_accepted"] == sum(acc)
    assert abs(rep["cost_final"] - costs[-1]) <= tol * costs[-1]


@pytest.mark.parametrize("level", [1, 3])
def test_operators_mixed(level):
    """Mixed precision: the FP64 cost of FP32 values is exact; FP32 products
    agree with the FP64 oracle on the same FP32-rounded inputs to 1e-5 of their
    largest entry (a vertex sums a few dozen FP32 terms)."""
    d, x = _mesh(level)
    d32 = f32_inputs(d)
    x32 = np.asarray(x, np.float32).astype(np.float64)
    e = o.make_energy(d32)
    lin = o.Linearization(e, x32)
    prob = make_problem(d, "mixed")
    xt = to_dev(prob, x32)
    assert abs(prob.cost(xt) - lin.E) <= 1e-12 * lin.E
    assert abs(prob.linearize(xt) - lin.E) <= 1e-12 * lin.E
    b, dg = prob.eval_jtf()
    p = np.random.default_rng(2).normal(size=lin.diag.size)
    p32 = np.asarray(p, np.float32).astype(np.float64)
    errs = [relmax(to_np(b), lin.jtf()), relmax(to_np(dg), lin.diag),
            relmax(to_np(prob.apply_jtj(to_dev(prob, p32))), lin.apply(p32))]
    print("mesh mixed operator errors", errs)
    assert max(errs) < 1e-5


def test_deterministic_mixed():
    d = w.arap_mesh(4, seed=6)
    outs = []
    for _ in range(2):
        prob = make_problem(d, "mixed")
        xt = to_dev(prob, d["x0"])
        rep = prob.solve(xt, method="lm", outer_iters=3, pcg_iters=15)
        outs.append((rep["cost_trace"], to_np(xt)))
    assert outs[0][0] == outs[1][0] and np.array_equal(outs[0][1], outs[1][1])


def test_bad_edge_rejected():
    import paper_1604_06525_amd as pkg
    d = w.arap_mesh(1, seed=3)
    d["edges"] = d["edges"].copy()
    d["edges"][5, 1] = d["V"] + 3
    with pytest.raises(pkg.OptError) as err:
        make_problem(d, "mixed")
    assert err.value.code == pkg.OPT_EINVAL


def _scrambled(level, seed=3):
    """The ARAP mesh workload with its vertex ids randomly relabelled: almost
    every edge then leaves its chunk of 256 consecutive ids, so the per-chunk
    halos overflow their LDS cap and pcg_a reads the rest from global memory."""
    d, x = _mesh(level, seed=seed)
    V = d["V"]
    perm = np.random.default_rng(seed + 100).permutation(V)  # new id k holds old vertex perm[k]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(V)
    d = dict(d, U=d["U"][:, perm].copy(), C=d["C"][:, perm].copy(), x0=d["x0"][:, perm].copy(),
             edges=inv[d["edges"]].astype(np.int32), handles=np.sort(inv[d["handles"]]))
    return d, x[:, perm].copy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_scrambled_ids_halo_overflow(prec):
    d, x = _scrambled(4)
    if prec == "mixed":
        d = f32_inputs(d)
        x = np.asarray(x, np.float32).astype(np.float64)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, prec)
    xt = to_dev(prob, x)
    prob.linearize(xt)
    tol = 1e-12 if prec == "fp64" else 1e-5
    p = np.random.default_rng(7).normal(size=lin.diag.size)
    if prec == "mixed":
        p = np.asarray(p, np.float32).astype(np.float64)
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p))), lin.apply(p)) < tol
    if prec == "fp64":
        ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), 20)
        assert relmax(to_np(prob.pcg(20, variant="split")), ref) < 1e-9


def _custom_mesh(U, edges, handles, seed=9):
    """An ARAP mesh problem on any vertex set and edge list (fit targets at the
    handles, U + N(0, 0.05^2); unknowns start at (U, 0) plus noise)."""
    V = U.shape[1]
    rng = np.random.default_rng(seed)
    C = np.full((3, V), -1e7)
    C[:, handles] = U[:, handles] + rng.normal(0.0, 0.05, (3, len(handles)))
    x0 = np.concatenate([U, np.zeros((3, V))])
    d = dict(energy="arap_mesh", V=V, edges=np.asarray(edges, np.int32).reshape(-1, 2), U=U, C=C, x0=x0,
             handles=np.sort(handles), params=dict(w_fit=10.0, w_reg=1.0))
    return d, x0 + 0.2 * rng.normal(size=x0.shape)


def _degenerate(kind):
    rng = np.random.default_rng(11)
    if kind == "hub":
        # vertex 0 joined to every other vertex (degree 2999, more incidence
        # entries than a chunk stages) plus a ring through the rest
        V = 3000
        e = [(0, v) for v in range(1, V)] + [(v, v + 1) for v in range(1, V - 1)]
        U = rng.normal(size=(3, V))
        return _custom_mesh(U, e, rng.choice(V, 30, replace=False))
    if kind == "isolated":
        # a level-2 icosphere followed by 200 vertices with no edge
        v, _, e = w.icosphere(2)
        V = len(v) + 200
        U = np.concatenate([v.T, rng.normal(size=(3, 200))], axis=1)
        return _custom_mesh(U, e, rng.choice(V, 20, replace=False))
    # no edges at all: only the fit terms of the handles remain
    V = 300
    return _custom_mesh(rng.normal(size=(3, V)), np.zeros((0, 2), np.int32), rng.choice(V, 25, replace=False))


@pytest.mark.parametrize("kind", ["hub", "isolated", "no_edges"])
def test_degenerate_graphs_fp64(kind):
    """Graphs the staged gather must also handle: a vertex of very high degree
    (its chunk's incidence slice overflows the staged slots and its halo the
    cap), vertices without edges (zero diagonal, M^-1 = 0), no edges at all."""
    d, x = _degenerate(kind)
    e = o.make_energy(d)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    assert abs(prob.linearize(xt) - lin.E) <= 1e-12 * lin.E
    b, dg = prob.eval_jtf()
    assert relmax(to_np(b), lin.jtf()) < 1e-12
    assert relmax(to_np(dg), lin.diag) < 1e-12
    p = np.random.default_rng(3).normal(size=lin.diag.size)
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, p))), lin.apply(p)) < 1e-12
    ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), 15)
    for variant in ("split", "fused"):
        assert relmax(to_np(prob.pcg(15, variant=variant)), ref) < 1e-9, variant
