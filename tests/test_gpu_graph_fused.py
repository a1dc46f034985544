"""The fused PCG form on graphs (one kernel per iteration; each block stages a
chunk of 256 vertices with its one- and two-ring neighbourhoods) against the
FP64 oracle and against the split form.

Parity: PCG iterates against the oracle's PCG (the oracle-spread rule of
gpu_util.pcg_tol), against the split form of the same problem (the two
recurrences agree in exact arithmetic; in FP64 they differ by rounding only,
so under the same oracle-spread tolerance), GN/LM cost traces 1e-9 relative in FP64, the Laplacian's exact
minimiser 1e-9, mixed precision 1e-4 relative final cost (5% handles).  The
meshes are Morton-ordered icospheres (the order the lists' caps assume); levels
3 and 5 have 3 and 41 chunks, the last one ragged (642 = 2*256 + 130 and
10242 = 40*256 + 2 vertices)."""
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


def _mesh(level, seed=3, handle_frac=0.05, sigma=0.1, scale=0.2):
    d = w.arap_mesh(level, seed=seed, handle_frac=handle_frac, sigma=sigma)
    x = d["x0"] + scale * np.random.default_rng(seed).normal(size=d["x0"].shape)
    return d, x


def _lap_graph(level, seed=4, w_fit=0.3, w_reg=0.9):
    """The graph Laplacian on a Morton-ordered icosphere (the ARAP workload's
    vertex order), data = rest positions plus noise."""
    m = w.arap_mesh(level, seed=seed)
    A = m["U"] + 0.05 * np.random.default_rng(seed).normal(size=m["U"].shape)
    return dict(energy="laplacian_graph", V=m["V"], edges=m["edges"], A=A, x0=np.zeros_like(A),
                params=dict(w_fit=w_fit, w_reg=w_reg))


def test_form_selection():
    for lev in (1, 3, 5):
        assert make_problem(_mesh(lev)[0], "fp64").pcg_form("fused") == "fused", lev
        assert make_problem(_mesh(lev)[0], "mixed").pcg_form("fused") == "fused", lev
    assert make_problem(_lap_graph(3), "fp64").pcg_form("fused") == "fused"
    assert make_problem(_mesh(3)[0], "fp64").pcg_form("split") == "split"
    # a random graph's rings pass the caps: the split form runs
    rng = np.random.default_rng(1)
    V = 5000
    m = w.arap_mesh(1, seed=1)
    U = rng.normal(size=(3, V))
    C = np.full((3, V), -1e7)
    C[:, :50] = U[:, :50]
    d = dict(energy="arap_mesh", V=V, edges=rng.integers(0, V, size=(15000, 2)).astype(np.int32), U=U, C=C,
             x0=np.concatenate([U, np.zeros((3, V))]), params=m["params"])
    assert make_problem(d, "fp64").pcg_form("fused") == "split"


@pytest.mark.parametrize("level", [3, 5])
@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_pcg_fp64_against_oracle_and_split(level, lam):
    d, x = _mesh(level)
    lin = o.Linearization(o.make_energy(d), x)
    D = lin.damping()
    prob = make_problem(d, "fp64")
    prob.linearize(to_dev(prob, x))
    A = ((lin.JT @ lin.J) + lam * sp.diags(D)).tocsr()
    for L in (1, 2, 3, 10, 25):
        ref, _ = o.pcg(lambda v: lin.apply(v, lam, D), lin.jtf(), lin.minv(True, lam, D), L)
        ref2, _ = o.pcg(lambda v: A @ v, lin.jtf(), lin.minv(True, lam, D), L)
        tol = pcg_tol(ref, ref2)
        got = to_np(prob.pcg(L, lam=lam, variant="fused"))
        assert relmax(got, ref) < tol, (L, relmax(got, ref))
        split = to_np(prob.pcg(L, lam=lam, variant="split"))
        assert relmax(got, split) < tol, (L, relmax(got, split))


def test_pcg_without_preconditioner():
    d, x = _mesh(3, seed=6)
    lin = o.Linearization(o.make_energy(d), x)
    prob = make_problem(d, "fp64")
    prob.linearize(to_dev(prob, x))
    for L in (1, 6):
        ref, _ = o.pcg(lin.apply, lin.jtf(), np.ones(lin.diag.size), L)
        got = to_np(prob.pcg(L, use_precond=False, variant="fused"))
        assert relmax(got, ref) < 1e-9, L


def test_gn_and_lm_fp64():
    d = w.arap_mesh(3, seed=3, handle_frac=0.02, sigma=0.2)
    e = o.make_energy(d)
    xo, costs, acc = o.levenberg_marquardt(e, d["x0"], 5, 20)
    prob = make_problem(d, "fp64")
    assert prob.pcg_form() == "fused"
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="lm", outer_iters=5, pcg_iters=20)
    assert rep["steps_accepted"] == sum(acc)
    assert np.allclose(rep["cost_trace"][:len(costs)], costs, rtol=1e-9, atol=0)
    d2 = w.arap_mesh(5, seed=4, handle_frac=0.05)
    xo, costs = o.gauss_newton(o.make_energy(d2), d2["x0"], 3, 15)
    prob2 = make_problem(d2, "fp64")
    rep = prob2.solve(to_dev(prob2, d2["x0"]), method="gn", outer_iters=3, pcg_iters=15)
    assert np.allclose(rep["cost_trace"], costs, rtol=1e-9, atol=0)


def test_lm_mixed_level5():
    d = w.arap_mesh(5, seed=3, handle_frac=0.05)
    xo, costs, acc = o.levenberg_marquardt(o.make_energy(d), d["x0"], 4, 40)
    prob = make_problem(d, "mixed")
    assert prob.pcg_form() == "fused"
    rep = prob.solve(to_dev(prob, d["x0"]), method="lm", outer_iters=4, pcg_iters=40)
    assert rep["steps_accepted"] == sum(acc)
    assert abs(rep["cost_final"] - costs[-1]) <= 1e-4 * costs[-1]


def test_laplacian_graph_reaches_the_minimiser():
    """A linear energy: GN with enough inner iterations lands on the solution
    of (w_f^2 I + w_r^2 L) x = w_f^2 A (scipy, from the edge list directly),
    also with iterations past convergence (the stop on a non-positive
    curvature, if it comes, keeps d)."""
    d = _lap_graph(3)
    V, E = d["V"], d["edges"]
    wf, wr = d["params"]["w_fit"], d["params"]["w_reg"]
    Inc = sp.csr_matrix((np.r_[np.ones(len(E)), -np.ones(len(E))],
                         (np.r_[np.arange(len(E)), np.arange(len(E))], np.r_[E[:, 0], E[:, 1]])), shape=(len(E), V))
    M = (wf ** 2) * sp.eye(V) + (wr ** 2) * (Inc.T @ Inc)
    x_star = np.stack([spla.spsolve(M.tocsc(), (wf ** 2) * d["A"][c]) for c in range(3)])
    prob = make_problem(d, "fp64")
    assert prob.pcg_form() == "fused"
    for L in (200, 701):
        xt = to_dev(prob, d["x0"])
        prob.solve(xt, method="gn", outer_iters=1, pcg_iters=L)
        assert np.abs(to_np(xt) - x_star.ravel()).max() < 1e-9 * np.abs(x_star).max(), L


def test_laplacian_graph_pcg_fp64():
    d = _lap_graph(5)
    x = np.random.default_rng(2).normal(size=d["x0"].size)
    lin = o.Linearization(o.make_energy(d), x)
    prob = make_problem(d, "fp64")
    assert prob.pcg_form() == "fused"
    prob.linearize(to_dev(prob, x))
    A = (lin.JT @ lin.J).tocsr()
    for L in (1, 4, 15):
        ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), L)
        ref2, _ = o.pcg(lambda v: A @ v, lin.jtf(), lin.minv(True), L)
        assert relmax(to_np(prob.pcg(L, variant="fused")), ref) < pcg_tol(ref, ref2), L


def test_hub_vertex_and_isolated_vertices():
    """A vertex joined to 199 others spread over three chunks (each other
    chunk has the hub in its one-ring and the hub's other neighbours in its
    two-ring) and vertices without edges (zero diagonal, M^-1 = 0)."""
    rng = np.random.default_rng(7)
    V = 600
    U = rng.normal(size=(3, V))
    hub = np.array([[0, 3 * k] for k in range(1, 200)], np.int32)
    ring = np.array([[k, k + 1] for k in range(201, 499)], np.int32)
    edges = np.concatenate([hub, ring])
    C = np.full((3, V), -1e7)
    h = rng.choice(V, 30, replace=False)
    C[:, h] = U[:, h] + 0.1 * rng.normal(size=(3, 30))
    d = dict(energy="arap_mesh", V=V, edges=edges, U=U, C=C, x0=np.concatenate([U, np.zeros((3, V))]),
             params=dict(w_fit=10.0, w_reg=1.0))
    x = d["x0"] + 0.1 * rng.normal(size=d["x0"].shape)
    lin = o.Linearization(o.make_energy(d), x)
    prob = make_problem(d, "fp64")
    assert prob.pcg_form() == "fused"
    prob.linearize(to_dev(prob, x))
    A = (lin.JT @ lin.J).tocsr()
    for L in (1, 5, 12):
        ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), L)
        ref2, _ = o.pcg(lambda v: A @ v, lin.jtf(), lin.minv(True), L)
        assert relmax(to_np(prob.pcg(L, variant="fused")), ref) < pcg_tol(ref, ref2), L


def test_level7_mixed_against_split():
    """The benchmark's level-7 mesh (163,842 vertices, 641 chunks) in mixed
    precision: a whole LM solve in the fused form against the split form of
    the same problem (5% handles, where FP32 rounding does not decide the
    result: the two stay within 1e-4 in final cost and take the same steps)."""
    d = w.arap_mesh(7, seed=3, handle_frac=0.05)
    prob = make_problem(d, "mixed")
    assert prob.pcg_form() == "fused"
    reps = {}
    for v in ("fused", "split"):
        xt = to_dev(prob, d["x0"])
        reps[v] = prob.solve(xt, method="lm", outer_iters=4, pcg_iters=40, pcg_variant=v)
    assert reps["fused"]["steps_accepted"] == reps["split"]["steps_accepted"]
    assert abs(reps["fused"]["cost_final"] - reps["split"]["cost_final"]) <= 1e-4 * reps["split"]["cost_final"]


def test_graph_replay_and_repeat_bits():
    d, _ = _mesh(5, seed=9)
    prob = make_problem(d, "mixed")
    x0 = to_dev(prob, d["x0"])
    x = x0.clone()
    out = []
    for _ in range(4):
        x.copy_(x0)
        prob.solve(x, method="lm", outer_iters=3, pcg_iters=20, report=False)
        torch.cuda.synchronize()
        out.append(x.cpu().clone())
    assert all(torch.equal(out[0], t) for t in out[1:])
