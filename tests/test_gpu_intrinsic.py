"""GPU parity of the intrinsic image decomposition (A.2.4, Fig. 33) solved by
IRLS (Sec. 7) against the FP64 oracle: each linearisation freezes one weight per
reflectance edge, and the operators, the PCG and whole IRLS solves must match
the oracle's frozen problem and its IRLS loop.

Tolerances as for the other grid energies: FP64 operators 1e-12 of their
largest entry (the objective 1e-12 relative), FP64 PCG the oracle-spread rule,
FP64 IRLS objective traces 1e-9 relative, mixed precision 1e-4 relative final
objective on FP32-rounded inputs.  The decomposition's null direction (r down,
s up) leaves the objective unchanged; the PCG runs well short of convergence,
so the iterates themselves are compared too."""
import numpy as np
import pytest

import oracle as o
import paper_1604_06525_amd as pkg
import workloads as w
from tests.gpu_util import f32_inputs, make_problem, pcg_tol, relmax, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _case(W, H, seed, p=0.8, eps=0.02, scale=0.05):
    d = w.intrinsic_image(W, H, seed=seed, p=p, eps=eps)
    x = d["x0"].ravel() + scale * np.random.default_rng(seed).normal(size=4 * W * H)
    return d, x


@pytest.mark.parametrize("W,H,p", [(9, 7, 1.0), (70, 53, 0.6), (64, 64, 1.5)])
def test_operators_fp64(W, H, p):
    d, x = _case(W, H, seed=2, p=p)
    e = o.make_energy(d)
    e.freeze(x)
    lin = o.Linearization(e, x)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, x)
    phi = e.objective(x)
    assert abs(prob.cost(xt) - phi) <= 1e-12 * phi
    assert abs(prob.linearize(xt) - phi) <= 1e-12 * phi
    b, dg = prob.eval_jtf()
    assert relmax(to_np(b), lin.jtf()) < 1e-12
    assert relmax(to_np(dg), lin.diag) < 1e-12
    v = np.random.default_rng(3).normal(size=4 * W * H)
    assert relmax(to_np(prob.apply_jtj(to_dev(prob, v))), lin.apply(v)) < 1e-12


@pytest.mark.parametrize("variant", ["fused", "split"])
def test_pcg_fp64(variant):
    d, x = _case(41, 30, seed=4)
    e = o.make_energy(d)
    e.freeze(x)
    lin = o.Linearization(e, x)
    A = (lin.JT @ lin.J).tocsr()
    prob = make_problem(d, "fp64")
    prob.linearize(to_dev(prob, x))
    for L in (1, 2, 7, 20):
        ref, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), L)
        ref2, _ = o.pcg(lambda v: A @ v, lin.jtf(), lin.minv(True), L)
        assert relmax(to_np(prob.pcg(L, variant=variant)), ref) < pcg_tol(ref, ref2), L


@pytest.mark.parametrize("variant", ["fused", "split"])
@pytest.mark.parametrize("p", [1.0, 0.5])
def test_irls_fp64(variant, p):
    d = w.intrinsic_image(48, 37, seed=5, p=p, eps=0.02)
    x_ref, objs = o.irls(o.make_energy(d), d["x0"], 5, 25)
    prob = make_problem(d, "fp64")
    xt = to_dev(prob, d["x0"])
    rep = prob.solve(xt, method="gn", outer_iters=5, pcg_iters=25, pcg_variant=variant)
    assert np.allclose(rep["cost_trace"], objs, rtol=1e-9, atol=0)
    assert relmax(to_np(xt) - d["x0"].ravel(), x_ref - d["x0"].ravel()) < 1e-8


def test_irls_mixed():
    d = w.intrinsic_image(150, 110, seed=7, p=0.8, eps=0.02)
    d32 = f32_inputs(d)
    x_ref, objs = o.irls(o.make_energy(d32), d32["x0"], 6, 30)
    prob = make_problem(d, "mixed")
    rep = prob.solve(to_dev(prob, d32["x0"]), method="gn", outer_iters=6, pcg_iters=30)
    assert abs(rep["cost_final"] - objs[-1]) <= 1e-4 * objs[-1]
    # PCG from d = 0 lowers the reweighted quadratic, which majorises the objective
    assert all(b <= a * (1 + 1e-6) for a, b in zip(rep["cost_trace"], rep["cost_trace"][1:]))


def test_lm_is_refused():
    d, _ = _case(20, 10, seed=8)
    prob = make_problem(d, "fp64")
    with pytest.raises(pkg.OptError) as ei:
        prob.solve(to_dev(prob, d["x0"]), method="lm", outer_iters=2, pcg_iters=5)
    assert ei.value.code == pkg.OPT_EUNSUPPORTED
