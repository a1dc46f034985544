"""opt_solve_scratch, the entry point that allocates no device memory, against
opt_problem_create + opt_solve on the same problems.

Both run the same kernels with the same (automatic) launch shape, so the
unknowns and the report must agree bit for bit.  Each case makes two scratch
calls in a row, the second on a smaller problem, so that whatever the first
call left in the shared scratch array cannot leak into the second result.
"""
import numpy as np
import pytest
import torch

import paper_1604_06525_amd as pkg
import workloads as w
from workloads.layout import problem_args
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _tensors(d, precision):
    dt = np.float64 if precision == "fp64" else np.float32
    energy, arrs, params, dims = problem_args(d, dt)
    t_arrs = [torch.from_numpy(a).to(DEV) for a in arrs]
    if "edges" in dims:
        dims = dict(dims, edges=torch.from_numpy(dims["edges"]).to(DEV))
    x0 = torch.from_numpy(np.ascontiguousarray(np.asarray(d["x0"], dt).reshape(-1))).to(DEV)
    return energy, t_arrs, params, dims, x0


def _reference(d, precision, solve):
    energy, arrs, params, dims, x0 = _tensors(d, precision)
    prob = pkg.Problem(energy, arrs, params, precision=precision, tuning=None, **dims)
    x = x0.clone().reshape(prob.channels, -1)
    rep = prob.solve(x, **solve)
    torch.cuda.synchronize()
    return x.reshape(-1).cpu(), rep


def _scratch(d, precision, solve, report=True):
    energy, arrs, params, dims, x0 = _tensors(d, precision)
    x = x0.clone()
    rep = pkg.solve_scratch(energy, arrs, x, params, precision=precision, report=report, **dims, **solve)
    torch.cuda.synchronize()
    return x.cpu(), rep


def _same(a, b):
    xa, ra = a
    xb, rb = b
    assert torch.equal(xa, xb), f"unknowns differ: max |dx| {(xa.double() - xb.double()).abs().max().item():.3e}"
    for k in ("cost_initial", "cost_final", "outer_done", "steps_accepted", "cost_trace"):
        assert ra[k] == rb[k], (k, ra[k], rb[k])


CASES = {
    # (first workload, second smaller workload, precision, solve parameters)
    "warp_mixed_gn_fused": (
        lambda: w.arap_warp(150, 110, seed=2, n_constraints=80, margin=4),
        lambda: w.arap_warp(61, 37, seed=3, n_constraints=20, margin=3),
        "mixed", dict(method="gn", outer_iters=3, pcg_iters=12)),
    "sfs_fp64_gn": (
        lambda: w.shape_from_shading(90, 70, seed=2),
        lambda: w.shape_from_shading(40, 33, seed=4),
        "fp64", dict(method="gn", outer_iters=2, pcg_iters=10)),
    "poisson_mixed_split": (
        lambda: w.poisson_edit(120, 90, seed=5),
        lambda: w.poisson_edit(50, 41, seed=6),
        "mixed", dict(method="gn", outer_iters=2, pcg_iters=9, pcg_variant="split")),
    "mesh_lm": (
        lambda: w.arap_mesh(3, seed=3, handle_frac=0.05, sigma=0.1),
        lambda: w.arap_mesh(2, seed=4, handle_frac=0.05, sigma=0.1),
        "fp64", dict(method="lm", outer_iters=4, pcg_iters=10)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_scratch_matches_workspace_solve(case):
    big, small, precision, solve = CASES[case]
    d1, d2 = big(), small()
    s1 = _scratch(d1, precision, solve)
    s2 = _scratch(d2, precision, solve)
    _same(s1, _reference(d1, precision, solve))
    _same(s2, _reference(d2, precision, solve))


def test_scratch_enqueue_only():
    d = w.arap_warp(77, 59, seed=7, n_constraints=30, margin=3)
    solve = dict(method="lm", outer_iters=3, pcg_iters=8)
    x, rep = _scratch(d, "mixed", solve, report=False)
    assert rep is None
    xr, _ = _reference(d, "mixed", solve)
    assert torch.equal(x, xr)


def test_scratch_rejects_a_problem_past_its_size():
    # 2048^2 FP64 warp: about 1.4 GB of workspace, past the 128 MB scratch; the
    # size check runs before any kernel
    W = H = 2048
    U = torch.zeros((2, W * H), dtype=torch.float64, device=DEV)
    mask = torch.zeros(W * H, dtype=torch.uint8, device=DEV)
    x = torch.zeros(3 * W * H, dtype=torch.float64, device=DEV)
    need = pkg.workspace_size("arap_warp", [U, U, mask], [10.0, 1.0], precision="fp64", width=W, height=H)
    assert need > pkg.SCRATCH_BYTES
    with pytest.raises(pkg.OptError) as ei:
        pkg.solve_scratch("arap_warp", [U, U, mask], x, [10.0, 1.0], precision="fp64", width=W, height=H,
                          method="gn", outer_iters=1, pcg_iters=1)
    assert ei.value.code == pkg.OPT_ENOMEM
    assert "static scratch" in str(ei.value)
