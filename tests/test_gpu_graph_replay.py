"""Graph replay of repeated solves (opt_problem_set_graph_replay) against the
same solves launched kernel by kernel.

From the second opt_solve with the same unknowns pointer, parameters and tuning,
the library records the solve's launches as one HIP graph and replays it.  Every
replay must give the bits of the eager solve, also when other calls on the
problem (cost, linearise, J^T F, a solve with other parameters) ran between
replays and left other argument rows behind, and with host synchronisations
between them.
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


def _problem(d, precision, graphs):
    dt = np.float64 if precision == "fp64" else np.float32
    energy, arrs, params, dims = problem_args(d, dt)
    t_arrs = [torch.from_numpy(a).to(DEV) for a in arrs]
    if "edges" in dims:
        dims = dict(dims, edges=torch.from_numpy(dims["edges"]).to(DEV))
    prob = pkg.Problem(energy, t_arrs, params, precision=precision, tuning=None, **dims)
    prob.set_graph_replay(graphs)
    x0 = torch.from_numpy(np.ascontiguousarray(np.asarray(d["x0"], dt).reshape(prob.channels, -1))).to(DEV)
    return prob, x0


CASES = {
    "warp_mixed_gn": (lambda: w.arap_warp(96, 80, seed=2, n_constraints=40, margin=3), "mixed",
                      dict(method="gn", outer_iters=3, pcg_iters=12)),
    "warp_mixed_lm": (lambda: w.arap_warp(70, 64, seed=3, n_constraints=30, margin=3), "mixed",
                      dict(method="lm", outer_iters=4, pcg_iters=10)),
    "sfs_fp64_gn": (lambda: w.shape_from_shading(64, 48, seed=2), "fp64",
                    dict(method="gn", outer_iters=2, pcg_iters=10)),
    "flow_mixed_split": (lambda: w.optical_flow(72, 56, seed=4), "mixed",
                         dict(method="gn", outer_iters=2, pcg_iters=8, pcg_variant="split")),
    "mesh_mixed_lm": (lambda: w.arap_mesh(3, seed=3, handle_frac=0.05, sigma=0.1), "mixed",
                      dict(method="lm", outer_iters=4, pcg_iters=10)),
}


def _eager(d, precision, solve):
    prob, x0 = _problem(d, precision, graphs=False)
    x = x0.clone()
    rep = prob.solve(x, **solve)
    torch.cuda.synchronize()
    return x.cpu(), rep


@pytest.mark.parametrize("case", sorted(CASES))
def test_replays_equal_eager_solve(case):
    gen, precision, solve = CASES[case]
    d = gen()
    x_ref, rep_ref = _eager(d, precision, solve)
    prob, x0 = _problem(d, precision, graphs=True)
    x = x0.clone()
    other = dict(solve, pcg_iters=solve["pcg_iters"] + 3)
    for k in range(5):
        x.copy_(x0)
        # calls 0 and 1 run eagerly and the second records the graph; 2..4 replay it
        rep = prob.solve(x, **solve)
        torch.cuda.synchronize()
        assert torch.equal(x.cpu(), x_ref), f"solve {k}: unknowns differ from the eager solve"
        for key in ("cost_initial", "cost_final", "outer_done", "steps_accepted", "cost_trace"):
            assert rep[key] == rep_ref[key], (k, key)
        # the program's own work between replays, touching other argument rows
        y = x0.clone()
        prob.cost(y)
        prob.linearize(y)
        prob.eval_jtf()
        if k == 2:
            # a solve with other parameters, on another tensor: eager, and it
            # must not disturb the recorded graph
            z = x0.clone()
            prob.solve(z, **other)
        torch.cuda.synchronize()


def test_replay_off_and_on_again():
    gen, precision, solve = CASES["warp_mixed_gn"]
    d = gen()
    x_ref, _ = _eager(d, precision, solve)
    prob, x0 = _problem(d, precision, graphs=True)
    x = x0.clone()
    for on in (True, True, False, True, True, True):
        prob.set_graph_replay(on)
        x.copy_(x0)
        prob.solve(x, report=False, **solve)
        torch.cuda.synchronize()
        assert torch.equal(x.cpu(), x_ref)
