"""The batching server (opt_server_*) against single-problem solves.

A request served in any batch must give the same bits as opt_solve on that
problem alone (same unknowns after the solve, same report), because each
request keeps its own grid, partial sums and reduction order.  The alone solves
are themselves checked against the FP64 oracle by the other GPU tests.
"""
import numpy as np
import pytest
import torch

import paper_1604_06525_amd as pkg
import workloads as w
from workloads.layout import problem_args
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


DEV = torch.device("cuda:0")


def _request(d, precision, **solve):
    """Device tensors of a workload: (energy, arrays, params, dims, x0)."""
    dt = np.float64 if precision == "fp64" else np.float32
    energy, arrs, params, dims = problem_args(d, dt)
    t_arrs = [torch.from_numpy(a).to(DEV) for a in arrs]
    if "edges" in dims:
        dims = dict(dims, edges=torch.from_numpy(dims["edges"]).to(DEV))
    x0 = torch.from_numpy(np.ascontiguousarray(np.asarray(d["x0"], dt).reshape(-1))).to(DEV)
    return dict(energy=energy, arrays=t_arrs, params=params, dims=dims, x0=x0, precision=precision,
                solve=solve)


def _alone(r):
    # the launch shape the server gives the request (tuning entries, served form)
    prob = pkg.Problem(r["energy"], r["arrays"], r["params"], precision=r["precision"], tuning="served",
                       **r["dims"])
    x = r["x0"].clone().reshape(prob.channels, -1)
    rep = prob.solve(x, **r["solve"])
    return x.reshape(-1), rep


def _mix():
    """Requests of every energy, both precisions, GN and LM, both PCG forms (the
    IRLS energy with both)."""
    return [
        _request(w.arap_warp(33, 17, seed=1, n_constraints=12, margin=2), "fp64",
                 method="gn", outer_iters=3, pcg_iters=10),
        _request(w.arap_warp(130, 70, seed=2, n_constraints=60, margin=2, mask="random"), "mixed",
                 method="lm", outer_iters=4, pcg_iters=12),
        _request(w.poisson_edit(97, 41, seed=5), "mixed", method="gn", outer_iters=2, pcg_iters=15),
        _request(w.poisson_edit(64, 64, seed=6), "fp64", method="gn", outer_iters=3, pcg_iters=9,
                 pcg_variant="split"),
        _request(w.optical_flow(80, 60, seed=4), "mixed", method="gn", outer_iters=3, pcg_iters=8),
        _request(w.shape_from_shading(70, 50, seed=2), "fp64", method="gn", outer_iters=2, pcg_iters=10),
        _request(w.arap_mesh(2, seed=3, handle_frac=0.05, sigma=0.1), "fp64", method="lm",
                 outer_iters=3, pcg_iters=10),
        _request(w.arap_mesh(3, seed=4, handle_frac=0.05, sigma=0.1), "mixed", method="lm",
                 outer_iters=5, pcg_iters=8),
        _request(w.arap_warp(64, 64, seed=7, n_constraints=40, margin=2), "mixed",
                 method="gn", outer_iters=0, pcg_iters=5),
        _request(w.lp_smooth(90, 70, seed=8, p=1.0, eps=0.02), "mixed", method="gn", outer_iters=4,
                 pcg_iters=12),
        _request(w.lp_smooth(40, 33, seed=9, p=0.8, eps=0.05), "fp64", method="gn", outer_iters=3,
                 pcg_iters=10, pcg_variant="split"),
    ]


def _submit(sv, r):
    x = r["x0"].clone()
    t = sv.submit(r["energy"], r["arrays"], x, r["params"], precision=r["precision"], **r["dims"],
                  **r["solve"])
    return t, x


def _same(rep_a, rep_b):
    for k in ("cost_initial", "cost_final", "outer_done", "steps_accepted", "cost_trace"):
        assert rep_a[k] == rep_b[k], k


def _run_until_done(sv, tickets, max_steps=100):
    out = {}
    for _ in range(max_steps):
        sv.step()
        for t in list(tickets):
            rep = sv.poll(t)
            if rep is not None:
                out[t] = rep
                tickets.remove(t)
        if not tickets:
            return out
    raise AssertionError("server did not finish")


def test_batch_equals_alone():
    reqs = _mix()
    alone = [_alone(r) for r in reqs]
    sv = pkg.Server(256 << 20, max_slots=16)
    subs = [_submit(sv, r) for r in reqs]
    assert all(t is not None for t, _ in subs)
    out = _run_until_done(sv, [t for t, _ in subs])
    for (t, x), (xa, repa) in zip(subs, alone):
        assert torch.equal(x, xa)
        _same(out[t], repa)
    assert sv.info() == (0, (256 << 20) - pkg.Server.reserved_bytes(16))


def test_staggered_admission_equals_alone():
    """Requests join while others run: the batch changes every step."""
    reqs = _mix()
    alone = [_alone(r) for r in reqs]
    sv = pkg.Server(256 << 20, max_slots=4)
    pending = list(range(len(reqs)))
    live, results, xs = {}, {}, {}
    for _ in range(200):
        while pending:
            t, x = _submit(sv, reqs[pending[0]])
            if t is None:
                break
            live[t] = pending.pop(0)
            xs[live[t]] = x
        sv.step()
        for t in list(live):
            rep = sv.poll(t)
            if rep is not None:
                results[live.pop(t)] = rep
        if not pending and not live:
            break
    assert len(results) == len(reqs)
    for k, (xa, repa) in enumerate(alone):
        assert torch.equal(xs[k], xa)
        _same(results[k], repa)


def test_admission_limits_and_reuse():
    r = _request(w.arap_warp(200, 150, seed=3, n_constraints=100, margin=2), "mixed",
                 method="gn", outer_iters=2, pcg_iters=5)
    need = pkg.workspace_size(r["energy"], r["arrays"], r["params"], precision="mixed", **r["dims"])
    # room for one request, not two
    arena = pkg.Server.reserved_bytes(8) + need + need // 2
    sv = pkg.Server(arena, max_slots=8)
    t1, x1 = _submit(sv, r)
    t2, _ = _submit(sv, r)
    assert t1 is not None and t2 is None
    out = _run_until_done(sv, [t1])
    xa, repa = _alone(r)
    assert torch.equal(x1, xa)
    _same(out[t1], repa)
    # the range is free again
    t3, x3 = _submit(sv, r)
    assert t3 is not None
    _run_until_done(sv, [t3])
    assert torch.equal(x3, xa)
    # slot limit
    sv2 = pkg.Server(64 << 20, max_slots=2)
    small = _request(w.poisson_edit(32, 32, seed=1), "mixed", outer_iters=1, pcg_iters=3)
    ts = [_submit(sv2, small)[0] for _ in range(3)]
    assert ts[0] is not None and ts[1] is not None and ts[2] is None


def test_cancel_and_unknown_ticket():
    reqs = _mix()[:3]
    sv = pkg.Server(128 << 20, max_slots=8)
    subs = [_submit(sv, r) for r in reqs]
    sv.step()
    held, free_before = sv.info()
    assert held == 3
    sv.cancel(subs[1][0])
    sv.wait()
    held, free_after = sv.info()
    assert held == 2 and free_after > free_before
    out = _run_until_done(sv, [subs[0][0], subs[2][0]])
    for k in (0, 2):
        xa, repa = _alone(reqs[k])
        assert torch.equal(subs[k][1], xa)
        _same(out[subs[k][0]], repa)
    with pytest.raises(pkg.OptError):
        sv.poll(subs[0][0])
    with pytest.raises(pkg.OptError):
        sv.cancel(12345)


def test_lm_early_stop_equals_alone():
    """An LM request whose radius falls below its minimum leaves early, with the
    same report as the single-problem solve, and both match the oracle, which
    stops there too.  A radius cap below the minimum ends the solve right after
    its first, accepted, step: that step must be applied exactly once."""
    import oracle as o
    d = w.arap_warp(48, 40, seed=5, n_constraints=20, margin=2)
    prm = dict(lm_radius0=2.0, lm_radius_min=1.0, lm_radius_max=0.5)
    r = _request(d, "fp64", method="lm", outer_iters=6, pcg_iters=6, **prm)
    xa, repa = _alone(r)
    xo, costs, acc = o.levenberg_marquardt(o.make_energy(d), d["x0"], 6, 6,
                                           o.LMParams(radius0=2.0, radius_min=1.0, radius_max=0.5))
    assert acc == [True]
    assert repa["outer_done"] == 1 and repa["steps_accepted"] == 1
    assert np.allclose(repa["cost_trace"][:1], costs[:1], rtol=1e-9, atol=0)
    assert abs(repa["cost_final"] - costs[-1]) <= 1e-9 * costs[-1]
    assert np.abs(xa.cpu().numpy() - np.asarray(xo).ravel()).max() < 1e-9
    sv = pkg.Server(64 << 20, max_slots=4)
    t, x = _submit(sv, r)
    out = _run_until_done(sv, [t])
    assert torch.equal(x, xa)
    _same(out[t], repa)


def test_lm_radius_below_minimum_does_nothing():
    """An LM solve whose initial radius is already below its minimum takes no
    iteration (as the oracle), alone and served."""
    import oracle as o
    d = w.arap_warp(40, 24, seed=6, n_constraints=10, margin=2)
    r = _request(d, "fp64", method="lm", outer_iters=3, pcg_iters=4, lm_radius0=0.5, lm_radius_min=1.0)
    xa, repa = _alone(r)
    xo, costs, acc = o.levenberg_marquardt(o.make_energy(d), d["x0"], 3, 4,
                                           o.LMParams(radius0=0.5, radius_min=1.0))
    assert acc == [] and repa["outer_done"] == 0 and repa["steps_accepted"] == 0
    assert torch.equal(xa, r["x0"])
    assert abs(repa["cost_final"] - costs[0]) <= 1e-12 * costs[0]
    assert repa["cost_trace"] == [repa["cost_final"]] * 4
    sv = pkg.Server(64 << 20, max_slots=2)
    t, x = _submit(sv, r)
    out = _run_until_done(sv, [t])
    assert torch.equal(x, xa)
    _same(out[t], repa)


def test_graph_submit_does_not_wait_for_steps_in_flight():
    """Admitting a mesh copies its edge list behind the work on the server's
    stream and builds its lists at a later step: submit returns without waiting
    for the steps already enqueued (here about three outer iterations of a
    4096^2 warp, tens of milliseconds of GPU work)."""
    import time
    big = _request(w.arap_warp(4096, 4096, seed=9, n_constraints=2000, margin=8), "mixed",
                   method="gn", outer_iters=3, pcg_iters=50)
    mesh = _request(w.arap_mesh(4, seed=3, handle_frac=0.05, sigma=0.1), "mixed", method="lm",
                    outer_iters=3, pcg_iters=10)
    xa, repa = _alone(mesh)
    sv = pkg.Server(3 << 30, max_slots=4)
    tb, _ = _submit(sv, big)
    for _ in range(3):
        sv.step()
    torch.cuda.synchronize()  # (nothing else of ours is queued; the server's steps run on its stream)
    tb2, _ = _submit(sv, big)
    for _ in range(3):
        sv.step()  # three steps of the second warp in flight
    t0 = time.perf_counter()
    tm, xm = _submit(sv, mesh)
    dt = time.perf_counter() - t0
    out = _run_until_done(sv, [tb, tb2, tm], max_steps=50)
    assert torch.equal(xm, xa)
    _same(out[tm], repa)
    assert dt < 0.02, f"submit took {dt * 1e3:.1f} ms"


def test_invalid_edge_list_is_dropped_at_a_later_step():
    d = w.arap_mesh(2, seed=3)
    d["edges"] = d["edges"].copy()
    d["edges"][7, 0] = d["V"] + 5
    r = _request(d, "mixed", method="lm", outer_iters=2, pcg_iters=5)
    ok = _request(w.arap_warp(40, 30, seed=2, n_constraints=10, margin=2), "mixed", method="gn",
                  outer_iters=2, pcg_iters=5)
    xa, repa = _alone(ok)
    sv = pkg.Server(64 << 20, max_slots=4)
    tbad, _ = _submit(sv, r)
    tok, xok = _submit(sv, ok)
    assert tbad is not None
    for _ in range(10):
        sv.step()
    with pytest.raises(pkg.OptError) as ei:
        sv.poll(tbad)
    assert ei.value.code == pkg.OPT_EINVAL and "outside" in str(ei.value)
    out = _run_until_done(sv, [tok])
    assert torch.equal(xok, xa)
    _same(out[tok], repa)


def test_nonfinite_request_is_isolated():
    """A request whose data holds a NaN reports OPT_ENUMERIC; the requests
    batched with it (same energy kind, same launches) give the bits they give
    alone."""
    good = [_request(w.arap_warp(64, 48, seed=s, n_constraints=20, margin=2), "mixed", method="gn",
                     outer_iters=3, pcg_iters=10) for s in (11, 12)]
    d = w.arap_warp(64, 48, seed=13, n_constraints=20, margin=2)
    d["U"] = d["U"].copy()
    d["U"][0, 20, 30] = np.nan  # one rest position: its regularisers are NaN
    bad = _request(d, "mixed", method="gn", outer_iters=3, pcg_iters=10)
    alone = [_alone(r) for r in good]
    sv = pkg.Server(128 << 20, max_slots=4)
    subs = [_submit(sv, good[0]), _submit(sv, bad), _submit(sv, good[1])]
    tickets = [t for t, _ in subs]
    out = _run_until_done(sv, list(tickets))
    assert out[tickets[1]]["code"] == pkg.OPT_ENUMERIC
    for (t, x), (xa, repa) in zip([subs[0], subs[2]], alone):
        assert torch.equal(x, xa)
        _same(out[t], repa)
