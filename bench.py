"""Benchmark of the matrix-free GN PCG path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one whole solve: ARAP image warping on a 1024 x 1024 pixel grid
(3 unknowns per pixel, 8,192 positional constraints), Gauss-Newton 10 outer x 50
PCG iterations, mixed precision (FP32 bulk, FP64 dot products and costs).  Inputs
are seeded and synthetic and already resident on the GPU when timing starts; each
step restarts the solve from the same initial unknowns (a 12 MB device copy).

Printed: one JSON line.  ``value`` is PCG iterations per second over whole solves.
``roofline`` rates one PCG iteration, timed live with HIP events on the library's
stream around the PCG phases, against MI355X's 8 TB/s HBM peak, counting the
algorithmic bytes of an iteration (p, d and r each read and written once per
unknown, plus the per-pixel angle, rest position and flags).  ``cpu_baseline`` is the
FP64 oracle (explicit sparse Jacobian, scipy) on one outer iteration of the same
workload on the host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WARP = dict(W=1024, H=1024, seed=2, outer=10, pcg=50)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def warp_bytes_per_iter(n):
    """Algorithmic bytes of one PCG iteration of the mixed-precision warp path:
    p, d, r (3 unknowns per pixel, FP32) each read and written once = 24 B per
    unknown, plus per pixel the angle (4 B), rest position (8 B) and flags (1 B)."""
    return 24 * 3 * n + 13 * n


def cpu_baseline(d, pcg_iters):
    import oracle
    e = oracle.make_energy(d)
    t0 = time.perf_counter()
    lin = oracle.Linearization(e, d["x0"])
    oracle.pcg(lin.apply, lin.jtf(), lin.minv(True), pcg_iters)
    dt = time.perf_counter() - t0
    return {"value": pcg_iters / dt, "unit": "PCG iters/s", "cores": 1, "kind": "oracle",
            "sample": f"one GN outer iteration (explicit Jacobian assembly + {pcg_iters} PCG "
                      f"iterations, FP64, scipy CSR, single thread) of the same 1024x1024 warp; "
                      f"{dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path is single-GPU; see the design notes on sharding)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1604_06525_amd as pkg
    import workloads
    from workloads.layout import problem_args

    dev = torch.device("cuda:0")
    d = workloads.arap_warp(WARP["W"], WARP["H"], seed=WARP["seed"])
    energy, arrs, params, dims = problem_args(d, np.float32)
    t_arrs = [torch.from_numpy(a).to(dev) for a in arrs]
    prob = pkg.Problem(energy, t_arrs, params, precision="mixed", **dims)
    x0 = torch.from_numpy(np.ascontiguousarray(d["x0"].reshape(3, -1).astype(np.float32))).to(dev)
    x = x0.clone()
    sp = pkg.default_params(method="gn", outer_iters=WARP["outer"], pcg_iters=WARP["pcg"])

    def step():
        x.copy_(x0)
        prob.solve(x, params=sp, report=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    prob.profile_enable(True)
    prob.profile_read()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    pcg_ms, pcg_iters = prob.profile_read()
    prob.profile_enable(False)
    rep = prob.solve(x.copy_(x0), params=sp)

    iters = args.steps * WARP["outer"] * WARP["pcg"]
    n = WARP["W"] * WARP["H"]
    iter_us = 1e3 * pcg_ms / pcg_iters
    bpi = warp_bytes_per_iter(n)
    achieved = bpi / (iter_us * 1e-6) / 1e9
    out = {
        "metric": "PCG iters/s + HBM GB/s fraction",
        "value": iters / (total_ms / 1e3),
        "unit": "PCG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "arap_warp_1024x1024_gn10x50_mixed", "grid": [WARP["W"], WARP["H"]],
                   "unknowns": 3 * n, "outer_iters": WARP["outer"], "pcg_iters": WARP["pcg"],
                   "precision": "mixed: FP32 bulk, FP64 dot products and costs", "seed": WARP["seed"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "unit_of_work": "one PCG iteration = one k_fused launch",
                     "bytes_per_iter": bpi, "iter_us": iter_us},
        "pcg_phase_iters_per_s": pcg_iters / (pcg_ms / 1e3),
        "cost_initial": rep["cost_initial"],
        "cost_final": rep["cost_final"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, WARP["pcg"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
