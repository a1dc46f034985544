"""Benchmark of the matrix-free GN PCG path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --serve [--serve-requests N]
    python bench.py --configs all
    python bench.py --accuracy [--configs NAME,...]

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

``--configs all`` measures every configuration of the measurement table instead
(ARAP warp 64^2 FP64 and 1024^2 mixed/FP64, shape from shading 1024^2, ARAP
icosphere meshes of levels 7 and 8, optical flow 1920x1080 mixed/FP64, Poisson
1024^2, and the 1024^2 warp with implicit grid vs explicit graph connectivity):
one JSON line each, not the contract line.

The default run also times the oracle on the host first (``cpu_baseline``: one
outer iteration of the same workload, on one core and in one process per core)
and ends with a compact serving leg: the batching server against plain FIFO
solves on the serving mix at 1.0 and 2.0 x the plain capacity
(``--serve-leg-requests`` per load, 0 skips it).

``--accuracy`` compares the GPU with the FP64 oracle at every configuration's
full size and schedule: relative final-cost error, unknown error (relative to
the oracle's own step from the initial unknowns, and max-abs), accepted LM steps,
and for shape from shading the smoothness-mask flips at every linearisation
point; the oracle's whole-solve time on one thread is reported beside them.

``--serve`` measures the batching server instead: a seeded Poisson-arrival
stream of mixed requests (ARAP warps and Poisson edits on grids of side
128..1024, ARAP icosphere meshes of 10k..164k vertices; mixed precision) is
served at several loads, relative to the measured capacity of plain FIFO
single-problem solves, once by the server (continuous batching, 8 GiB arena) and
once plainly; it prints one JSON line with p50/p99 latency (arrival to result on
the host) and sustained solves/s for both, and whether every request gave
bit-identical unknowns both ways.
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
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-loads", type=str, default="0.25,0.5,0.75,0.9,1.0,1.2")
    ap.add_argument("--configs", type=str, default="",
                    help="'all' or a comma list: per-configuration PCG rates instead of the headline line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run device copies of a known size (to scale memory counters)")
    ap.add_argument("--accuracy", action="store_true",
                    help="GPU final cost and unknowns against the FP64 oracle for every configuration "
                         "(or those named by --configs), at full size and schedule")
    ap.add_argument("--serve-leg-requests", type=int, default=500,
                    help="requests per load of the serving leg of the default run (0: skip the leg)")
    return ap.parse_args()


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "fused_arap_warp_1024_mixed_counters.md")


def measured_traffic(tuning):
    """HBM bytes per fused launch from the committed counter summary (FETCH_SIZE
    and WRITE_SIZE, each scaled by a plain copy's reading), or None when the
    kernel sources or the launch shape differ from those the counters were
    taken on."""
    import hashlib
    if not os.path.exists(TRAFFIC_RECORD):
        return None
    rec = None
    for line in open(TRAFFIC_RECORD):
        if line.strip().startswith("traffic-record:"):
            rec = json.loads(line.split("traffic-record:", 1)[1])
    if rec is None or rec.get("tuning") != tuning:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def warp_bytes_per_iter(n):
    """Algorithmic bytes of one PCG iteration of the mixed-precision warp path:
    p, d, r (3 unknowns per pixel, FP32) each read and written once = 24 B per
    unknown, plus per pixel the angle (4 B), rest position (8 B) and flags (1 B)."""
    return 24 * 3 * n + 13 * n


def _oracle_outer_sample(pcg_iters):
    """One Gauss-Newton outer iteration of the FP64 oracle on the headline warp
    (explicit Jacobian assembly, then pcg_iters PCG iterations with scipy CSR
    products), single thread.  Returns (assembly seconds, PCG seconds)."""
    import oracle
    import workloads
    d = workloads.arap_warp(WARP["W"], WARP["H"], seed=WARP["seed"])
    e = oracle.make_energy(d)
    t0 = time.perf_counter()
    lin = oracle.Linearization(e, d["x0"])
    b, minv = lin.jtf(), lin.minv(True)
    t1 = time.perf_counter()
    oracle.pcg(lin.apply, b, minv, pcg_iters)
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def _host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_pool(n):
    """Worker processes for the oracle, one thread each.  Started before the
    GPU is touched (spawned, not forked)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    return ProcessPoolExecutor(n, mp_context=mp.get_context("spawn"))


CPU_PROCS_MAX = 16


def cpu_baseline(pcg_iters):
    """The FP64 oracle on the host, on samples of the headline workload: one
    outer iteration alone on one core (Jacobian assembly and PCG timed apart),
    then the same sample in one process per core at once (the oracle's
    throughput on all cores: its sparse products use one thread each).  Runs
    before the GPU is used."""
    n = max(1, min(_host_cores(), CPU_PROCS_MAX))
    with _oracle_pool(n) as pool:
        pool.submit(int, 0).result()  # workers up before timing
        asm1, pcg1 = pool.submit(_oracle_outer_sample, pcg_iters).result()
        t0 = time.perf_counter()
        res = list(pool.map(_oracle_outer_sample, [pcg_iters] * n))
        wall = time.perf_counter() - t0
    total = sum(pcg_iters / r[1] for r in res)
    K = WARP["outer"]
    print(f"cpu_baseline: oracle {pcg_iters / pcg1:.2f} PCG iters/s on one core, {total:.1f} on {n}",
          file=sys.stderr, flush=True)
    return {"value": total, "unit": "PCG iters/s", "cores": n, "kind": "oracle",
            "model": _cpu_model(), "host_cores": _host_cores(),
            "sample": f"one GN outer iteration of the same 1024x1024 warp (FP64, explicit Jacobian, "
                      f"scipy CSR, {pcg_iters} PCG iterations) per process: {n} single-thread processes "
                      f"at once ({wall:.1f} s wall), value = their summed PCG iterations/s over the PCG "
                      f"phase only (Jacobian assembly excluded)",
            "one_core": {"pcg_iters_per_s": pcg_iters / pcg1, "jacobian_assembly_s": asm1,
                         "outer_iteration_s": asm1 + pcg1,
                         "solve_s_estimate": K * (asm1 + pcg1),
                         "note": f"solve_s_estimate = {K} outer iterations x (assembly + PCG) of the sample"},
            "all_cores": {"processes": n, "pcg_iters_per_s_total": total,
                          "jacobian_assembly_s_mean": float(np.mean([r[0] for r in res])),
                          "pcg_s_mean": float(np.mean([r[1] for r in res]))}}


COPY_BYTES = 2 << 30  # far larger than the 256 MB Infinity Cache


def copy_calibration(reps=5):
    """Device-to-device copies of COPY_BYTES each: a kernel that reads and writes
    a known number of bytes, against which the memory counters of a profiled run
    are scaled.  Also reports the copy's bandwidth (read + write bytes / time)."""
    import torch
    dev = torch.device("cuda:0")
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "reps": reps,
                      "ms_per_copy": ms, "GB_per_s": 2 * COPY_BYTES / (ms * 1e-3) / 1e9}), flush=True)


SERVE_ARENA = 8 << 30
SERVE_SLOTS = 64


def _serve_pool(torch, pkg, dev):
    import workloads
    from workloads.layout import problem_args
    from workloads.serving import SCHEDULE, pool_spec
    entries = []
    for spec in pool_spec():
        kind, size, seed = spec["kind"], spec["size"], spec["seed"]
        if kind == "arap_warp":
            d = workloads.arap_warp(size, size, seed=seed)
        elif kind == "poisson":
            d = workloads.poisson_edit(size, size, seed=seed)
        else:
            d = workloads.arap_mesh(size, seed=seed)
        energy, arrs, params, dims = problem_args(d, np.float32)
        arrays = [torch.from_numpy(a).to(dev) for a in arrs]
        if "edges" in dims:
            dims = dict(dims, edges=torch.from_numpy(dims["edges"]).to(dev))
        x0 = torch.from_numpy(np.ascontiguousarray(np.asarray(d["x0"], np.float32).reshape(-1))).to(dev)
        method, K, L = SCHEDULE[kind]
        sp = pkg.default_params(method=method, outer_iters=K, pcg_iters=L)
        # plain solves run the shape the server gives the request, so that the
        # two legs can be compared bit for bit
        plain = pkg.Problem(energy, arrays, params, precision="mixed", tuning="served", **dims)
        entries.append(dict(spec=spec, energy=energy, arrays=arrays, params=params, dims=dims, x0=x0,
                            sp=sp, plain=plain))
    return entries


def _pct(v, q):
    return float(np.percentile(np.asarray(v) * 1e3, q))


def _run_plain(entries, arrivals, which, keep):
    lat, xs = [], {}
    t0 = time.perf_counter()
    for k in range(len(arrivals)):
        wait = arrivals[k] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        e = entries[which[k]]
        x = e["x0"].clone().reshape(e["plain"].channels, -1)
        e["plain"].solve(x, params=e["sp"], report=True)
        lat.append(time.perf_counter() - t0 - arrivals[k])
        if keep:
            xs[k] = x.reshape(-1)
    span = time.perf_counter() - t0
    return lat, span, xs


def _run_batched(pkg, entries, arrivals, which, keep):
    sv = pkg.Server(SERVE_ARENA, max_slots=SERVE_SLOTS)
    n = len(arrivals)
    lat = [None] * n
    xs, live, queue = {}, {}, []
    nxt, done, steps, held_sum = 0, 0, 0, 0
    t0 = time.perf_counter()
    while done < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            queue.append(nxt)
            nxt += 1
        while queue:
            k = queue[0]
            e = entries[which[k]]
            x = e["x0"].clone()
            t = sv.submit(e["energy"], e["arrays"], x, e["params"], precision="mixed", **e["dims"],
                          solve_params=e["sp"])
            if t is None:
                break
            queue.pop(0)
            live[t] = (k, x)
        if not live:
            wait = arrivals[nxt] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            continue
        held_sum += len(live)
        steps += 1
        sv.step()
        now = time.perf_counter() - t0
        for t in list(live):
            if sv.poll(t) is not None:
                k, x = live.pop(t)
                lat[k] = now - arrivals[k]
                done += 1
                if keep:
                    xs[k] = x
    span = time.perf_counter() - t0
    return lat, span, xs, held_sum / max(1, steps)


def _serving_setup(torch, pkg, dev):
    """The request pool, each problem solved once (warm-up), and the plain
    capacity: FIFO solves/s over a 40-request sample of the mix."""
    from workloads.serving import request_stream
    entries = _serve_pool(torch, pkg, dev)
    print(f"serve: pool of {len(entries)} problems ready", file=sys.stderr, flush=True)
    for e in entries:
        e["plain"].solve(e["x0"].clone().reshape(e["plain"].channels, -1), params=e["sp"], report=True)
    _, which = request_stream([e["spec"] for e in entries], 40, 1.0, seed=99)
    t0 = time.perf_counter()
    for k in which:
        e = entries[k]
        e["plain"].solve(e["x0"].clone().reshape(e["plain"].channels, -1), params=e["sp"], report=True)
    capacity = len(which) / (time.perf_counter() - t0)
    print(f"serve: plain capacity {capacity:.1f} solves/s", file=sys.stderr, flush=True)
    return entries, capacity


def serving_sweep(torch, pkg, entries, capacity, loads, n_requests):
    """Replay one seeded Poisson-arrival stream per load (rate = load x the
    plain capacity) through the server and through plain FIFO opt_solve.
    Returns (rows, requests compared bitwise, equal): the first load's results
    are compared request by request between the two."""
    from workloads.serving import request_stream
    spec = [e["spec"] for e in entries]
    rows, equal, compared = [], 0, 0
    for li, load in enumerate(loads):
        arrivals, which = request_stream(spec, n_requests, load * capacity, seed=5 + li)
        keep = li == 0
        lat_b, span_b, xs_b, mean_held = _run_batched(pkg, entries, arrivals, which, keep)
        lat_p, span_p, xs_p = _run_plain(entries, arrivals, which, keep)
        if keep:
            for k in xs_p:
                compared += 1
                equal += int(torch.equal(xs_p[k], xs_b[k]))
        n = len(arrivals)
        rows.append({"load": load, "rate_per_s": load * capacity,
                     "batched": {"p50_ms": _pct(lat_b, 50), "p99_ms": _pct(lat_b, 99),
                                 "solves_per_s": n / span_b, "mean_requests_per_step": mean_held},
                     "plain": {"p50_ms": _pct(lat_p, 50), "p99_ms": _pct(lat_p, 99),
                               "solves_per_s": n / span_p}})
        print(f"serve: load {load}: batched p50/p99 {rows[-1]['batched']['p50_ms']:.1f}/"
              f"{rows[-1]['batched']['p99_ms']:.1f} ms {rows[-1]['batched']['solves_per_s']:.1f}/s, plain "
              f"{rows[-1]['plain']['p50_ms']:.1f}/{rows[-1]['plain']['p99_ms']:.1f} ms "
              f"{rows[-1]['plain']['solves_per_s']:.1f}/s", file=sys.stderr, flush=True)
    return rows, compared, equal


SERVE_WORKLOAD = ("serving mix: 40% ARAP warp / 40% Poisson edit (grid side 128..1024, GN 10x50), "
                  "20% ARAP icosphere mesh (level 5..7, LM 10x40); mixed precision")


def serve_main(args):
    import torch
    import paper_1604_06525_amd as pkg
    dev = torch.device("cuda:0")
    entries, capacity = _serving_setup(torch, pkg, dev)
    loads = [float(v) for v in args.serve_loads.split(",")]
    rows, compared, equal = serving_sweep(torch, pkg, entries, capacity, loads, args.serve_requests)
    at1 = min(rows, key=lambda r: abs(r["load"] - 1.0))
    out = {
        "metric": "serving p99 latency at the plain capacity (batched)",
        "value": at1["batched"]["p99_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": SERVE_WORKLOAD,
                   "requests_per_load": args.serve_requests, "arena_bytes": SERVE_ARENA,
                   "max_slots": SERVE_SLOTS, "pool": [e["spec"] for e in entries]},
        "plain_capacity_solves_per_s": capacity,
        "loads": rows,
        "bitwise_equal_to_plain": f"{equal}/{compared}",
    }
    print(json.dumps(out), flush=True)


# The configurations of the measurement table (besides the headline warp run):
# name, generator, precision, method, outer, inner, algorithmic bytes per PCG
# iteration as (bytes per unknown, bytes per site) for FP32 bulk; FP64 doubles
# the per-unknown part.
CONFIGS = [
    ("warp_64x64_gn5x20_fp64", lambda w: w.arap_warp(64, 64, seed=1), "fp64", "gn", 5, 20, (24, 13)),
    ("warp_1024x1024_gn10x50_mixed", lambda w: w.arap_warp(1024, 1024, seed=2), "mixed", "gn", 10, 50, (24, 13)),
    ("warp_1024x1024_gn10x50_fp64", lambda w: w.arap_warp(1024, 1024, seed=2), "fp64", "gn", 10, 50, (24, 13)),
    ("sfs_1024x1024_gn10x50_mixed", lambda w: w.shape_from_shading(1024, 1024, seed=2), "mixed", "gn", 10, 50, (24, 13)),
    ("mesh_icosphere7_lm10x40_mixed", lambda w: w.arap_mesh(7, seed=3), "mixed", "lm", 10, 40, (24, 52)),
    ("mesh_icosphere8_lm10x40_mixed", lambda w: w.arap_mesh(8, seed=3), "mixed", "lm", 10, 40, (24, 52)),
    ("flow_1920x1080_gn10x50_mixed", lambda w: w.optical_flow(1920, 1080, seed=4), "mixed", "gn", 10, 50, (24, 8)),
    ("flow_1920x1080_gn10x50_fp64", lambda w: w.optical_flow(1920, 1080, seed=4), "fp64", "gn", 10, 50, (24, 8)),
    ("poisson_1024x1024_gn10x50_mixed", lambda w: w.poisson_edit(1024, 1024, seed=5), "mixed", "gn", 10, 50, (24, 1)),
    # a small grid alone on the chip: the tuning table's one-row strips, and
    # the four-row strips a server gives the same request
    ("warp_128x128_gn10x50_mixed", lambda w: w.arap_warp(128, 128, seed=8), "mixed", "gn", 10, 50, (24, 13)),
    ("warp_128x128_gn10x50_mixed_served", lambda w: w.arap_warp(128, 128, seed=8), "mixed", "gn", 10, 50, (24, 13),
     dict(tuning="served")),
    # large grids: at 8192^2 a vector (805 MB) is past the regular fused
    # instantiation's 256 MB buffer range and its large-grid instantiation runs
    ("warp_4096x4096_gn10x50_mixed", lambda w: w.arap_warp(4096, 4096, seed=6), "mixed", "gn", 10, 50, (24, 13)),
    ("warp_8192x8192_gn5x50_mixed", lambda w: w.arap_warp(8192, 8192, seed=7), "mixed", "gn", 5, 50, (24, 13)),
    # the warp with explicit connectivity (the lattice's 4-neighbour edge list):
    # the implicit vs explicit comparison of the paper (Fig. 18, GN 8 x 100)
    ("warp_1024x1024_gn8x100_mixed", lambda w: w.arap_warp(1024, 1024, seed=2), "mixed", "gn", 8, 100, (24, 13)),
    ("warp_graph_1024x1024_gn8x100_mixed", lambda w: _as_graph(w.arap_warp(1024, 1024, seed=2)), "mixed", "gn",
     8, 100, (24, 13)),
    # matrix-free against materialised products (Sec. 7, evalJ): the same
    # problem and schedule in the split form (the recurrence the materialised
    # form runs) and in the materialised form; bytes are the matrix-free
    # algorithmic bytes in all three, so the columns compare times
    ("warp_1024x1024_gn10x50_mixed_split", lambda w: w.arap_warp(1024, 1024, seed=2), "mixed", "gn", 10, 50,
     (24, 13), dict(pcg_variant="split")),
    ("warp_1024x1024_gn10x50_mixed_materialized", lambda w: w.arap_warp(1024, 1024, seed=2), "mixed", "gn", 10, 50,
     (24, 13), dict(pcg_variant="materialized", materialize=True)),
    # shape from shading's materialisation strategies (Sec. 8.3, Fig. 17): the
    # lighting term and its partials stored per linearisation with the rest of
    # J recomputed (the fused line above, and the split form), against the
    # whole J stored and against nothing stored (the lighting recomputed in
    # every product); bytes are the lighting-stored algorithmic bytes throughout
    ("sfs_1024x1024_gn10x50_mixed_split", lambda w: w.shape_from_shading(1024, 1024, seed=2), "mixed", "gn", 10, 50,
     (24, 13), dict(pcg_variant="split")),
    ("sfs_1024x1024_gn10x50_mixed_materialized", lambda w: w.shape_from_shading(1024, 1024, seed=2), "mixed", "gn",
     10, 50, (24, 13), dict(pcg_variant="materialized", materialize=True)),
    ("sfs_1024x1024_gn10x50_mixed_recompute", lambda w: w.shape_from_shading(1024, 1024, seed=2), "mixed", "gn",
     10, 50, (24, 13), dict(pcg_variant="recompute")),
    # volumetric ARAP on a 64^3 voxel block (implicit 3D connectivity), and the
    # Laplacian on a 1024^2 image
    ("volume_64x64x64_lm10x40_mixed", lambda w: w.arap_volume(64, 64, 64, seed=6), "mixed", "lm", 10, 40, (24, 37)),
    ("laplacian_1024x1024_gn10x50_mixed", lambda w: w.laplacian_grid(1024, 1024, seed=0), "mixed", "gn", 10, 50,
     (24, 5)),
    # l_p edge-preserving smoothing (p = 1) by IRLS: the Laplacian stencil with
    # two frozen edge weights per pixel as state
    ("lp_smooth_1024x1024_gn10x50_mixed", lambda w: w.lp_smooth(1024, 1024, seed=0), "mixed", "gn", 10, 50,
     (24, 9)),
    # the paper's IRLS example: intrinsic image decomposition at its 640 x 360
    # (reflectance and shading, 4 unknowns per pixel; p = 0.8)
    ("intrinsic_640x360_gn10x50_mixed", lambda w: w.intrinsic_image(640, 360, seed=0), "mixed", "gn", 10, 50,
     (24, 9)),
    # the level-8 mesh in the split form (two kernels per iteration), beside
    # its fused graph form above
    ("mesh_icosphere8_lm10x40_mixed_split", lambda w: w.arap_mesh(8, seed=3), "mixed", "lm", 10, 40, (24, 52),
     dict(pcg_variant="split")),
]


def _as_graph(d):
    """A grid workload as a graph: vertex j*W+i, the lattice's 4-neighbour edges."""
    from workloads.mesh import grid_edges
    return dict(d, V=d["W"] * d["H"], edges=grid_edges(d["W"], d["H"]))


def configs_main(args):
    """One JSON line per configuration: PCG iterations/s over the PCG phases,
    the per-iteration time against the algorithmic bytes, and the whole-solve
    time (median of `steps` solves after `warmup`)."""
    import torch
    import paper_1604_06525_amd as pkg
    import workloads
    from workloads.layout import problem_args
    dev = torch.device("cuda:0")
    only = set(args.configs.split(",")) if args.configs != "all" else None
    for name, gen, prec, method, outer, inner, (bu, bs), *extra in CONFIGS:
        if only and name not in only:
            continue
        extra = dict(extra[0]) if extra else {}
        variant = extra.pop("pcg_variant", "fused")
        d = gen(workloads)
        dt = np.float64 if prec == "fp64" else np.float32
        energy, arrs, params, dims = problem_args(d, dt)
        if "edges" in dims:
            dims = dict(dims, edges=torch.from_numpy(dims["edges"]).to(dev))
        prob = pkg.Problem(energy, [torch.from_numpy(a).to(dev) for a in arrs], params, precision=prec, **dims,
                           **extra)
        x0 = torch.from_numpy(np.ascontiguousarray(np.asarray(d["x0"], dt).reshape(prob.channels, -1))).to(dev)
        sp = pkg.default_params(method=method, outer_iters=outer, pcg_iters=inner, pcg_variant=variant)
        x = x0.clone()
        for _ in range(args.warmup):
            x.copy_(x0)
            prob.solve(x, params=sp, report=False)
        torch.cuda.synchronize()
        prob.profile_enable(True)
        prob.profile_read()
        solve_ms = []
        stream = torch.cuda.current_stream()
        for _ in range(args.steps):
            x.copy_(x0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            prob.solve(x, params=sp, report=False)
            e1.record(stream)
            torch.cuda.synchronize()
            solve_ms.append(e0.elapsed_time(e1))
        pcg_ms, pcg_iters = prob.profile_read()
        prob.profile_enable(False)
        n = prob.n_sites
        N = n * prob.channels
        per_unknown = bu * (2 if prec == "fp64" else 1)
        bpi = per_unknown * N + bs * n
        iter_us = 1e3 * pcg_ms / pcg_iters
        achieved = bpi / (iter_us * 1e-6) / 1e9
        rep = prob.solve(x.copy_(x0), params=sp)
        print(json.dumps({"config": name, "sites": n, "unknowns": N, "precision": prec, "method": method,
                          "outer_iters": outer, "pcg_iters": inner,
                          "pcg_form": prob.pcg_form(variant),
                          "pcg_iters_per_s": pcg_iters / (pcg_ms / 1e3), "iter_us": iter_us,
                          "bytes_per_iter": bpi, "achieved_GBs": achieved, "frac_of_8TBs": achieved / HBM_PEAK_GBS,
                          "solve_ms_median": float(np.median(solve_ms)), "cost_initial": rep["cost_initial"],
                          "cost_final": rep["cost_final"], "launch": prob.get_tuning()}), flush=True)
        del prob
        torch.cuda.synchronize()


# ---------------------------------------------------------------- accuracy against the oracle
# Every configuration of the measurement table at its full size and schedule:
# name, generator, precision, method, outer, inner.  The FP64 oracle solves the
# same problem on the host (for mixed precision on the FP32-rounded inputs the
# GPU holds); the GPU's final cost and unknowns are compared with it.
ACCURACY = [
    ("warp_64x64_gn5x20_fp64", lambda w: w.arap_warp(64, 64, seed=1), "fp64", "gn", 5, 20),
    ("warp_1024x1024_gn10x50_mixed", lambda w: w.arap_warp(1024, 1024, seed=2), "mixed", "gn", 10, 50),
    ("warp_1024x1024_gn10x50_fp64", lambda w: w.arap_warp(1024, 1024, seed=2), "fp64", "gn", 10, 50),
    ("sfs_1024x1024_gn10x50_mixed", lambda w: w.shape_from_shading(1024, 1024, seed=2), "mixed", "gn", 10, 50),
    # the same problem in FP64, and under LM (whose accepted steps never raise
    # the cost): Gauss-Newton is not monotone on it
    ("sfs_1024x1024_gn10x50_fp64", lambda w: w.shape_from_shading(1024, 1024, seed=2), "fp64", "gn", 10, 50),
    ("sfs_1024x1024_lm10x50_mixed", lambda w: w.shape_from_shading(1024, 1024, seed=2), "mixed", "lm", 10, 50),
    ("mesh_icosphere7_lm10x40_mixed", lambda w: w.arap_mesh(7, seed=3), "mixed", "lm", 10, 40),
    ("mesh_icosphere7_lm10x40_fp64", lambda w: w.arap_mesh(7, seed=3), "fp64", "lm", 10, 40),
    ("mesh_icosphere8_lm10x40_mixed", lambda w: w.arap_mesh(8, seed=3), "mixed", "lm", 10, 40),
    ("flow_1920x1080_gn10x50_mixed", lambda w: w.optical_flow(1920, 1080, seed=4), "mixed", "gn", 10, 50),
    ("flow_1920x1080_gn10x50_fp64", lambda w: w.optical_flow(1920, 1080, seed=4), "fp64", "gn", 10, 50),
    ("poisson_1024x1024_gn10x50_mixed", lambda w: w.poisson_edit(1024, 1024, seed=5), "mixed", "gn", 10, 50),
    ("lp_smooth_1024x1024_gn10x50_mixed", lambda w: w.lp_smooth(1024, 1024, seed=0), "mixed", "gn", 10, 50),
    ("lp_smooth_1024x1024_gn10x50_fp64", lambda w: w.lp_smooth(1024, 1024, seed=0), "fp64", "gn", 10, 50),
    ("intrinsic_640x360_gn10x50_mixed", lambda w: w.intrinsic_image(640, 360, seed=0), "mixed", "gn", 10, 50),
    ("intrinsic_640x360_gn10x50_fp64", lambda w: w.intrinsic_image(640, 360, seed=0), "fp64", "gn", 10, 50),
    ("laplacian_1024x1024_gn10x50_mixed", lambda w: w.laplacian_grid(1024, 1024, seed=0), "mixed", "gn", 10, 50),
    ("volume_64x64x64_lm10x40_mixed", lambda w: w.arap_volume(64, 64, 64, seed=6), "mixed", "lm", 10, 40),
]


def _as_held(d, precision):
    """The workload as the GPU holds it: under mixed precision every float array
    rounded to float32 (and back to float64 for the oracle).  Re-packaging only."""
    if precision == "fp64":
        return d
    return {k: (v.astype(np.float32).astype(np.float64) if isinstance(v, np.ndarray) and v.dtype.kind == "f" else v)
            for k, v in d.items()}


def _oracle_config(name):
    """Worker process: the oracle's whole solve of one configuration (FP64, one
    thread).  Returns its cost trace, final unknowns, accepted steps (LM), the
    smoothness masks at every linearisation point (shape from shading) and the
    time taken.  Prints one progress line per outer iteration."""
    import oracle
    import workloads
    spec = {c[0]: c for c in ACCURACY}[name]
    _, gen, precision, method, K, L = spec
    d = _as_held(gen(workloads), precision)
    e = oracle.make_energy(d)
    masks = []
    t0 = time.perf_counter()

    def progress(k, x):
        if d["energy"] == "sfs" and k < K:
            masks.append(e.smooth_valid(np.asarray(x).reshape(d["H"], d["W"])))
        print(f"accuracy: oracle {name} iteration {k}/{K} ({time.perf_counter() - t0:.0f} s)",
              file=sys.stderr, flush=True)

    if d["energy"] == "sfs":
        masks.append(e.smooth_valid(np.asarray(d["x0"], float).reshape(d["H"], d["W"])))
    if d["energy"] in ("lp_smooth", "intrinsic"):
        # IRLS: Gauss-Newton steps with the weights frozen at each linearisation
        x, costs = oracle.irls(e, d["x0"], K, L, callback=progress)
        acc = None
    elif method == "gn":
        x, costs = oracle.gauss_newton(e, d["x0"], K, L, callback=progress)
        acc = None
    else:
        x, costs, acc = oracle.levenberg_marquardt(e, d["x0"], K, L, callback=progress)
    return {"costs": costs, "x": x, "accepted": acc, "masks": masks, "seconds": time.perf_counter() - t0}


def accuracy_main(args):
    """One JSON line per configuration: the GPU's final cost and unknowns against
    the FP64 oracle's at full size and schedule, plus the oracle's whole-solve
    time on one host core."""
    only = set(args.configs.split(",")) if args.configs and args.configs != "all" else None
    todo = [c for c in ACCURACY if not only or c[0] in only]
    # the oracle workers are started before anything touches the GPU, one
    # thread each
    workers = max(1, min(len(todo), _host_cores() - 1))
    pool = _oracle_pool(workers)
    # longest first
    futs = {c[0]: pool.submit(_oracle_config, c[0]) for c in sorted(todo, key=lambda c: -_oracle_weight(c))}
    import torch
    import paper_1604_06525_amd as pkg
    import workloads
    import oracle
    from workloads.layout import problem_args
    dev = torch.device("cuda:0")
    gpu = {}
    for name, gen, precision, method, K, L in todo:
        d = gen(workloads)
        dt = np.float64 if precision == "fp64" else np.float32
        energy, arrs, params, dims = problem_args(d, dt)
        if "edges" in dims:
            dims = dict(dims, edges=torch.from_numpy(dims["edges"]).to(dev))
        prob = pkg.Problem(energy, [torch.from_numpy(a).to(dev) for a in arrs], params, precision=precision, **dims)
        x0 = torch.from_numpy(np.ascontiguousarray(np.asarray(d["x0"], dt).reshape(prob.channels, -1))).to(dev)
        x = x0.clone()
        rep = prob.solve(x, method=method, outer_iters=K, pcg_iters=L)
        out = {"rep": rep, "x": x.cpu().double().numpy().ravel()}
        if energy == "sfs" and method == "gn":
            # the iterate at every linearisation point: Gauss-Newton keeps no
            # state between outer iterations, so K solves of one iteration each
            # pass through the same iterates
            e = oracle.make_energy(_as_held(d, precision))
            xs = x0.clone()
            masks = [e.smooth_valid(xs.cpu().double().numpy().reshape(d["H"], d["W"]))]
            for k in range(K - 1):
                prob.solve(xs, method=method, outer_iters=1, pcg_iters=L, report=False)
                masks.append(e.smooth_valid(xs.cpu().double().numpy().reshape(d["H"], d["W"])))
            out["masks"] = masks
        gpu[name] = out
        print(f"accuracy: GPU {name} done, cost {rep['cost_final']:.10g}", file=sys.stderr, flush=True)
        del prob
        torch.cuda.synchronize()
    rows = []
    for name, gen, precision, method, K, L in todo:
        ref = futs[name].result()
        g = gpu[name]
        d0 = np.asarray(_as_held(gen(__import__("workloads")), precision)["x0"], float).ravel()
        xo, xg = np.asarray(ref["x"], float).ravel(), g["x"]
        Eo, Eg = ref["costs"][-1], g["rep"]["cost_final"]
        row = {"config": name, "precision": precision, "method": method, "outer_iters": K, "pcg_iters": L,
               "cost_oracle": Eo, "cost_gpu": Eg, "rel_cost_err": abs(Eg - Eo) / Eo,
               "rel_cost_err_max_over_trace": max(abs(a - b) / b for a, b in zip(g["rep"]["cost_trace"], ref["costs"])),
               "unknown_err_rel": float(np.linalg.norm(xg - xo) / max(np.linalg.norm(xo - d0), 1e-300)),
               "unknown_err_maxabs": float(np.abs(xg - xo).max()),
               "oracle_solve_s": ref["seconds"], "oracle_threads": 1,
               "oracle_processes_at_once": workers}
        if method == "lm":
            row["accepted_oracle"] = int(sum(ref["accepted"]))
            row["accepted_gpu"] = int(g["rep"]["steps_accepted"])
        if "masks" in g:
            row["smooth_mask_flips_per_linearisation"] = [int(np.count_nonzero(a != b))
                                                          for a, b in zip(g["masks"], ref["masks"])]
        rows.append(row)
        print(json.dumps(row), flush=True)
    pool.shutdown()
    print(json.dumps({"accuracy_summary": {r["config"]: r["rel_cost_err"] for r in rows},
                      "host": {"cores": _host_cores(), "model": _cpu_model()}}), flush=True)


def _oracle_weight(c):
    """Rough oracle cost of a configuration, to start the longest first."""
    name = c[0]
    for key, wgt in (("icosphere8", 8), ("flow", 6), ("sfs", 4), ("1024x1024", 3), ("icosphere7", 2)):
        if key in name:
            return wgt
    return 1


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path is single-GPU; see the design notes on sharding)", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_main(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.accuracy:
        accuracy_main(args)
        return
    if args.configs:
        configs_main(args)
        return
    # the oracle's CPU baseline runs first, in worker processes started before
    # anything touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(WARP["pcg"])
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
    # the PCG phase holds one priming launch per outer iteration besides the
    # iteration launches; this is the average over all of them (what a kernel
    # trace reports for the fused kernel)
    launch_avg_us = 1e3 * pcg_ms / (pcg_iters + pcg_iters // WARP["pcg"])
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
                   "launch": prob.get_tuning(),
                   "unknowns": 3 * n, "outer_iters": WARP["outer"], "pcg_iters": WARP["pcg"],
                   "precision": "mixed: FP32 bulk, FP64 dot products and costs", "seed": WARP["seed"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(prob.get_tuning()),
                     "unit_of_work": "one PCG iteration = one k_fused launch",
                     "bytes_per_iter": bpi, "iter_us": iter_us, "launch_avg_us": launch_avg_us},
        "pcg_phase_iters_per_s": pcg_iters / (pcg_ms / 1e3),
        "cost_initial": rep["cost_initial"],
        "cost_final": rep["cost_final"],
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if args.serve_leg_requests > 0:
        # compact serving leg: the batching server against plain FIFO solves on
        # the same Poisson-arrival streams, at the plain capacity (latency) and
        # at twice it (where plain saturates and throughput shows)
        del prob
        torch.cuda.synchronize()
        entries, capacity = _serving_setup(torch, pkg, dev)
        rows, compared, equal = serving_sweep(torch, pkg, entries, capacity, [1.0, 2.0], args.serve_leg_requests)
        out["serving"] = {"workload": SERVE_WORKLOAD, "requests_per_load": args.serve_leg_requests,
                          "plain_capacity_solves_per_s": capacity, "loads": rows,
                          "bitwise_equal_to_plain": f"{equal}/{compared}",
                          "note": "latency = result on the host minus arrival; solves/s over the whole stream"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
