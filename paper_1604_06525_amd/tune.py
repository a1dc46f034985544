"""Autotuner for the launch shape of the fused PCG kernel.

    python -m paper_1604_06525_amd.tune [--out tuning.json] [--quick]

For each grid energy with a fused kernel (ARAP warp, Poisson, optical flow,
shape from shading, the Laplacian, l_p smoothing, intrinsic decomposition), each
precision and each size class (grid sides 64, 128, 256, 512, 1024, 2048), it times
the PCG phase of a short solve on a seeded synthetic problem for every candidate
launch shape (fixed strip heights, and balanced partitions with 1 to 4 strips
per SIMD), and keeps the fastest.  The result is a JSON list of entries
{energy, precision, min_sites, max_sites, strip_rows, waves_per_simd, iter_us,
candidates}; a class covers the sites from half its own count up to twice it.  ``apply()``
feeds the entries to a Server (used at admission) and ``best()`` looks one up for
a single Problem.  Every choice gives the same iterates up to rounding; only the
speed differs.

A small grid alone on the chip is fastest in strips of one to three rows (its
launch is latency-bound and a strip's walk is its rows plus four halo steps).
A served request shares each batched launch with others, whose length the
largest request sets, so there such strips only add waves: the server takes the
fastest candidate of at least SERVED_MIN_ROWS rows from the same entry (``best``
and ``apply`` with ``served=True``), and a Problem created with
``tuning="served"`` runs the shape the server would give it, bit for bit the
same solve.
"""
import argparse
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "tuning.json")
CANDIDATES = tuple(("rows", r) for r in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32)) + \
    tuple(("waves", w) for w in (1, 2, 3, 4)) + (("auto", 0),)
SIDES = (64, 128, 256, 512, 1024, 2048)
SERVED_MIN_ROWS = 4
ENERGIES = ("arap_warp", "poisson", "flow", "sfs", "laplacian", "lp_smooth", "intrinsic")


def _problem(energy, side, precision):
    import torch
    import paper_1604_06525_amd as pkg
    import workloads
    from workloads.layout import problem_args
    if energy == "arap_warp":
        d = workloads.arap_warp(side, side, seed=2)
    elif energy == "poisson":
        d = workloads.poisson_edit(side, side, seed=5)
    elif energy == "sfs":
        d = workloads.shape_from_shading(side, side, seed=2)
    elif energy == "laplacian":
        d = workloads.laplacian_grid(side, side, seed=0)
    elif energy == "lp_smooth":
        d = workloads.lp_smooth(side, side, seed=0)
    elif energy == "intrinsic":
        d = workloads.intrinsic_image(side, side, seed=0)
    else:
        d = workloads.optical_flow(side, side, seed=4)
    dt = np.float64 if precision == "fp64" else np.float32
    name, arrs, params, dims = problem_args(d, dt)
    dev = torch.device("cuda:0")
    prob = pkg.Problem(name, [torch.from_numpy(a).to(dev) for a in arrs], params, precision=precision, **dims)
    x0 = torch.from_numpy(np.ascontiguousarray(np.asarray(d["x0"], dt).reshape(prob.channels, -1))).to(dev)
    return prob, x0


def _fields(cand):
    kind, v = cand
    return {"strip_rows": v if kind == "rows" else 0, "waves_per_simd": v if kind == "waves" else 0}


def time_candidate(prob, x0, cand, pcg_iters=50, repeats=3):
    """Microseconds per PCG iteration (median of repeats) with this launch shape."""
    import paper_1604_06525_amd as pkg
    prob.set_tuning(**_fields(cand))
    sp = pkg.default_params(method="gn", outer_iters=1, pcg_iters=pcg_iters)
    x = x0.clone()
    prob.solve(x, params=sp, report=False)  # warm-up
    prob.profile_enable(True)
    prob.profile_read()
    times = []
    for _ in range(repeats):
        x.copy_(x0)
        prob.solve(x, params=sp, report=False)
        ms, iters = prob.profile_read()
        times.append(1e3 * ms / iters)
    prob.profile_enable(False)
    return float(np.median(times))


def autotune(energies=ENERGIES, precisions=("mixed", "fp64"), sides=SIDES, candidates=CANDIDATES,
             log=sys.stderr):
    entries = []
    for energy in energies:
        for precision in precisions:
            for side in sides:
                prob, x0 = _problem(energy, side, precision)
                res = {}
                for c in candidates:
                    if c[0] == "rows" and c[1] > side:
                        continue
                    res[c] = time_candidate(prob, x0, c)
                best = min(res, key=res.get)
                n = side * side
                entries.append(dict(energy=energy, precision=precision, min_sites=n // 2, max_sites=2 * n,
                                    side=side, **_fields(best), iter_us=res[best],
                                    candidates={f"{k[0]}={k[1]}": v for k, v in res.items()}))
                print(f"tune {energy} {precision} {side}^2: {best[0]}={best[1]} ({res[best]:.2f} us/iter)",
                      file=log, flush=True)
    return entries


def save(entries, path=DEFAULT_PATH):
    with open(path, "w") as f:
        json.dump(entries, f, indent=1)


def load(path=DEFAULT_PATH):
    if not os.path.exists(path):
        return []
    with open(path) as f:
        return json.load(f)


def choice(entry, served=False):
    """The entry's launch shape: its fastest candidate, or with served=True the
    fastest one whose strips have at least SERVED_MIN_ROWS rows."""
    rows = entry.get("strip_rows", 0)
    if not served or rows == 0 or rows >= SERVED_MIN_ROWS:
        return {"strip_rows": rows, "waves_per_simd": entry.get("waves_per_simd", 0)}
    ok = {}
    for k, v in entry.get("candidates", {}).items():
        kind, val = k.split("=")
        if kind != "rows" or int(val) >= SERVED_MIN_ROWS:
            ok[(kind, int(val))] = v
    if not ok:
        return {"strip_rows": SERVED_MIN_ROWS, "waves_per_simd": 0}
    return _fields(min(ok, key=ok.get))


def best(entries, energy, precision, n_sites, served=False):
    """Tuning fields of the last matching entry, or the automatic choice."""
    hit = {"strip_rows": 0, "waves_per_simd": 0}
    for e in entries:
        if e["energy"] == energy and e["precision"] == precision and e["min_sites"] <= n_sites <= e["max_sites"]:
            hit = choice(e, served)
    return hit


def apply(server, entries):
    """Register the entries with a Server, in their served form."""
    for e in entries:
        c = choice(e, served=True)
        server.add_tuning(e["energy"], e["precision"], e["min_sites"], e["max_sites"],
                          c["strip_rows"], c["waves_per_simd"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--quick", action="store_true", help="mixed precision, ARAP warp only")
    ap.add_argument("--energies", default="", help="comma list: retune these energies only, keeping the "
                    "other energies' entries of --base")
    ap.add_argument("--sides", default="", help="comma list: retune these grid sides only, keeping the other "
                    "sides' entries of --base")
    ap.add_argument("--base", default=DEFAULT_PATH)
    a = ap.parse_args()
    if a.quick:
        entries = autotune(energies=("arap_warp",), precisions=("mixed",))
    elif a.energies or a.sides:
        names = tuple(a.energies.split(",")) if a.energies else ENERGIES
        sides = tuple(int(v) for v in a.sides.split(",")) if a.sides else SIDES
        kept = [e for e in load(a.base) if not (e["energy"] in names and e["side"] in sides)]
        entries = kept + autotune(energies=names, sides=sides)
        order = {(en, p, s): i for i, (en, p, s) in enumerate(
            (en, p, s) for en in ENERGIES for p in ("mixed", "fp64") for s in SIDES)}
        entries.sort(key=lambda e: order.get((e["energy"], e["precision"], e["side"]), len(order)))
    else:
        entries = autotune()
    save(entries, a.out)
    print(json.dumps({"entries": len(entries), "path": a.out}))


if __name__ == "__main__":
    main()
