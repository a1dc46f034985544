"""Seeded request streams for the serving benchmark.

A request names a problem from a fixed pool and its solve schedule.  Requests
are ARAP image warps and Poisson edits on square grids whose side is drawn
uniformly from [128, 1024], and ARAP deformations of icospheres of level 5, 6 or
7 (10,242 / 40,962 / 163,842 vertices), in the proportions 40 / 40 / 20.  Grid
requests run Gauss-Newton 10 x 50, mesh requests Levenberg-Marquardt 10 x 40.
Arrivals form a Poisson process: exponential gaps of mean 1/rate.  Generating a
fresh problem per request is too slow for long streams, so each request draws
its kind with the proportions above and then one problem of that kind from a
pool; every request starts from its problem's initial unknowns.
"""
import numpy as np

KINDS = ("arap_warp", "poisson", "arap_mesh")
KIND_P = (0.4, 0.4, 0.2)
SCHEDULE = {"arap_warp": ("gn", 10, 50), "poisson": ("gn", 10, 50), "arap_mesh": ("lm", 10, 40)}


def pool_spec(per_kind=(8, 8, 3), seed=5):
    """Problem specs: dicts with kind, size (grid side or icosphere level) and the
    seed of the problem's own data.  The mesh pool holds levels 5, 6, 7 in turn."""
    rng = np.random.default_rng(seed)
    out = []
    for kind, count in zip(KINDS, per_kind):
        for k in range(count):
            size = 5 + k % 3 if kind == "arap_mesh" else int(rng.integers(128, 1025))
            out.append(dict(kind=kind, size=size, seed=int(seed * 1000 + len(out))))
    return out


def request_stream(pool, n_requests, rate, seed=5):
    """(arrival times in seconds from 0, pool index of each request)."""
    rng = np.random.default_rng(seed + 17)
    gaps = rng.exponential(1.0 / rate, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    by_kind = {k: [i for i, p in enumerate(pool) if p["kind"] == k] for k in KINDS}
    kinds = rng.choice(len(KINDS), size=n_requests, p=KIND_P)
    which = np.array([by_kind[KINDS[k]][rng.integers(0, len(by_kind[KINDS[k]]))] for k in kinds])
    return arrivals, which
