"""Helpers for the GPU parity tests: build a library problem from a seeded
workload, move vectors between numpy and the device."""
import numpy as np
import pytest
import torch

from workloads.layout import problem_args


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def make_problem(d, precision="fp64", tuning="auto"):
    import paper_1604_06525_amd as pkg
    dt = np.float64 if precision == "fp64" else np.float32
    energy, arrs, params, dims = problem_args(d, dt)
    dev = torch.device("cuda:0")
    t_arrs = [torch.from_numpy(a).to(dev) for a in arrs]
    if "edges" in dims:
        dims = dict(dims, edges=torch.from_numpy(dims["edges"]).to(dev))
    prob = pkg.Problem(energy, t_arrs, params, precision=precision, tuning=tuning, **dims)
    return prob


def to_dev(prob, v):
    c = prob.channels
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(c, -1))
    return torch.from_numpy(a).to(device=prob.device, dtype=prob.dtype).contiguous()


def to_np(t):
    return t.detach().cpu().double().numpy().ravel()


def relmax(a, b):
    """max |a-b| / max |b| (0 when both vanish)."""
    a, b = np.asarray(a, float).ravel(), np.asarray(b, float).ravel()
    s = np.abs(b).max()
    d = np.abs(a - b).max()
    return 0.0 if d == 0 else d / (s if s > 0 else 1.0)


def f32_inputs(d):
    """The workload with every float array rounded to float32 (and back to
    float64): the data a mixed-precision problem actually holds, so that the FP64
    oracle can be evaluated on exactly those values."""
    out = {}
    for k, v in d.items():
        if isinstance(v, np.ndarray) and v.dtype.kind == "f":
            out[k] = v.astype(np.float32).astype(np.float64)
        else:
            out[k] = v
    return out


PCG_TOL_CAP = 1e-6
PCG_SPREAD_MAX = 1e-8


def pcg_tol(ref, ref2):
    """Tolerance for PCG iterates against the oracle: 100x the oracle's own
    spread between two valid evaluation orders of the same product (J^T(J p) and
    (J^T J) p), at least 1e-9.  A case where CG has lost orthogonality (spread
    above 1e-8) could not tell a wrong product from rounding, so it is refused
    instead of being compared loosely: the tolerance never exceeds 1e-6."""
    spread = relmax(ref2, ref)
    assert spread <= PCG_SPREAD_MAX, f"oracle spread {spread:.2e}: this PCG case is rounding-dominated"
    tol = max(1e-9, 100 * spread)
    assert tol <= PCG_TOL_CAP
    return tol
