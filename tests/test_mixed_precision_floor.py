"""Why two configurations cannot meet a 1e-4 relative-cost bound in FP32 bulk
arithmetic: the ARAP mesh with 1% handles (the tolerance of the mixed-precision
mesh test), and shape from shading under Gauss-Newton (the last test here).

This is a study of the oracle's own algorithm, no GPU: Levenberg-Marquardt with
the textbook PCG run with every vector rounded to float32 and the dot products
accumulated in float64 (the mixed-precision definition), and J^T J p formed from
the FP32-rounded Jacobian in FP32.  Perturbing each q = J^T J p by at most one
FP32 ulp (a change of summation order does as much) moves the final cost by far
more than 1e-4 on the 1%-handle icosphere, because that system is nearly
singular (few handles pin a nearly free surface) and 40 PCG iterations do not
converge: rounding decides where the truncated Krylov solve ends.  The same
perturbation at FP64 ulp size moves the FP64 solve by about 1e-11, and with 5%
handles the FP32 runs agree with the oracle to about 1e-6.  The bound used for
the 1%-handle mixed LM test (1e-3 after 4 x 40 iterations) covers this measured
spread; it is a property of the configuration, not of the kernels.
"""
import numpy as np
import pytest

import oracle as o
import workloads as w

F32 = np.float32


def _lm(energy, x0, outer, inner, fp32, seed, prm=o.LMParams()):
    """LM of Sec. 4 as the oracle runs it; fp32: vectors, J and q in float32,
    dots in float64; seed > 0: each q entry perturbed by -1, 0 or +1 ulp (of its
    precision)."""
    rng = np.random.default_rng(seed)
    dt = F32 if fp32 else np.float64
    ulp = 2.0 ** -24 if fp32 else 2.0 ** -53
    x = np.asarray(x0, float).ravel().astype(dt)
    radius, nu, lin = prm.radius0, 2.0, None
    for _ in range(outer):
        if lin is None:
            lin = o.Linearization(energy, x.astype(float))
            J, JT = lin.J.astype(dt), lin.JT.astype(dt)
        lam = 1.0 / radius
        dg = lin.diag.astype(dt)
        Dl = (dt(lam) * np.clip(dg, dt(prm.diag_min), dt(prm.diag_max)) * lin.active).astype(dt)
        den = (dg + Dl).astype(dt)
        minv = np.where(lin.active & (den > 0), dt(1) / np.where(den > 0, den, 1), 0).astype(dt)
        r = (-(JT @ lin.F.astype(dt))).astype(dt)
        d = np.zeros_like(r)
        z = (minv * r).astype(dt)
        p = z.copy()
        rz = float(r.astype(float) @ z.astype(float))
        for _ in range(inner):
            q = (JT @ (J @ p) + Dl * p).astype(dt)
            if seed:
                q = (q * (1 + rng.choice([-1.0, 0.0, 1.0], q.size) * ulp)).astype(dt)
            pq = float(p.astype(float) @ q.astype(float))
            if not pq > 0:
                break
            a = dt(rz / pq)
            d = (d + a * p).astype(dt)
            r = (r - a * q).astype(dt)
            z = (minv * r).astype(dt)
            rzn = float(r.astype(float) @ z.astype(float))
            p = (z + dt(rzn / rz) * p).astype(dt)
            rz = rzn
        Jd = lin.J @ d.astype(float)
        m = -float(Jd @ (2.0 * lin.F + Jd))
        xt = (x + d).astype(dt)
        E1 = o.cost(energy, xt.astype(float))
        rho = (lin.E - E1) / m if m != 0 else -np.inf
        if m > 0 and rho > prm.min_rel_decrease:
            x = xt
            radius = min(radius / max(1 / 3, 1 - (2 * rho - 1) ** 3), prm.radius_max)
            nu, lin = 2.0, None
        else:
            radius, nu = radius / nu, 2 * nu
    return o.cost(energy, x.astype(float))


def _rounded(d):
    return {k: (v.astype(F32).astype(float) if isinstance(v, np.ndarray) and v.dtype.kind == "f" else v)
            for k, v in d.items()}


@pytest.fixture(scope="module")
def one_percent():
    d = _rounded(w.arap_mesh(5, seed=3, handle_frac=0.01))
    e = o.make_energy(d)
    _, costs, _ = o.levenberg_marquardt(e, d["x0"], 4, 40)
    return d, e, costs[-1]


def test_fp32_rounding_spreads_past_1e4_with_one_percent_handles(one_percent):
    d, e, E_ref = one_percent
    rel = [abs(_lm(e, d["x0"], 4, 40, True, s) - E_ref) / E_ref for s in (1, 2, 3)]
    assert max(rel) > 1e-4, rel       # the bound is out of reach for FP32 bulk
    assert max(rel) < 1e-3, rel       # and the test's 1e-3 covers the spread


def test_fp64_rounding_does_not(one_percent):
    d, e, E_ref = one_percent
    rel = abs(_lm(e, d["x0"], 4, 40, False, 1) - E_ref) / E_ref
    assert rel < 1e-9, rel


def test_five_percent_handles_meet_1e4_in_fp32():
    d = _rounded(w.arap_mesh(5, seed=3, handle_frac=0.05))
    e = o.make_energy(d)
    _, costs, _ = o.levenberg_marquardt(e, d["x0"], 4, 40)
    rel = abs(_lm(e, d["x0"], 4, 40, True, 1) - costs[-1]) / costs[-1]
    assert rel < 1e-5, rel


def test_sfs_gauss_newton_amplifies_fp32_depth_storage():
    """Shape from shading, Gauss-Newton 10 x 50 (the configuration's schedule):
    the FP64 cost trace is not monotone (GN overshoots on this nonlinear shading
    energy), and storing only the depth in float32 between outer iterations
    (every other operation FP64) moves the cost trace by more than 1e-4.  The
    mixed-precision GPU path stores the depth in float32, so its distance to the
    FP64 oracle on this configuration is set by this sensitivity (at 1024^2 the
    same experiment moves the final cost by 1e-1, the GPU's by 4e-2), not by its
    kernels (the FP64 GPU run agrees with the oracle to 5e-7)."""
    d = _rounded(w.shape_from_shading(256, 256, seed=2))
    e = o.make_energy(d)
    _, ref = o.gauss_newton(e, d["x0"], 10, 50)
    assert any(b > a for a, b in zip(ref, ref[1:]))  # not monotone
    x = np.asarray(d["x0"], float).ravel().astype(F32)
    costs = []
    for _ in range(10):
        lin = o.Linearization(e, x.astype(float))
        costs.append(lin.E)
        dl, _ = o.pcg(lin.apply, lin.jtf(), lin.minv(True), 50)
        x = (x + dl.astype(F32)).astype(F32)
    costs.append(o.cost(e, x.astype(float)))
    rel = max(abs(a - b) / b for a, b in zip(costs, ref))
    assert rel > 1e-4, rel
