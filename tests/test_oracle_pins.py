"""Pins of the oracle's shape-from-shading normal and lighting and of its LM step
control, each against something other than the oracle's own formulas.

* Normal (eq. 10): the listed components equal minus the cross product of the
  two backward differences of the back-projected positions (eq. 8),
  p(a,b) - p(a-1,b) and p(a,b) - p(a,b-1).  The test forms the positions and
  takes the cross product with numpy, with f_x != f_y and u_x != u_y, so a swapped
  focal length, centre or normal component fails it.
* Lighting (Fig. 26): each of the nine coefficients, set alone, must give the
  matching real spherical-harmonic basis function (up to order two, without its
  constant) of that unit normal; the order-two zonal term is written here as
  3 n_z^2 - 1, which equals the listed -n_x^2 - n_y^2 + 2 n_z^2 only for a unit
  normal, so the normalisation is pinned too.
* LM (Sec. 4, with the Nielsen trust-region reading): on a problem whose only
  residuals are linear the gain ratio is exactly 1, so each accepted step
  triples the radius and x - C shrinks by lambda/(1 + lambda) per step; with an
  acceptance threshold above 1 every step is rejected and the radius falls by
  2, 4, 8, ...; and a hand-derived scalar trace (tests/golden) exercises accepted
  steps with gain ratios inside (0, 1) and runs of rejections.
"""
import json
import os

import numpy as np
import pytest

import oracle as o
import workloads as w

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

FX, FY, UX, UY = 23.0, 31.0, 4.3, 2.7


def _sfs_field(W=11, H=9, seed=6):
    d = w.shape_from_shading(W, H, seed=seed, amplitude=0.004, focal=(FX, FY), center=(UX, UY))
    rng = np.random.default_rng(seed)
    X = d["D"] + 0.01 * rng.normal(size=(H, W))
    return d, X


def _energy(d, L, Im=None):
    p = d["params"]
    return o.ShapeFromShading(d["W"], d["H"], d["D"], d["Im"] if Im is None else Im, d["edge_r"],
                              d["edge_c"], p["w_p"], p["w_s"], p["w_g"], p["f_x"], p["f_y"],
                              p["u_x"], p["u_y"], L)


def _cross_normals(X):
    """Unit normals from the cross product of back-projected differences, and
    the pixels where the shading term is defined (one pixel inside the border,
    depth > 0 at (a,b), (a-1,b), (a,b-1))."""
    H, W = X.shape
    j, i = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    P = np.stack([(i - UX) / FX * X, (j - UY) / FY * X, X])
    e1 = np.zeros((3, H, W))
    e2 = np.zeros((3, H, W))
    e1[:, :, 1:] = P[:, :, 1:] - P[:, :, :-1]   # p(a,b) - p(a-1,b)
    e2[:, 1:, :] = P[:, 1:, :] - P[:, :-1, :]   # p(a,b) - p(a,b-1)
    c = -np.cross(e1, e2, axis=0)
    n = c / np.linalg.norm(c, axis=0).clip(1e-300)
    ok = (i >= 1) & (i <= W - 2) & (j >= 1) & (j <= H - 2)
    return n, ok


def _basis(n):
    x, y, z = n
    return [np.ones_like(x), y, z, x, x * y, y * z, 3 * z * z - 1, z * x, x * x - y * y]


@pytest.mark.parametrize("k", range(9))
def test_sfs_lighting_term_is_sh_basis_of_cross_product_normal(k):
    d, X = _sfs_field()
    L = [0.0] * 9
    L[k] = 1.0
    e = _energy(d, L, Im=np.zeros_like(d["Im"]))
    BI = np.real(e.B_I(X))
    n, ok = _cross_normals(X)
    want = _basis(n)[k]
    assert ok.sum() > 40
    assert np.abs(BI[ok] - want[ok]).max() < 1e-12
    assert np.all(BI[~ok] == 0)


def test_sfs_lighting_is_linear_in_coefficients():
    d, X = _sfs_field()
    L = np.array([0.5, 0.07, -0.3, 0.04, 0.03, -0.02, 0.05, 0.06, -0.04])
    e = _energy(d, tuple(L), Im=np.zeros_like(d["Im"]))
    n, ok = _cross_normals(X)
    want = sum(c * b for c, b in zip(L, _basis(n)))
    assert np.abs(np.real(e.B_I(X))[ok] - want[ok]).max() < 1e-12


def test_sfs_intensity_blur():
    # with all lighting off, B_I = -(Im(a,b)/2 + (Im(a-1,b) + Im(a,b-1))/4)
    d, X = _sfs_field()
    Im = np.random.default_rng(3).random(d["Im"].shape)
    e = _energy(d, (0.0,) * 9, Im=Im)
    _, ok = _cross_normals(X)
    want = np.zeros_like(Im)
    want[1:, 1:] = -(0.5 * Im[1:, 1:] + 0.25 * (Im[1:, :-1] + Im[:-1, 1:]))
    assert np.abs(np.real(e.B_I(X))[ok] - want[ok]).max() < 1e-15


def test_sfs_normal_changes_with_swapped_intrinsics():
    # the pin above is sensitive to the roles of f_x/f_y and u_x/u_y: swapping
    # them in the energy moves the normal far beyond the tolerance
    d, X = _sfs_field()
    n, ok = _cross_normals(X)
    p = d["params"]
    for fx, fy, ux, uy in ((FY, FX, UX, UY), (FX, FY, UY, UX)):
        e = o.ShapeFromShading(d["W"], d["H"], d["D"], np.zeros_like(d["Im"]), d["edge_r"], d["edge_c"],
                               p["w_p"], p["w_s"], p["w_g"], fx, fy, ux, uy, (0, 0, 0, 1, 0, 0, 0, 0, 0))
        assert np.abs(np.real(e.B_I(X))[ok] - n[0][ok]).max() > 1e-4


def _one_pixel_warp(x0_off=(2.0, -1.5), target=(20.0, 30.0)):
    """A 3 x 3 ARAP warp whose only free pixel is the centre: every other pixel
    is masked, so no regulariser is valid and the centre's offsets see only their
    linear fit residuals w_fit (O - C); its angle is touched by nothing."""
    d = w.arap_warp(3, 3, seed=1, n_constraints=1, margin=1)
    d["mask"] = np.ones((3, 3), np.uint8)
    d["mask"][1, 1] = 0
    d["C"] = -np.ones((2, 3, 3))
    d["C"][:, 1, 1] = target
    d["U"] = d["U"] + 17.0
    x0 = np.concatenate([d["U"], np.zeros((1, 3, 3))])
    x0[0, 1, 1] = target[0] + x0_off[0]
    x0[1, 1, 1] = target[1] + x0_off[1]
    d["x0"] = x0
    return d


def linear_lm_offsets(x0_off, radius0, K):
    """x - C after each of K accepted steps of LM on a linear residual: the
    gain ratio is 1, so the radius triples every step (the update divides by
    max(1/3, 1 - 1) = 1/3), and the damped step d = -(x - C)/(1 + lambda)
    leaves (x - C) lambda/(1 + lambda)."""
    off = np.array(x0_off, float)
    out = []
    radius = radius0
    for _ in range(K):
        lam = 1.0 / radius
        off = off * lam / (1.0 + lam)
        out.append(off.copy())
        radius *= 3.0
    return out


def test_lm_linear_gain_ratio_one_triples_radius():
    d = _one_pixel_warp()
    e = o.make_energy(d)
    hist = []
    x, costs, acc = o.levenberg_marquardt(e, d["x0"], 4, 3, o.LMParams(radius0=1.0), history=hist)
    assert all(acc)
    assert [h["radius_used"] for h in hist] == pytest.approx([1.0, 3.0, 9.0, 27.0], rel=1e-15)
    assert [h["rho"] for h in hist] == pytest.approx([1.0] * 4, rel=1e-12)
    want = linear_lm_offsets((2.0, -1.5), 1.0, 4)[-1]
    xs = x.reshape(3, 3, 3)
    # (x is near 20 and 30, so x - C carries about 4e-15 of absolute rounding)
    assert np.allclose([xs[0, 1, 1] - 20.0, xs[1, 1, 1] - 30.0], want, rtol=0, atol=1e-13)
    # (1/2)(1/4)(1/10)(1/28): lambda = 1, 1/3, 1/9, 1/27
    assert np.allclose(want, np.array([2.0, -1.5]) / 2240.0, rtol=1e-14)


def test_lm_all_rejected_radius_halves_with_growing_nu():
    d = _one_pixel_warp()
    e = o.make_energy(d)
    hist = []
    prm = o.LMParams(radius0=1.0, min_rel_decrease=2.0)
    x, costs, acc = o.levenberg_marquardt(e, d["x0"], 5, 3, prm, history=hist)
    assert not any(acc)
    assert np.array_equal(x, d["x0"].ravel())
    # nu = 2, 4, 8, ...: radius 1 -> 1/2 -> 1/8 -> 1/64 -> 1/1024 -> 1/32768
    assert [h["radius"] for h in hist] == [0.5, 0.125, 1 / 64, 1 / 1024, 1 / 32768]
    # and the solve stops once the radius is below its minimum
    hist2 = []
    prm2 = o.LMParams(radius0=1e-30, radius_min=1e-32, min_rel_decrease=2.0)
    x2, costs2, acc2 = o.levenberg_marquardt(e, d["x0"], 10, 3, prm2, history=hist2)
    # 1e-30 / 2 / 4 / 8 = 1.56e-32 >= 1e-32, then / 16 = 9.8e-34 < 1e-32: four iterations
    assert len(acc2) == 4


class _ScalarQuadratic:
    """One unknown, one residual f(x) = x^2 - c (complex-safe for the
    complex-step Jacobian)."""
    n_chan = 1
    n_sites = 1

    def __init__(self, c):
        self.c = c
        self.active = np.array([True])

    def residuals(self, x):
        x = np.asarray(x).ravel()
        return np.array([x[0] * x[0] - self.c])

    def row_sites(self):
        return np.array([[0]])

    def site_colors(self):
        return np.array([0]), 1


def test_lm_scalar_golden_trace():
    g = json.load(open(os.path.join(GOLDEN, "lm_scalar_trace.json")))
    e = _ScalarQuadratic(g["c"])
    hist = []
    x, costs, acc = o.levenberg_marquardt(e, np.array([g["x0"]]), g["iters"], 1,
                                          o.LMParams(radius0=g["radius0"]), history=hist)
    steps = g["steps"]
    assert len(hist) == len(steps)
    assert acc == [s["accepted"] for s in steps]
    for h, s, E in zip(hist, steps, costs):
        assert h["radius_used"] == pytest.approx(s["radius_used"], rel=1e-12)
        assert h["radius"] == pytest.approx(s["radius"], rel=1e-12)
        assert h["rho"] == pytest.approx(s["rho"], rel=1e-9, abs=1e-12)
        assert E == pytest.approx(s["E0"], rel=1e-12)
    assert x[0] == pytest.approx(g["x_final"], rel=1e-12)
    # the trace covers both branches and unclamped radius updates
    rho_acc = [s["rho"] for s in steps if s["accepted"]]
    assert any(0.1 < r < 0.9 for r in rho_acc) and not all(s["accepted"] for s in steps)
