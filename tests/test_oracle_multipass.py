"""Pins of the oracle's multi-pass steps (Sec. 7; hierarchical flow of A.2.3):
block-mean downsampling, derivative images and bilinear upsampling, against
closed forms (constants, linear ramps) and against numpy's gradient; the
pyramid's degenerate one-level case against a plain Gauss-Newton solve."""
import numpy as np

import oracle
from oracle import multipass as mp
import workloads as w


def _ramp(W, H, a, b, c):
    j, i = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    return a * i + b * j + c


def test_downsample_constant_and_ramp():
    assert np.array_equal(mp.downsample2(np.full((6, 9), 3.5)), np.full((3, 4), 3.5))
    a, b, c = 0.75, -1.25, 2.0
    f = _ramp(11, 8, a, b, c)  # odd width: the last column is dropped
    g = mp.downsample2(f)
    assert g.shape == (4, 5)
    # the mean of a linear function over a 2 x 2 block is its value at the
    # block centre (2i + 1/2, 2j + 1/2)
    jj, ii = np.meshgrid(np.arange(4, dtype=float), np.arange(5, dtype=float), indexing="ij")
    assert np.allclose(g, a * (2 * ii + 0.5) + b * (2 * jj + 0.5) + c, rtol=0, atol=1e-13)
    # planes are resampled independently
    st = np.stack([f, 2 * f])
    assert np.array_equal(mp.downsample2(st)[1], mp.downsample2(2 * f))


def test_gradient_matches_numpy_and_ramps():
    rng = np.random.default_rng(3)
    img = rng.normal(size=(13, 17))
    dx, dy = mp.gradient(img)
    ny, nx = np.gradient(img)
    assert np.array_equal(dx, nx) and np.array_equal(dy, ny)
    # a linear ramp's differences are exact everywhere, borders included
    dx, dy = mp.gradient(_ramp(9, 7, 0.3, -2.0, 1.0))
    assert np.allclose(dx, 0.3, rtol=0, atol=1e-14) and np.allclose(dy, -2.0, rtol=0, atol=1e-14)
    # a single row or column has no derivative across it
    dx, dy = mp.gradient(np.arange(5.0)[None, :])
    assert np.array_equal(dy, np.zeros((1, 5))) and np.allclose(dx, 1.0)


def test_upsample_constant_and_linear():
    c = np.stack([np.full((5, 6), 1.5), np.full((5, 6), -0.5)])
    u = mp.upsample(c, 12, 10, (2.0, 3.0))
    assert np.allclose(u[0], 3.0) and np.allclose(u[1], -1.5)
    # bilinear sampling reproduces a linear field wherever the sample point is
    # inside the coarse grid (clamping only acts outside it)
    a, b = 0.4, -0.7
    Ws, Hs, Wd, Hd = 6, 5, 13, 11
    f = _ramp(Ws, Hs, a, b, 0.25)[None]
    u = mp.upsample(f, Wd, Hd, (2.0,))[0]
    jj, ii = np.meshgrid(np.arange(Hd, dtype=float), np.arange(Wd, dtype=float), indexing="ij")
    x = (ii + 0.5) * Ws / Wd - 0.5
    y = (jj + 0.5) * Hs / Hd - 0.5
    inside = (x >= 0) & (x <= Ws - 1) & (y >= 0) & (y <= Hs - 1)
    assert inside.sum() > Wd * Hd // 2
    assert np.allclose(u[inside], 2.0 * (a * x + b * y + 0.25)[inside], rtol=0, atol=1e-13)
    # and clamps to the edge outside: the corner pixel takes the corner value
    assert np.isclose(u[0, 0], 2.0 * f[0, 0, 0])


def test_pyramid_levels_and_sizes():
    assert mp.pyramid_sizes(100, 61, 3) == [(100, 61), (50, 30), (25, 15)]


def test_one_level_pyramid_is_a_plain_solve():
    d = w.optical_flow(40, 32, seed=4)
    x, traces = mp.flow_pyramid(d["I"], d["Ihat"], 1, d["params"]["w_fit"], d["params"]["w_reg"], 2, 8)
    xo, costs = oracle.gauss_newton(oracle.make_energy(d), d["x0"], 2, 8)
    assert np.allclose(traces[0], costs, rtol=1e-14, atol=0)
    assert np.allclose(x.ravel(), xo, rtol=0, atol=1e-14)


def test_pyramid_recovers_a_smooth_flow_better_than_one_level():
    # not an exactness pin: the coarse-to-fine scheme exists because a single
    # linearisation at zero flow cannot follow motions past a pixel or two
    d = w.optical_flow(96, 80, seed=7, max_flow=3.0)
    p = d["params"]
    err = []
    for levels in (1, 3):
        x, _ = mp.flow_pyramid(d["I"], d["Ihat"], levels, p["w_fit"], p["w_reg"], 4, 30)
        err.append(np.sqrt(((x - d["flow_true"]) ** 2).sum(0)).mean())
    assert err[1] < err[0]
