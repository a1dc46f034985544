"""Pins of the oracle's Jacobian against mechanisms independent of its assembly.

* colour-grouped complex-step J == J built one column at a time (no colouring, no
  declared row structure): pins the colouring and ``row_sites``;
* J == central finite differences of F in real arithmetic: pins the complex-step
  derivative against plain differencing of the residual functions;
* optical flow: on a linear ramp image the bilinear sample is exact and the
  central-difference derivative images equal the ramp slopes, so the sampled-image
  partials (Sec. 7) must equal finite differences of the sampled value.
"""
import numpy as np
import pytest

import oracle as o
import workloads as w


def _rand_state(d, rng, scale):
    x = d["x0"].copy()
    x = x + scale * rng.normal(size=x.shape)
    return x


def _cases():
    rng = np.random.default_rng(11)
    out = []
    d = w.arap_warp(7, 6, seed=3, n_constraints=8, margin=1, mask="random")
    x = _rand_state(d, rng, 0.3)
    out.append(("arap_warp", d, x))
    d = w.poisson_edit(6, 5, seed=3)
    out.append(("poisson", d, _rand_state(d, rng, 0.1)))
    d = w.shape_from_shading(7, 6, seed=3, amplitude=0.002, invalid="none", edge_zero_frac=0.2)
    out.append(("sfs", d, d["x0"] + 1e-4 * rng.normal(size=d["x0"].shape)))
    d = w.shape_from_shading(9, 8, seed=4, amplitude=0.002, invalid="hole")
    out.append(("sfs_hole", d, d["x0"] + 1e-4 * rng.normal(size=d["x0"].shape)))
    # distinct focal lengths and centre coordinates, every lighting coefficient non-zero
    d = w.shape_from_shading(8, 7, seed=5, amplitude=0.002, focal=(6.5, 9.0), center=(3.2, 2.6),
                             lighting=(0.5, 0.07, -0.3, 0.04, 0.03, -0.02, 0.05, 0.06, -0.04))
    out.append(("sfs_general", d, d["x0"] + 1e-4 * rng.normal(size=d["x0"].shape)))
    d = w.arap_mesh(1, seed=3, handle_frac=0.1)
    out.append(("arap_mesh", d, _rand_state(d, rng, 0.2)))
    d = w.laplacian_grid(5, 4, seed=2)
    out.append(("laplacian", d, _rand_state(d, rng, 0.5)))
    d = w.laplacian_mesh(1, seed=2)
    out.append(("laplacian_graph", d, _rand_state(d, rng, 0.5)))
    return out


CASES = _cases()


@pytest.mark.parametrize("name,d,x", CASES, ids=[c[0] for c in CASES])
def test_colored_equals_columnwise(name, d, x):
    e = o.make_energy(d)
    J = o.jacobian(e, x).toarray()
    Jb = o.jacobian_dense_bruteforce(e, x)
    assert J.shape == Jb.shape
    assert np.abs(J - Jb).max() <= 1e-14 * max(1.0, np.abs(Jb).max())


@pytest.mark.parametrize("name,d,x", CASES, ids=[c[0] for c in CASES])
def test_matches_finite_differences(name, d, x):
    e = o.make_energy(d)
    if name.startswith("sfs"):
        # stay away from the switch of the smoothness validity test
        X = x.reshape(d["H"], d["W"])
        for k in range(X.size):
            for sgn in (1, -1):
                xp = x.ravel().copy()
                xp[k] += sgn * 1e-6 * max(1, abs(xp[k]))
                assert np.array_equal(e.smooth_valid(xp.reshape(X.shape)), e.smooth_valid(X))
    J = o.jacobian(e, x).toarray()
    Jfd = o.fd_jacobian(e, x)
    scale = max(1.0, np.abs(J).max())
    assert np.abs(J - Jfd).max() <= 1e-6 * scale, np.abs(J - Jfd).max()


def test_sfs_has_all_residual_kinds():
    d = w.shape_from_shading(9, 8, seed=4, amplitude=0.002)
    e = o.make_energy(d)
    x = d["x0"] + 1e-4 * np.random.default_rng(1).normal(size=d["x0"].shape)
    F = e.residuals(x)
    n = 72
    blocks = F.reshape(6, n)
    for k in range(6):
        assert np.count_nonzero(blocks[k]) > 0


def test_flow_sampled_partials_on_linear_ramp():
    W, H = 9, 7
    a, b, c = 0.03, -0.02, 0.4
    j, i = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
    ramp = a * i + b * j + c
    dy, dx = np.gradient(ramp)
    assert np.allclose(dx, a) and np.allclose(dy, b)
    rng = np.random.default_rng(5)
    I0 = rng.random((H, W))
    e = o.OpticalFlow(W, H, I0, ramp, dx, dy, w_fit=1.3, w_reg=0.2)
    x = rng.uniform(-0.4, 0.4, size=(2, H, W))
    J = o.jacobian(e, x).toarray()
    Jfd = o.fd_jacobian(e, x)
    n = W * H
    inner = ((i >= 1) & (i <= W - 2) & (j >= 1) & (j <= H - 2)).ravel()
    fit = np.arange(n)[inner]
    assert np.abs(J[fit] - Jfd[fit]).max() < 1e-8
    # the fit partials are the ramp slopes times -w_fit
    assert np.allclose(J[fit, fit], -1.3 * a) and np.allclose(J[fit, n + fit], -1.3 * b)
    # regularisation rows are exact everywhere
    assert np.abs(J[n:] - Jfd[n:]).max() < 1e-8


def test_flow_sampler_clamps_to_edge():
    img = np.arange(12, dtype=float).reshape(3, 4)
    s = o.energies.bilinear_clamped
    assert s(img, np.array(-5.0), np.array(-5.0)) == img[0, 0]
    assert s(img, np.array(10.0), np.array(1.0)) == img[1, 3]
    assert s(img, np.array(1.5), np.array(0.0)) == 0.5 * (img[0, 1] + img[0, 2])
    assert s(img, np.array(2.0), np.array(2.0)) == img[2, 2]
