import numpy as np
import pytest

import workloads as w


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_icosphere_counts(level):
    v, f, e = w.icosphere(level)
    assert len(v) == 10 * 4 ** level + 2
    assert len(f) == 20 * 4 ** level
    assert len(e) == 30 * 4 ** level
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    assert len(np.unique(np.sort(e, 1), axis=0)) == len(e)
    deg = np.bincount(e.ravel(), minlength=len(v))
    assert deg.min() == 5 and deg.max() == (5 if level == 0 else 6)


def test_morton_is_permutation():
    v, _, _ = w.icosphere(3)
    p = w.morton_order(v)
    assert np.array_equal(np.sort(p), np.arange(len(v)))


@pytest.mark.parametrize("gen,args", [
    (w.arap_warp, (20, 17)), (w.poisson_edit, (20, 17)), (w.shape_from_shading, (20, 17)),
    (w.optical_flow, (20, 17)), (w.laplacian_grid, (5, 4)), (w.arap_mesh, (2,)),
])
def test_deterministic(gen, args):
    a, b = gen(*args), gen(*args)
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), k


def test_warp_constraints():
    d = w.arap_warp(64, 64, seed=1)
    valid = (d["C"][0] >= 0) & (d["C"][1] >= 0)
    assert (d["C"][0] != -1).sum() == 32
    jj, ii = np.nonzero(d["C"][0] != -1)
    assert ii.min() >= 8 and ii.max() < 56 and jj.min() >= 8 and jj.max() < 56
    assert valid.sum() <= 32


def test_sfs_neighbour_differences_small():
    d = w.shape_from_shading(256, 256, seed=2)
    X = d["x0"][0]
    assert np.abs(np.diff(X, axis=0)).max() < 0.005
    assert np.abs(np.diff(X, axis=1)).max() < 0.005
