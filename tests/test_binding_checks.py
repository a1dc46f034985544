"""The binding refuses, on the host and before any pointer reaches the library,
data arrays and unknowns that do not match what the kernels will read and write:
wrong dtype for the precision, too few or too many elements, a non-contiguous
view, a host tensor, a wrong number of arrays.  No GPU is needed."""
import pytest
import torch

import paper_1604_06525_amd as pkg

N = 12 * 10  # sites


def _warp(dt=torch.float32):
    return [torch.zeros(2 * N, dtype=dt), torch.zeros(2 * N, dtype=dt), torch.zeros(N, dtype=torch.uint8)]


@pytest.mark.parametrize("case,arrays,x,match", [
    ("x in float64 under mixed", _warp(), torch.zeros(3 * N, dtype=torch.float64), "dtype torch.float32"),
    ("x too short", _warp(), torch.zeros(3 * N - 1), "360 elements"),
    ("x not contiguous", _warp(), torch.zeros(3 * N * 2)[::2], "contiguous"),
    ("bulk array in float64", [torch.zeros(2 * N, dtype=torch.float64)] + _warp()[1:], torch.zeros(3 * N),
     "array 0"),
    ("mask not uint8", _warp()[:2] + [torch.zeros(N)], torch.zeros(3 * N), "array 2"),
    ("targets one plane short", [_warp()[0], torch.zeros(N), _warp()[2]], torch.zeros(3 * N), "240 elements"),
    ("missing array", _warp()[:2], torch.zeros(3 * N), "takes 3 arrays"),
    ("host tensors", _warp(), torch.zeros(3 * N), "CUDA device"),
])
def test_mismatched_request_raises(case, arrays, x, match):
    with pytest.raises(ValueError, match=match):
        pkg.check_request("arap_warp", arrays, x, "mixed", N)


def test_every_energy_has_an_array_spec():
    assert set(pkg.ARRAY_SPEC) == set(pkg.ENERGIES)


def test_channel_table_matches_the_library():
    if not __import__("os").path.exists(pkg.LIB_PATH):
        from paper_1604_06525_amd import build
        build.build()
    for e in pkg.ARRAY_SPEC:
        assert pkg.len_channels(e) == pkg.energy_channels(e), e
