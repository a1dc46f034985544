"""Multi-pass optimisation (Sec. 7) in the oracle: the steps between solves of a
hierarchical (coarse-to-fine) optical flow (Appendix A.2.3), written from their
definitions, FP64, plain numpy.

Test infrastructure only (as the rest of ``oracle/``): tests, the smoke check
and the benchmark's CPU baseline use it; the HIP path does not.

Readings (the paper names the hierarchical scheme but not its resampling):
* level l of a pyramid has floor(W / 2^l) x floor(H / 2^l) pixels; its images
  are 2 x 2 block means of the level above (a box filter);
* the derivative images a level's flow energy samples are recomputed on that
  level: central differences inside, one-sided differences on the first and
  last column / row (the same construction the level-0 inputs use);
* the coarsest level starts from zero flow; a coarse solution is carried to the
  finer level by bilinear, clamp-to-edge sampling at the coarse point under
  each fine pixel's centre, x_c = (x_f + 1/2) Wc/Wf - 1/2, and scaled by the size
  ratio (flow is measured in pixels of its level).
"""
import numpy as np

from .energies import OpticalFlow, bilinear_clamped
from .solver import gauss_newton


def downsample2(img):
    """Mean of each 2 x 2 block of the last two axes (H, W); odd trailing rows or
    columns are dropped."""
    img = np.asarray(img, float)
    H, W = img.shape[-2], img.shape[-1]
    h, w = H // 2, W // 2
    a = img[..., 0:2 * h:2, 0:2 * w:2]
    b = img[..., 0:2 * h:2, 1:2 * w:2]
    c = img[..., 1:2 * h:2, 0:2 * w:2]
    d = img[..., 1:2 * h:2, 1:2 * w:2]
    return 0.25 * ((a + b) + (c + d))


def gradient(img):
    """(d/dx, d/dy) of an H x W image: central differences inside, one-sided on
    the border columns / rows, 0 along a dimension of one pixel."""
    img = np.asarray(img, float)
    H, W = img.shape
    dx = np.zeros_like(img)
    dy = np.zeros_like(img)
    if W > 1:
        dx[:, 1:-1] = (img[:, 2:] - img[:, :-2]) * 0.5
        dx[:, 0] = img[:, 1] - img[:, 0]
        dx[:, -1] = img[:, -1] - img[:, -2]
    if H > 1:
        dy[1:-1, :] = (img[2:, :] - img[:-2, :]) * 0.5
        dy[0, :] = img[1, :] - img[0, :]
        dy[-1, :] = img[-1, :] - img[-2, :]
    return dx, dy


def upsample(field, Wd, Hd, scale):
    """field: planes x Hs x Ws.  Returns planes x Hd x Wd: plane c sampled at the
    coarse point under each fine pixel centre and multiplied by scale[c]."""
    field = np.asarray(field, float)
    _, Hs, Ws = field.shape
    j, i = np.meshgrid(np.arange(Hd, dtype=float), np.arange(Wd, dtype=float), indexing="ij")
    x = (i + 0.5) * (Ws / Wd) - 0.5
    y = (j + 0.5) * (Hs / Hd) - 0.5
    return np.stack([scale[c] * bilinear_clamped(field[c], x, y) for c in range(field.shape[0])])


def pyramid_sizes(W, H, levels):
    return [(W >> l, H >> l) for l in range(levels)]


def flow_pyramid(I, Ihat, levels, w_fit, w_reg, outer, inner, x0=None, use_precond=True, callback=None):
    """Coarse-to-fine optical flow.  Returns (flow 2 x H x W at level 0, per-level
    cost traces finest first).  x0 is the starting flow when levels == 1 (zero by
    default); with more levels the coarsest starts from zero."""
    I = np.asarray(I, float)
    Ihat = np.asarray(Ihat, float)
    H, W = I.shape
    sizes = pyramid_sizes(W, H, levels)
    Is, Ihs = [I], [Ihat]
    for _ in range(1, levels):
        Is.append(downsample2(Is[-1]))
        Ihs.append(downsample2(Ihs[-1]))
    grads = [gradient(h) for h in Ihs]
    traces = [None] * levels
    Wl, Hl = sizes[-1]
    x = np.zeros((2, Hl, Wl)) if (levels > 1 or x0 is None) else np.asarray(x0, float).reshape(2, H, W)
    for l in range(levels - 1, -1, -1):
        Wl, Hl = sizes[l]
        e = OpticalFlow(Wl, Hl, Is[l], Ihs[l], grads[l][0], grads[l][1], w_fit, w_reg)
        xs, costs = gauss_newton(e, x.ravel(), outer, inner, use_precond)
        traces[l] = costs
        x = xs.reshape(2, Hl, Wl)
        if callback is not None:
            callback(l, x)
        if l > 0:
            Wf, Hf = sizes[l - 1]
            x = upsample(x, Wf, Hf, (Wf / Wl, Hf / Hl))
    return x, traces
