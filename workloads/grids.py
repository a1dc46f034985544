"""Seeded 2D-grid workloads.

Arrays use the planar layout the library takes: a c-channel field is a
``[c, H, W]`` float64 array whose last index ``i`` runs along the image width
(the first grid dimension of the paper's listings) and whose middle index ``j``
runs along the height.  Masks are ``uint8`` ``[H, W]``.  Callers cast the bulk
arrays to float32 for the mixed-precision path.
"""
import numpy as np
from scipy.ndimage import gaussian_filter

from .noise import sinusoid_field, Perlin2D
from .render import shade_surface

# Spherical-harmonic lighting coefficients L1..L9 for shape from shading.  A
# surface facing the camera, normal (0,0,-1), is lit with brightness
# L1 - L3 + 2*L7 = 0.9.
SFS_LIGHTING = (0.5, 0.05, -0.3, 0.05, 0.0, 0.0, 0.05, 0.0, 0.0)


def _lattice(W, H):
    j, i = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    return i, j


def _mask(kind, W, H, rng, frac=0.05):
    m = np.zeros((H, W), np.uint8)
    if kind == "none":
        return m
    if kind == "random":
        m[rng.random((H, W)) < frac] = 1
        return m
    if kind == "hole":
        i, j = _lattice(W, H)
        r = 0.15 * min(W, H)
        m[(i - 0.3 * W) ** 2 + (j - 0.6 * H) ** 2 < r * r] = 1
        return m
    raise ValueError(kind)


def arap_warp(W, H, seed=1, n_constraints=None, sigma=3.0, margin=8, mask="none",
              w_fit=10.0, w_reg=1.0):
    """As-rigid-as-possible image warp on a W x H pixel lattice.

    Rest shape U(i,j) = (i,j).  ``n_constraints`` pixels (default: 32 per 64x64,
    i.e. W*H/128) are drawn without replacement from the interior rectangle
    [margin, W-margin) x [margin, H-margin); their targets are U plus
    N(0, sigma^2) pixels per component.  Every other pixel carries the target
    (-1, -1), which fails the non-negative-target validity test of the fit term.
    Unknowns start at O = U, angle = 0.
    """
    rng = np.random.default_rng(seed)
    i, j = _lattice(W, H)
    U = np.stack([i, j])
    if n_constraints is None:
        n_constraints = max(1, (W * H) // 128)
    m = max(0, min(margin, (W - 1) // 2, (H - 1) // 2))
    iw, jh = W - 2 * m, H - 2 * m
    n_constraints = min(n_constraints, iw * jh)
    pick = rng.choice(iw * jh, n_constraints, replace=False)
    ci = pick % iw + m
    cj = pick // iw + m
    C = -np.ones((2, H, W))
    C[0, cj, ci] = U[0, cj, ci] + rng.normal(0.0, sigma, n_constraints)
    C[1, cj, ci] = U[1, cj, ci] + rng.normal(0.0, sigma, n_constraints)
    Mask = _mask(mask, W, H, rng)
    x0 = np.concatenate([U, np.zeros((1, H, W))])
    return dict(energy="arap_warp", W=W, H=H, U=U, C=C, mask=Mask, x0=x0,
                params=dict(w_fit=w_fit, w_reg=w_reg))


def _smooth_rgba(W, H, rng, lo, hi):
    chans = []
    for _ in range(4):
        v, _, _ = sinusoid_field((H, W), rng, 6, max(4.0, W / 6), max(8.0, 1.5 * W))
        chans.append(lo + (hi - lo) * (0.5 + 0.5 * v))
    return np.stack(chans)


def poisson_edit(W, H, seed=5, mask="rect"):
    """Poisson image editing: paste the gradients of T into base over a region.

    base and T are smooth seeded RGBA fields in [0, 1].  The unknown region
    (mask 0) is the central rectangle [W/4, 3W/4) x [H/4, 3H/4); everywhere else
    the mask is 1 and the pixel keeps its base value.  Unknowns start at base.
    """
    rng = np.random.default_rng(seed)
    base = _smooth_rgba(W, H, rng, 0.1, 0.9)
    T = _smooth_rgba(W, H, rng, 0.0, 1.0) + 0.02 * rng.normal(size=(4, H, W))
    M = np.ones((H, W), np.uint8)
    if mask == "rect":
        M[H // 4:(3 * H) // 4, W // 4:(3 * W) // 4] = 0
    elif mask == "all":
        M[:] = 0
    else:
        raise ValueError(mask)
    return dict(energy="poisson", W=W, H=H, T=T, mask=M, x0=base.copy(), base=base, params={})


def shape_from_shading(W, H, seed=2, amplitude=None, noise=0.01, invalid="none",
                       edge_zero_frac=0.0, w_p=1.0, w_s=100.0, w_g=1.0, focal=None, center=None,
                       lighting=SFS_LIGHTING):
    """Depth refinement from shading.

    True depth = 1.5 + amplitude * g, with g a sum of 16 seeded plane waves of
    period W/8 .. W, scaled to max |g| = 1.  The default amplitude 0.1*min(1, W/1024)
    keeps neighbouring depth differences at or below about 0.005.  The input depth
    D_i is a Gaussian blur (sigma 4 px) of the true depth.  The intensity image is
    the true surface rendered under ``lighting`` (``render.shade_surface``: the
    analytic surface normal of the back-projected depth field, lit by the
    second-order spherical-harmonic model) plus N(0, noise^2).  Edge masks are 1
    (``edge_zero_frac`` zeroes a random fraction of them).  ``invalid="hole"``
    sets D_i = 0 (no depth) inside a disc, which excludes those pixels.
    ``focal`` is f, or (f_x, f_y) (default 1000 W/1024 for both); ``center`` is
    (u_x, u_y) (default the image centre).  Unknown X starts at D_i.
    """
    rng = np.random.default_rng(seed)
    if amplitude is None:
        amplitude = 0.1 * min(1.0, W / 1024.0)
    g, gi, gj = sinusoid_field((H, W), rng, 16, max(2.0, W / 8.0), float(W))
    s = 1.0 / np.max(np.abs(g))
    depth = 1.5 + amplitude * s * g
    di, dj = amplitude * s * gi, amplitude * s * gj
    if focal is None:
        focal = 1000.0 * W / 1024.0
    fx, fy = (float(focal), float(focal)) if np.isscalar(focal) else (float(focal[0]), float(focal[1]))
    ux, uy = ((W - 1) / 2.0, (H - 1) / 2.0) if center is None else (float(center[0]), float(center[1]))
    Im = shade_surface(depth, di, dj, fx, fy, ux, uy, lighting) + rng.normal(0.0, noise, (H, W))
    D = gaussian_filter(depth, 4.0, mode="nearest")
    if invalid == "hole":
        i, j = _lattice(W, H)
        r = 0.12 * min(W, H)
        D[(i - 0.35 * W) ** 2 + (j - 0.4 * H) ** 2 < r * r] = 0.0
    elif invalid != "none":
        raise ValueError(invalid)
    eR = np.ones((H, W), np.uint8)
    eC = np.ones((H, W), np.uint8)
    if edge_zero_frac > 0:
        eR[rng.random((H, W)) < edge_zero_frac] = 0
        eC[rng.random((H, W)) < edge_zero_frac] = 0
    params = dict(w_p=w_p, w_s=w_s, w_g=w_g, f_x=fx, f_y=fy, u_x=ux, u_y=uy, L=tuple(lighting))
    return dict(energy="sfs", W=W, H=H, D=D, Im=Im, edge_r=eR, edge_c=eC,
                x0=D[None].copy(), depth_true=depth, params=params)


def optical_flow(W, H, seed=4, max_flow=1.5, base_period=64.0, w_fit=1.0, w_reg=0.02):
    """Dense optical flow between a Perlin-noise texture and a warped copy.

    I = 4-octave Perlin noise (base period 64 px) on the pixel lattice.  The true
    flow f is a sum of 8 seeded plane waves per component (periods >= max(W,H)/4,
    at least 16 px), scaled to max |f| = max_flow.  The second frame is
    I_hat(x) = I(x - f(x)), evaluated from the noise function itself; its
    derivative images are central differences (one-sided at the border).
    Unknown flow starts at (0, 0).
    """
    rng = np.random.default_rng(seed)
    layers = [Perlin2D(rng) for _ in range(4)]

    def tex(x, y):
        out = 0.0
        amp, freq, tot = 1.0, 1.0 / base_period, 0.0
        for layer in layers:
            out = out + amp * layer(x * freq, y * freq)
            tot += amp
            amp *= 0.5
            freq *= 2.0
        return np.clip(0.5 + 0.5 * out / (0.71 * tot), 0.0, 1.0)

    i, j = _lattice(W, H)
    pmin = max(16.0, max(W, H) / 4.0)
    fu, _, _ = sinusoid_field((H, W), rng, 8, pmin, 4.0 * pmin)
    fv, _, _ = sinusoid_field((H, W), rng, 8, pmin, 4.0 * pmin)
    mag = np.sqrt(fu * fu + fv * fv).max()
    fu *= max_flow / mag
    fv *= max_flow / mag
    I0 = tex(i, j)
    I1 = tex(i - fu, j - fv)
    dy, dx = np.gradient(I1)
    return dict(energy="flow", W=W, H=H, I=I0, Ihat=I1, Ihat_dx=dx, Ihat_dy=dy,
                x0=np.zeros((2, H, W)), flow_true=np.stack([fu, fv]),
                params=dict(w_fit=w_fit, w_reg=w_reg))


def laplacian_grid(W, H, seed=0, w_fit=0.1, w_reg=0.9):
    """Laplacian smoothing of a noisy smooth image (weights of the paper's example)."""
    rng = np.random.default_rng(seed)
    v, _, _ = sinusoid_field((H, W), rng, 4, max(2.0, W / 4), float(max(W, 4)))
    A = v + 0.1 * rng.normal(size=(H, W))
    return dict(energy="laplacian", W=W, H=H, A=A[None], x0=np.zeros((1, H, W)),
                params=dict(w_fit=w_fit, w_reg=w_reg))


def lp_smooth(W, H, seed=0, p=1.0, eps=1e-2, w_fit=1.0, w_reg=0.5, noise=0.1, blocks=12):
    """Edge-preserving smoothing input: a piecewise-constant image (random
    axis-aligned blocks of random grey levels over a background) plus Gaussian
    noise; the solve starts from the noisy image."""
    rng = np.random.default_rng(seed)
    A = np.full((H, W), 0.5)
    for _ in range(blocks):
        x0, y0 = rng.integers(0, W), rng.integers(0, H)
        w, h = rng.integers(max(1, W // 8), max(2, W // 2)), rng.integers(max(1, H // 8), max(2, H // 2))
        A[y0:y0 + h, x0:x0 + w] = rng.uniform(0.0, 1.0)
    A = A + noise * rng.normal(size=(H, W))
    return dict(energy="lp_smooth", W=W, H=H, A=A[None], x0=A[None].copy(),
                params=dict(w_fit=w_fit, w_reg=w_reg, p=p, eps=eps))


def intrinsic_image(W, H, seed=0, p=0.8, eps=1e-2, w_fit=1.0, w_a=1.0, w_s=3.0, noise=0.02, blocks=12):
    """Intrinsic decomposition input in the log domain: a reflectance that is
    piecewise constant per channel (random axis-aligned blocks of random
    colours over a background), plus a smooth shading field (a seeded sum of
    plane waves), plus Gaussian noise per channel.  The solve starts with all of
    the image as reflectance and zero shading."""
    rng = np.random.default_rng(seed)
    R = np.empty((3, H, W))
    R[:] = rng.uniform(-0.5, 0.5, size=(3, 1, 1))
    for _ in range(blocks):
        x0, y0 = rng.integers(0, W), rng.integers(0, H)
        w, h = rng.integers(max(1, W // 8), max(2, W // 2)), rng.integers(max(1, H // 8), max(2, H // 2))
        R[:, y0:y0 + h, x0:x0 + w] = rng.uniform(-1.0, 0.5, size=(3, 1, 1))
    S, _, _ = sinusoid_field((H, W), rng, 4, max(2.0, W / 2), float(max(W, 4)))
    I = R + 0.5 * S[None] + noise * rng.normal(size=(3, H, W))
    x0 = np.concatenate([I, np.zeros((1, H, W))])
    return dict(energy="intrinsic", W=W, H=H, I=I, x0=x0,
                params=dict(w_fit=w_fit, w_a=w_a, w_s=w_s, p=p, eps=eps))
