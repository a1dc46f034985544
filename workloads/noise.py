"""Smooth seeded fields: sums of sinusoids and Perlin gradient noise.

Perlin noise follows Perlin's published improved-noise construction
(random unit gradients on an integer lattice, quintic fade 6t^5-15t^4+10t^3,
bilinear blend of the four corner dot products), written here from that
description; octaves are summed with halving amplitude and doubling frequency.
"""
import numpy as np


def sinusoid_field(shape, rng, n_terms, period_min, period_max):
    """Sum of ``n_terms`` plane waves with random direction, period and phase.

    Returns (value, d/di, d/dj) evaluated analytically on the pixel lattice,
    where i is the column (fast) index and j the row index.  The sum is divided by
    ``n_terms`` so each term has amplitude 1/n_terms.
    """
    H, W = shape
    j, i = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    v = np.zeros(shape)
    di = np.zeros(shape)
    dj = np.zeros(shape)
    for _ in range(n_terms):
        ang = rng.uniform(0, 2 * np.pi)
        per = rng.uniform(period_min, period_max)
        ph = rng.uniform(0, 2 * np.pi)
        k = 2 * np.pi / per
        kx, ky = k * np.cos(ang), k * np.sin(ang)
        arg = kx * i + ky * j + ph
        v += np.sin(arg)
        c = np.cos(arg)
        di += kx * c
        dj += ky * c
    return v / n_terms, di / n_terms, dj / n_terms


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


class Perlin2D:
    """Gradient noise on a periodic lattice of ``size`` cells per axis."""

    def __init__(self, rng, size=256):
        ang = rng.uniform(0, 2 * np.pi, size=(size, size))
        self.gx = np.cos(ang)
        self.gy = np.sin(ang)
        self.size = size

    def __call__(self, x, y):
        s = self.size
        x0 = np.floor(x)
        y0 = np.floor(y)
        fx = x - x0
        fy = y - y0
        ix = x0.astype(np.int64) % s
        iy = y0.astype(np.int64) % s
        ix1 = (ix + 1) % s
        iy1 = (iy + 1) % s

        def corner(cx, cy, ox, oy):
            return self.gx[cy, cx] * (fx - ox) + self.gy[cy, cx] * (fy - oy)

        n00 = corner(ix, iy, 0, 0)
        n10 = corner(ix1, iy, 1, 0)
        n01 = corner(ix, iy1, 0, 1)
        n11 = corner(ix1, iy1, 1, 1)
        u = _fade(fx)
        v = _fade(fy)
        nx0 = n00 + u * (n10 - n00)
        nx1 = n01 + u * (n11 - n01)
        return nx0 + v * (nx1 - nx0)


def perlin_texture(rng, x, y, base_period=64.0, octaves=4):
    """Fractal Perlin noise at pixel coordinates (x, y), rescaled to about [0, 1]."""
    layers = [Perlin2D(rng) for _ in range(octaves)]
    out = np.zeros(np.broadcast(x, y).shape)
    amp = 1.0
    freq = 1.0 / base_period
    total = 0.0
    for layer in layers:
        out += amp * layer(x * freq, y * freq)
        total += amp
        amp *= 0.5
        freq *= 2.0
    # plain 2D Perlin noise lies in about [-0.71, 0.71]; map the octave sum to [0, 1]
    return np.clip(0.5 + 0.5 * out / (0.71 * total), 0.0, 1.0)
