"""Image formation for the synthetic shape-from-shading input.

The shading image a camera would record of a smooth depth field under distant
lighting described by nine spherical-harmonic coefficients (the lighting model of
the shape-from-shading example, Appendix A.1.3).  This is scene synthesis only:
the surface normal is the exact normal of the continuous, back-projected depth
field, taken from the analytic depth gradient that the seeded generator returns,
not the one-pixel difference normal the energy evaluates, and nothing here is a
residual or a derivative of one.
"""
import numpy as np


def surface_normals(depth, d_di, d_dj, fx, fy, ux, uy):
    """Unit normals (n_x, n_y, n_z) of the surface P(i, j) = ((i-u_x)/f_x z,
    (j-u_y)/f_y z, z), z = depth(i, j), from the depth's partial derivatives along
    i (columns) and j (rows).  Oriented toward the camera: a fronto-parallel
    surface has normal (0, 0, -1).  Arrays are [H, W]."""
    H, W = depth.shape
    j, i = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    kx, ky = (i - ux) / fx, (j - uy) / fy
    # tangents dP/di and dP/dj
    ti = np.stack([(depth + (i - ux) * d_di) / fx, ky * d_di, d_di])
    tj = np.stack([kx * d_dj, (depth + (j - uy) * d_dj) / fy, d_dj])
    n = -np.cross(ti, tj, axis=0)
    return n / np.linalg.norm(n, axis=0)


def sh_shading(n, L):
    """Brightness of unit normals n ([3, ...]) under the nine lighting
    coefficients L: constant, the three linear terms (y, z, x) and the five
    quadratic terms (xy, yz, 3z^2 - 1, zx, x^2 - y^2) of real spherical harmonics
    up to order two, each without its normalisation constant."""
    x, y, z = n
    basis = (np.ones_like(x), y, z, x, x * y, y * z, 3.0 * z * z - 1.0, z * x, x * x - y * y)
    return sum(float(c) * b for c, b in zip(L, basis))


def shade_surface(depth, d_di, d_dj, fx, fy, ux, uy, L):
    """Rendered intensity [H, W] of the depth field under lighting L."""
    return sh_shading(surface_normals(depth, d_di, d_dj, fx, fy, ux, uy), L)
