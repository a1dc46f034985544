"""Seeded 3D grid workload: ARAP volumetric deformation of a voxel block."""
import numpy as np


def arap_volume(W, H, D, seed=6, handle_frac=0.01, sigma=0.5, w_fit=10.0, w_reg=1.0):
    """ARAP deformation of a W x H x D voxel block (voxel (i, j, k) at index
    (k*H + j)*W + i).

    Rest positions U are the lattice points (i, j, k) (unit spacing).  The voxels
    of the bottom face (k = 0) are anchored (target = U); besides them
    floor(handle_frac * n) voxels (at least one), drawn without replacement from
    the rest, get targets U + N(0, sigma^2) per component.  Other voxels carry the
    target (-1e7, -1e7, -1e7), below the validity threshold of the fit term.
    Unknowns (offset xyz, Euler angles xyz) start at (U, 0).
    """
    rng = np.random.default_rng(seed)
    k, j, i = np.meshgrid(np.arange(D, dtype=float), np.arange(H, dtype=float), np.arange(W, dtype=float),
                          indexing="ij")
    U = np.stack([i.ravel(), j.ravel(), k.ravel()])
    n = W * H * D
    C = np.full((3, n), -1e7)
    base = np.arange(W * H)
    C[:, base] = U[:, base]
    rest = np.arange(W * H, n)
    m = max(1, int(np.floor(handle_frac * n))) if len(rest) else 0
    handles = rng.choice(rest, m, replace=False) if m else np.zeros(0, np.int64)
    C[:, handles] = U[:, handles] + rng.normal(0.0, sigma, (3, m))
    x0 = np.concatenate([U, np.zeros((3, n))])
    return dict(energy="arap_volume", W=W, H=H, D=D, U=U, C=C, x0=x0, handles=np.sort(handles),
                params=dict(w_fit=w_fit, w_reg=w_reg))


def lattice_edges(W, H, D):
    """Edges of a W x H x D voxel lattice to the +x, +y and +z neighbours (voxel
    index (k*H + j)*W + i): all x edges in index order, then y, then z."""
    s = np.arange(W * H * D).reshape(D, H, W)
    ex = np.stack([s[:, :, :-1].ravel(), s[:, :, 1:].ravel()], 1)
    ey = np.stack([s[:, :-1, :].ravel(), s[:, 1:, :].ravel()], 1)
    ez = np.stack([s[:-1, :, :].ravel(), s[1:, :, :].ravel()], 1)
    return np.concatenate([ex, ey, ez]).astype(np.int32)
