"""Seeded graph workloads: subdivided icospheres and ARAP handle sets."""
import itertools

import numpy as np


def _icosahedron():
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a, b in itertools.product((-1.0, 1.0), (-phi, phi)):
        v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v)
    # faces: vertex triples whose three pairwise distances equal the edge length 2
    faces = []
    for a, b, c in itertools.combinations(range(12), 3):
        if all(abs(np.linalg.norm(v[p] - v[q]) - 2.0) < 1e-9 for p, q in ((a, b), (b, c), (a, c))):
            if np.dot(np.cross(v[b] - v[a], v[c] - v[a]), v[a] + v[b] + v[c]) < 0:
                b, c = c, b
            faces.append((a, b, c))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, np.array(faces, np.int64)


def icosphere(level):
    """Unit icosphere after ``level`` midpoint subdivisions.

    Returns (vertices [V,3] float64, faces [F,3] int64, edges [E,2] int64) with
    V = 10*4^level + 2, F = 20*4^level, E = 30*4^level.  A new vertex takes the next
    id at the first visit of its edge (faces in order, edges ab, bc, ca); edges are
    listed once each, as (smaller id, larger id), in order of first visit.
    """
    v, f = _icosahedron()
    for _ in range(level):
        nv = len(v)
        e = np.stack([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=1).reshape(-1, 2)
        key = np.minimum(e[:, 0], e[:, 1]) * nv + np.maximum(e[:, 0], e[:, 1])
        uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
        order = np.argsort(first, kind="stable")
        rank = np.empty_like(order)
        rank[order] = np.arange(len(order))
        mid_id = nv + rank[inv].reshape(-1, 3)
        ue = np.stack([uniq // nv, uniq % nv], axis=1)[order]
        mids = v[ue[:, 0]] + v[ue[:, 1]]
        mids /= np.linalg.norm(mids, axis=1, keepdims=True)
        v = np.concatenate([v, mids])
        a, b, c = f[:, 0], f[:, 1], f[:, 2]
        mab, mbc, mca = mid_id[:, 0], mid_id[:, 1], mid_id[:, 2]
        f = np.concatenate([np.stack([a, mab, mca], 1), np.stack([b, mbc, mab], 1),
                            np.stack([c, mca, mbc], 1), np.stack([mab, mbc, mca], 1)])
    e = np.stack([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=1).reshape(-1, 2)
    key = np.minimum(e[:, 0], e[:, 1]) * len(v) + np.maximum(e[:, 0], e[:, 1])
    uniq, first = np.unique(key, return_index=True)
    order = np.argsort(first, kind="stable")
    edges = np.stack([uniq // len(v), uniq % len(v)], axis=1)[order]
    return v, f, edges


def morton_order(points, bits=10):
    """Permutation sorting points by the 3D Morton code of their quantised
    coordinates (ties keep the original order)."""
    lo = points.min(0)
    span = np.maximum(points.max(0) - lo, 1e-30)
    q = np.minimum(((points - lo) / span * (2 ** bits)).astype(np.int64), 2 ** bits - 1)
    code = np.zeros(len(points), np.int64)
    for b in range(bits):
        for k in range(3):
            code |= ((q[:, k] >> b) & 1) << (3 * b + k)
    return np.argsort(code, kind="stable")


def _reorder(v, edges, perm):
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    return v[perm], inv[edges]


def arap_mesh(level, seed=3, handle_frac=0.01, sigma=0.05, reorder=True, w_fit=10.0, w_reg=1.0):
    """ARAP deformation of an icosphere of the given subdivision level.

    Rest positions U are the unit-sphere vertices (Morton-ordered when
    ``reorder``).  floor(handle_frac*V) handles (at least one) are drawn without
    replacement; their targets are U + N(0, sigma^2) per component.  Other
    vertices carry the target (-1e7, -1e7, -1e7), below the validity threshold of
    the fit term.  Unknowns (offset xyz, Euler angles xyz) start at (U, 0).
    """
    rng = np.random.default_rng(seed)
    v, _, edges = icosphere(level)
    if reorder:
        v, edges = _reorder(v, edges, morton_order(v))
    V = len(v)
    k = max(1, int(np.floor(handle_frac * V)))
    handles = rng.choice(V, k, replace=False)
    U = v.T.copy()
    C = np.full((3, V), -1e7)
    C[:, handles] = U[:, handles] + rng.normal(0.0, sigma, (3, k))
    x0 = np.concatenate([U, np.zeros((3, V))])
    return dict(energy="arap_mesh", V=V, edges=edges.astype(np.int32), U=U, C=C, x0=x0,
                handles=np.sort(handles), params=dict(w_fit=w_fit, w_reg=w_reg))


def laplacian_mesh(level, seed=0, w_fit=0.1, w_reg=0.9):
    """Laplacian smoothing of a noisy icosphere (float3 per vertex)."""
    rng = np.random.default_rng(seed)
    v, _, edges = icosphere(level)
    A = v.T + 0.05 * rng.normal(size=(3, len(v)))
    return dict(energy="laplacian_graph", V=len(v), edges=edges.astype(np.int32), A=A,
                x0=np.zeros((3, len(v))), params=dict(w_fit=w_fit, w_reg=w_reg))


def grid_edges(W, H):
    """Edges of a W x H pixel grid to the right and down neighbours, site id j*W+i:
    first all horizontal edges in row-major order, then all vertical ones."""
    s = np.arange(W * H).reshape(H, W)
    h = np.stack([s[:, :-1].ravel(), s[:, 1:].ravel()], 1)
    v = np.stack([s[:-1, :].ravel(), s[1:, :].ravel()], 1)
    return np.concatenate([h, v]).astype(np.int32)
