"""Residual definitions of the energies, FP64, written from the energies the paper defines.

Conventions (Sec. 3 and the energy definitions of Appendix C):

* A grid site is (i, j): i runs along the width W (first dimension), j along the
  height H.  Arrays are [c, H, W]; the unknown vector is the planes flattened,
  index ch*W*H + j*W + i.
* The Energy function squares its arguments, so weights are square roots of the
  energy weights (Fig. 3 caption).
* A term with an out-of-bounds access, or whose Select condition is false,
  contributes a zero residual (Sec. 3, "Boundaries").  Such residuals stay as rows
  of F and J that are identically zero.
* Exclude(...) marks sites whose unknowns are constants: they keep their
  residuals but their Jacobian columns are dropped (``active`` is False there).

Every ``residuals`` accepts complex input and evaluates every Select condition on
the real part, so comparisons carry no derivative; ``assemble`` relies on that.

``row_sites()`` lists, for every residual row, the sites whose unknowns it can
read (-1 for none).  ``site_colors()`` gives a colouring of the sites such that
no row reads two sites of one colour.
"""
import numpy as np

OFFSETS4 = ((1, 0), (-1, 0), (0, 1), (0, -1))


def _shift(A, di, dj):
    """Return (B, inb) with B[..., j, i] = A[..., j+dj, i+di] where (i+di, j+dj)
    lies on the grid and 0 elsewhere; inb marks where it does."""
    H, W = A.shape[-2:]
    B = np.zeros_like(A)
    inb = np.zeros((H, W), bool)
    j0, j1 = max(0, -dj), min(H, H - dj)
    i0, i1 = max(0, -di), min(W, W - di)
    if j1 > j0 and i1 > i0:
        B[..., j0:j1, i0:i1] = A[..., j0 + dj:j1 + dj, i0 + di:i1 + di]
        inb[j0:j1, i0:i1] = True
    return B, inb


def _grid_sites(W, H, offsets):
    """[H*W, len(offsets)] site ids anchor+offset, -1 where off the grid."""
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    cols = []
    for di, dj in offsets:
        ii, jj = i + di, j + dj
        ok = (ii >= 0) & (ii < W) & (jj >= 0) & (jj < H)
        cols.append(np.where(ok, jj * W + ii, -1).ravel())
    return np.stack(cols, 1)


def _pad_cols(a, k):
    if a.shape[1] == k:
        return a
    return np.concatenate([a, -np.ones((a.shape[0], k - a.shape[1]), a.dtype)], 1)


class _Grid:
    K = 2  # colouring period; must exceed the span of every residual footprint

    def site_colors(self):
        j, i = np.meshgrid(np.arange(self.H), np.arange(self.W), indexing="ij")
        return ((i % self.K) + self.K * (j % self.K)).ravel(), self.K * self.K

    @property
    def n_sites(self):
        return self.W * self.H

    def _x(self, x):
        return np.asarray(x).reshape(self.n_chan, self.H, self.W)


class _Graph:
    def site_colors(self):
        """Greedy colouring in vertex order of the graph whose edges join every
        pair of sites read by one residual row."""
        rs = self.row_sites()
        pairs = []
        for a in range(rs.shape[1]):
            for b in range(rs.shape[1]):
                if a != b:
                    ok = (rs[:, a] >= 0) & (rs[:, b] >= 0)
                    pairs.append(np.stack([rs[ok, a], rs[ok, b]], 1))
        p = np.unique(np.concatenate(pairs), axis=0) if pairs else np.zeros((0, 2), np.int64)
        n = self.n_sites
        ptr = np.zeros(n + 1, np.int64)
        np.add.at(ptr, p[:, 0] + 1, 1)
        ptr = np.cumsum(ptr)
        nbr = p[np.argsort(p[:, 0], kind="stable"), 1]
        color = -np.ones(n, np.int64)
        for v in range(n):
            used = set(color[nbr[ptr[v]:ptr[v + 1]]].tolist())
            c = 0
            while c in used:
                c += 1
            color[v] = c
        return color, int(color.max()) + 1


class ArapWarp(_Grid):
    """ARAP image warping (Fig. 24; A.1.1).  Unknowns per pixel: Offset (2), Angle.

    Per pixel p and stencil offset s in {(1,0),(-1,0),(0,1),(0,-1)}, q = p+s:
      r_reg = w_reg * [(O_p - O_q) - R(a_p)(U_p - U_q)]          (2 rows)
      valid iff q is on the grid, Mask(q) = 0 and Mask(p) = 0
    Fit: r_fit = w_fit * (O_p - C_p), valid iff both components of C_p >= 0.
    R(a) is the counter-clockwise rotation [[cos,-sin],[sin,cos]].
    Exclude: pixels with Mask != 0.
    Row order: for each s, x rows then y rows; then fit x, fit y.
    """
    n_chan = 3

    def __init__(self, W, H, U, C, mask, w_fit, w_reg):
        self.W, self.H = W, H
        self.U = np.asarray(U, float)
        self.C = np.asarray(C, float)
        self.mask = np.asarray(mask)
        self.w_fit, self.w_reg = float(w_fit), float(w_reg)
        self.active = (self.mask == 0).ravel()

    def residuals(self, x):
        x = self._x(x)
        O, th = x[:2], x[2]
        U, C, wr, wf = self.U, self.C, self.w_reg, self.w_fit
        act = self.mask == 0
        cs, sn = np.cos(th), np.sin(th)
        out = []
        for di, dj in OFFSETS4:
            Oq, inb = _shift(O, di, dj)
            Uq, _ = _shift(U, di, dj)
            aq, _ = _shift(act, di, dj)
            valid = inb & aq & act
            dx, dy = U[0] - Uq[0], U[1] - Uq[1]
            rx = wr * ((O[0] - Oq[0]) - (cs * dx - sn * dy))
            ry = wr * ((O[1] - Oq[1]) - (sn * dx + cs * dy))
            out += [np.where(valid, rx, 0), np.where(valid, ry, 0)]
        fv = (C[0] >= 0) & (C[1] >= 0)
        out += [np.where(fv, wf * (O[0] - C[0]), 0), np.where(fv, wf * (O[1] - C[1]), 0)]
        return np.concatenate([o.ravel() for o in out])

    def row_sites(self):
        blocks = []
        for s in OFFSETS4:
            g = _grid_sites(self.W, self.H, [(0, 0), s])
            blocks += [g, g]
        f = _pad_cols(_grid_sites(self.W, self.H, [(0, 0)]), 2)
        blocks += [f, f]
        return np.concatenate(blocks)


class Poisson(_Grid):
    """Poisson image editing (Fig. 27; A.1.4).  Unknown: RGBA (4) per pixel.

    Per pixel p, offset s, q = p+s on the grid:  r = (X_p - X_q) - (T_p - T_q)
    per channel, no weights.  Exclude: pixels with M != 0.
    Row order: for each s, channels 0..3.
    """
    n_chan = 4

    def __init__(self, W, H, T, mask):
        self.W, self.H = W, H
        self.T = np.asarray(T, float)
        self.mask = np.asarray(mask)
        self.active = (self.mask == 0).ravel()

    def residuals(self, x):
        X = self._x(x)
        out = []
        for di, dj in OFFSETS4:
            Xq, inb = _shift(X, di, dj)
            Tq, _ = _shift(self.T, di, dj)
            e = (X - Xq) - (self.T - Tq)
            out += [np.where(inb, e[c], 0) for c in range(4)]
        return np.concatenate([o.ravel() for o in out])

    def row_sites(self):
        blocks = []
        for s in OFFSETS4:
            g = _grid_sites(self.W, self.H, [(0, 0), s])
            blocks += [g] * 4
        return np.concatenate(blocks)


def bilinear_clamped(img, x, y):
    """Sample img at real coordinates (x = along W, y = along H): texel centres at
    integer coordinates, bilinear weights, each of the four texel indices clamped
    to the image (clamp-to-edge addressing)."""
    H, W = img.shape
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx = x - x0
    fy = y - y0
    ix0 = np.clip(x0.astype(np.int64), 0, W - 1)
    ix1 = np.clip(x0.astype(np.int64) + 1, 0, W - 1)
    iy0 = np.clip(y0.astype(np.int64), 0, H - 1)
    iy1 = np.clip(y0.astype(np.int64) + 1, 0, H - 1)
    return ((1 - fx) * (1 - fy) * img[iy0, ix0] + fx * (1 - fy) * img[iy0, ix1]
            + (1 - fx) * fy * img[iy1, ix0] + fx * fy * img[iy1, ix1])


class OpticalFlow(_Grid):
    """Dense optical flow (Fig. 30; A.2.3).  Unknown: flow (u, v) per pixel.

    r_fit = w_fit * (I(i,j) - S(I_hat; i+u, j+v))                   (1 row)
    r_reg = w_reg * (X_p - X_q) per channel, q = p+s on the grid    (2 rows per s)
    S is the sampled-image operator (Sec. 7): its value is a bilinear,
    clamp-to-edge sample of I_hat; its partial derivatives with respect to the
    sample coordinates are, by definition, the same samples of the supplied
    derivative images I_hat_dx, I_hat_dy.  With complex input the imaginary part
    carries exactly those partials.
    Row order: fit; then for each s, u rows then v rows.
    """
    n_chan = 2

    def __init__(self, W, H, I, Ihat, Ihat_dx, Ihat_dy, w_fit, w_reg):
        self.W, self.H = W, H
        self.I = np.asarray(I, float)
        self.Ih = np.asarray(Ihat, float)
        self.Idx = np.asarray(Ihat_dx, float)
        self.Idy = np.asarray(Ihat_dy, float)
        self.w_fit, self.w_reg = float(w_fit), float(w_reg)
        self.active = np.ones(W * H, bool)

    def sample(self, u, v):
        j, i = np.meshgrid(np.arange(self.H, dtype=float), np.arange(self.W, dtype=float), indexing="ij")
        xr, yr = i + np.real(u), j + np.real(v)
        val = bilinear_clamped(self.Ih, xr, yr)
        if np.iscomplexobj(u) or np.iscomplexobj(v):
            val = val + 1j * (np.imag(u) * bilinear_clamped(self.Idx, xr, yr)
                              + np.imag(v) * bilinear_clamped(self.Idy, xr, yr))
        return val

    def residuals(self, x):
        X = self._x(x)
        out = [self.w_fit * (self.I - self.sample(X[0], X[1]))]
        for di, dj in OFFSETS4:
            Xq, inb = _shift(X, di, dj)
            out += [np.where(inb, self.w_reg * (X[c] - Xq[c]), 0) for c in range(2)]
        return np.concatenate([o.ravel() for o in out])

    def row_sites(self):
        blocks = [_pad_cols(_grid_sites(self.W, self.H, [(0, 0)]), 2)]
        for s in OFFSETS4:
            g = _grid_sites(self.W, self.H, [(0, 0), s])
            blocks += [g, g]
        return np.concatenate(blocks)


class ShapeFromShading(_Grid):
    """Shape from shading (Fig. 26; A.1.3).  Unknown: depth X per pixel.

    Params (Fig. 26): w_p, w_s, w_g enter through their square roots; f_x, f_y,
    u_x, u_y are the camera intrinsics; L1..L9 the lighting coefficients.
      position p(a,b) = (((a-u_x)/f_x) X, ((b-u_y)/f_y) X, X)        (eq. 8)
      normal at (a,b) (eq. 10):
        n_x = X(a,b-1)(X(a,b)-X(a-1,b))/f_y
        n_y = X(a-1,b)(X(a,b)-X(a,b-1))/f_x
        n_z = n_x(u_x-a)/f_x + n_y(u_y-b)/f_y - X(a-1,b)X(a,b-1)/(f_x f_y)
        divided by its length when the squared length is > 0
      B = L1 + L2 n_y + L3 n_z + L4 n_x + L5 n_x n_y + L6 n_y n_z
          + L7 (-n_x^2 - n_y^2 + 2 n_z^2) + L8 n_z n_x + L9 (n_x^2 - n_y^2)
      I(a,b) = Im(a,b)/2 + (Im(a-1,b) + Im(a,b-1))/4
      B_I(a,b) = B - I if IBE(a,b) and D_i > 0 at (a-1,b), (a,b), (a,b-1), else 0
    with IBE(a,b) = "InBoundsExpanded(0,0,1)": 1 <= a <= W-2 and 1 <= b <= H-2.
    Residuals at (i,j) (row order):
      r_p  = sqrt(w_p) (X - D_i)                          if D_i(i,j) > 0
      r_gh = sqrt(w_g) eR(i,j) (B_I(i,j) - B_I(i+1,j))    if IBE(i,j)
      r_gv = sqrt(w_g) eC(i,j) (B_I(i,j) - B_I(i,j+1))    if IBE(i,j)
      r_s  = sqrt(w_s) (4p(i,j) - p(i-1,j) - p(i,j-1) - p(i+1,j) - p(i,j+1))  (3 rows)
             if D_i > 0 on the 5-point stencil, |X(i,j) - X(nbr)| < 0.01 for the four
             neighbours, and IBE(i,j).
    Exclude: pixels with D_i <= 0.
    """
    n_chan = 1
    K = 3
    THRESH = 0.01

    def __init__(self, W, H, D, Im, edge_r, edge_c, w_p, w_s, w_g, f_x, f_y, u_x, u_y, L):
        self.W, self.H = W, H
        self.D = np.asarray(D, float)
        self.Im = np.asarray(Im, float)
        self.eR = np.asarray(edge_r).astype(float)
        self.eC = np.asarray(edge_c).astype(float)
        self.sw_p, self.sw_s, self.sw_g = np.sqrt(w_p), np.sqrt(w_s), np.sqrt(w_g)
        self.fx, self.fy, self.ux, self.uy = float(f_x), float(f_y), float(u_x), float(u_y)
        self.L = tuple(float(v) for v in L)
        self.DV = self.D > 0
        self.active = self.DV.ravel()
        j, i = np.meshgrid(np.arange(H, dtype=float), np.arange(W, dtype=float), indexing="ij")
        self.ii, self.jj = i, j
        self.IBE = (i >= 1) & (i <= W - 2) & (j >= 1) & (j <= H - 2)

    def B_I(self, X):
        fx, fy, ux, uy = self.fx, self.fy, self.ux, self.uy
        Xl, _ = _shift(X, -1, 0)
        Xu, _ = _shift(X, 0, -1)
        nx = Xu * (X - Xl) / fy
        ny = Xl * (X - Xu) / fx
        nz = nx * (ux - self.ii) / fx + ny * (uy - self.jj) / fy - Xl * Xu / (fx * fy)
        sq = nx * nx + ny * ny + nz * nz
        pos = np.real(sq) > 0
        inv = np.where(pos, 1.0 / np.sqrt(np.where(pos, sq, 1.0)), 1.0)
        nx, ny, nz = nx * inv, ny * inv, nz * inv
        L1, L2, L3, L4, L5, L6, L7, L8, L9 = self.L
        B = (L1 + L2 * ny + L3 * nz + L4 * nx + L5 * nx * ny + L6 * ny * nz
             + L7 * (-nx * nx - ny * ny + 2 * nz * nz) + L8 * nz * nx + L9 * (nx * nx - ny * ny))
        Iml, _ = _shift(self.Im, -1, 0)
        Imu, _ = _shift(self.Im, 0, -1)
        Iv = 0.5 * self.Im + 0.25 * (Iml + Imu)
        dvl, _ = _shift(self.DV, -1, 0)
        dvu, _ = _shift(self.DV, 0, -1)
        valid = self.IBE & dvl & self.DV & dvu
        return np.where(valid, B - Iv, 0)

    def smooth_valid(self, X):
        Xr = np.real(X)
        ok = self.IBE & self.DV
        for di, dj in OFFSETS4:
            Xq, _ = _shift(Xr, di, dj)
            dq, _ = _shift(self.DV, di, dj)
            ok = ok & dq & (np.abs(Xr - Xq) < self.THRESH)
        return ok

    def residuals(self, x):
        X = self._x(x)[0]
        fx, fy, ux, uy = self.fx, self.fy, self.ux, self.uy
        rp = np.where(self.DV, self.sw_p * (X - self.D), 0)
        BI = self.B_I(X)
        BIr, _ = _shift(BI, 1, 0)
        BIc, _ = _shift(BI, 0, 1)
        rgh = np.where(self.IBE, self.sw_g * self.eR * (BI - BIr), 0)
        rgv = np.where(self.IBE, self.sw_g * self.eC * (BI - BIc), 0)
        kx = (self.ii - ux) / fx
        ky = (self.jj - uy) / fy
        P = np.stack([kx * X, ky * X, X])
        S = 4 * P
        for di, dj in OFFSETS4:
            Pq, _ = _shift(P, di, dj)
            S = S - Pq
        vs = self.smooth_valid(X)
        rs = [np.where(vs, self.sw_s * S[c], 0) for c in range(3)]
        return np.concatenate([o.ravel() for o in [rp, rgh, rgv] + rs])

    def row_sites(self):
        W, H = self.W, self.H
        fp = _pad_cols(_grid_sites(W, H, [(0, 0)]), 5)
        gh = _grid_sites(W, H, [(0, 0), (-1, 0), (0, -1), (1, 0), (1, -1)])
        gv = _grid_sites(W, H, [(0, 0), (-1, 0), (0, -1), (0, 1), (-1, 1)])
        sm = _grid_sites(W, H, [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)])
        return np.concatenate([fp, gh, gv, sm, sm, sm])


def euler_rotate(a, d):
    """R(a) d with R(a) = Rz(a_z) Ry(a_y) Rx(a_x) (right-handed, counter-clockwise
    about each axis).  a, d: [3, ...] arrays."""
    cx, sx = np.cos(a[0]), np.sin(a[0])
    cy, sy = np.cos(a[1]), np.sin(a[1])
    cz, sz = np.cos(a[2]), np.sin(a[2])
    x1, y1, z1 = d[0], cx * d[1] - sx * d[2], sx * d[1] + cx * d[2]
    x2, y2, z2 = cy * x1 + sy * z1, y1, -sy * x1 + cy * z1
    return np.stack([cz * x2 - sz * y2, sz * x2 + cz * y2, z2])


class ArapMesh(_Graph):
    """ARAP mesh deformation (Fig. 25; A.1.2).  Unknowns per vertex: Offset (3),
    Euler angles (3).

    Fit: r = w_fit (O_v - C_v), each component valid iff C_v >= -999999.9 there.
    For every listed undirected edge {v0, v1} both orientations are residuals
    (3 rows each):  r(v0->v1) = w_reg [(O_v0 - O_v1) - R(a_v0)(U_v0 - U_v1)].
    Row order: fit x,y,z (V rows each); then orientation v0->v1 components x,y,z
    (E rows each); then orientation v1->v0.
    """
    n_chan = 6

    def __init__(self, V, edges, U, C, w_fit, w_reg):
        self.V = V
        self.e = np.asarray(edges, np.int64)
        self.U = np.asarray(U, float)
        self.C = np.asarray(C, float)
        self.w_fit, self.w_reg = float(w_fit), float(w_reg)
        self.active = np.ones(V, bool)

    @property
    def n_sites(self):
        return self.V

    def residuals(self, x):
        x = np.asarray(x).reshape(6, self.V)
        O, A = x[:3], x[3:]
        fv = self.C >= -999999.9
        out = [np.where(fv[c], self.w_fit * (O[c] - self.C[c]), 0) for c in range(3)]
        for a, b in ((self.e[:, 0], self.e[:, 1]), (self.e[:, 1], self.e[:, 0])):
            Rd = euler_rotate(A[:, a], self.U[:, a] - self.U[:, b])
            r = self.w_reg * ((O[:, a] - O[:, b]) - Rd)
            out += [r[c] for c in range(3)]
        return np.concatenate([np.ravel(o) for o in out])

    def row_sites(self):
        v = np.arange(self.V)
        f = np.stack([v, -np.ones_like(v)], 1)
        fwd = self.e
        bwd = self.e[:, ::-1]
        return np.concatenate([f, f, f, fwd, fwd, fwd, bwd, bwd, bwd])


OFFSETS6 = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def _shift3(A, di, dj, dk):
    """B[..., k, j, i] = A[..., k+dk, j+dj, i+di] where that voxel exists, else 0;
    and the mask of where it does."""
    D, H, W = A.shape[-3:]
    B = np.zeros_like(A)
    inb = np.zeros((D, H, W), bool)
    k0, k1 = max(0, -dk), min(D, D - dk)
    j0, j1 = max(0, -dj), min(H, H - dj)
    i0, i1 = max(0, -di), min(W, W - di)
    if k1 > k0 and j1 > j0 and i1 > i0:
        B[..., k0:k1, j0:j1, i0:i1] = A[..., k0 + dk:k1 + dk, j0 + dj:j1 + dj, i0 + di:i1 + di]
        inb[k0:k1, j0:j1, i0:i1] = True
    return B, inb


class ArapVolume:
    """ARAP volumetric deformation on a 3D grid (Fig. 31; A.2.5).  Unknowns per
    voxel: Offset (3), Euler angles (3); voxel (i, j, k) has index (k*H + j)*W + i.

    Fit: r = w_fit (O_v - C_v), each component valid iff C_v >= -999999.9 there.
    For each voxel v and each neighbour u = v + s, s in +-x, +-y, +-z, that lies
    on the grid: r(v->u) = w_reg [(O_v - O_u) - R(a_v)(U_v - U_u)] (3 rows).
    Row order: fit x,y,z (n rows each); then per offset s (in OFFSETS6 order) the
    x, y, z rows (n each, zero where u is off the grid).
    """
    n_chan = 6

    def __init__(self, W, H, D, U, C, w_fit, w_reg):
        self.W, self.H, self.D = W, H, D
        self.U = np.asarray(U, float).reshape(3, D, H, W)
        self.C = np.asarray(C, float).reshape(3, D, H, W)
        self.w_fit, self.w_reg = float(w_fit), float(w_reg)
        self.active = np.ones(W * H * D, bool)

    @property
    def n_sites(self):
        return self.W * self.H * self.D

    def site_colors(self):
        k, j, i = np.meshgrid(np.arange(self.D), np.arange(self.H), np.arange(self.W), indexing="ij")
        return ((i % 2) + 2 * (j % 2) + 4 * (k % 2)).ravel(), 8

    def residuals(self, x):
        x = np.asarray(x).reshape(6, self.D, self.H, self.W)
        O, A = x[:3], x[3:]
        fv = self.C >= -999999.9
        out = [np.where(fv[c], self.w_fit * (O[c] - self.C[c]), 0) for c in range(3)]
        for di, dj, dk in OFFSETS6:
            Oq, inb = _shift3(O, di, dj, dk)
            Uq, _ = _shift3(self.U, di, dj, dk)
            Rd = euler_rotate(A, self.U - Uq)
            r = self.w_reg * ((O - Oq) - Rd)
            out += [np.where(inb, r[c], 0) for c in range(3)]
        return np.concatenate([np.ravel(o) for o in out])

    def row_sites(self):
        W, H, D = self.W, self.H, self.D
        k, j, i = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
        v = ((k * H + j) * W + i).ravel()
        f = np.stack([v, -np.ones_like(v)], 1)
        blocks = [f, f, f]
        for di, dj, dk in OFFSETS6:
            ii, jj, kk = i + di, j + dj, k + dk
            ok = ((ii >= 0) & (ii < W) & (jj >= 0) & (jj < H) & (kk >= 0) & (kk < D)).ravel()
            u = np.where(ok, ((kk * H + jj) * W + ii).ravel(), -1)
            g = np.stack([v, u], 1)
            blocks += [g, g, g]
        return np.concatenate(blocks)


class LaplacianGrid(_Grid):
    """Laplacian smoothing on an image (Fig. 3): r_fit = w_fit (X - A),
    r_h = w_reg (X(i,j) - X(i+1,j)), r_v = w_reg (X(i,j) - X(i,j+1)), the last two
    only where the neighbour is on the grid.  Row order: fit, h, v."""
    n_chan = 1

    def __init__(self, W, H, A, w_fit, w_reg):
        self.W, self.H = W, H
        self.A = np.asarray(A, float).reshape(H, W)
        self.w_fit, self.w_reg = float(w_fit), float(w_reg)
        self.active = np.ones(W * H, bool)

    def residuals(self, x):
        X = self._x(x)[0]
        Xr, inr = _shift(X, 1, 0)
        Xd, ind = _shift(X, 0, 1)
        return np.concatenate([(self.w_fit * (X - self.A)).ravel(),
                               np.where(inr, self.w_reg * (X - Xr), 0).ravel(),
                               np.where(ind, self.w_reg * (X - Xd), 0).ravel()])

    def row_sites(self):
        W, H = self.W, self.H
        return np.concatenate([_pad_cols(_grid_sites(W, H, [(0, 0)]), 2),
                               _grid_sites(W, H, [(0, 0), (1, 0)]),
                               _grid_sites(W, H, [(0, 0), (0, 1)])])


class LpSmoothGrid(_Grid):
    """Edge-preserving image smoothing with an l_p regulariser, solved by IRLS
    (Sec. 7, variants of GN/LM): data term r_fit = w_fit (X - A) (squared, l_2),
    edge terms f_h = w_reg (X(i,j) - X(i+1,j)) and f_v = w_reg (X(i,j) - X(i,j+1))
    where the neighbour is on the grid, each entering the objective as
    (f^2 + eps^2)^(p/2):

        Phi(x) = sum r_fit^2 + sum_edges (f^2 + eps^2)^(p/2).

    IRLS freezes a weight per edge at the current x (``freeze``) and takes a
    least-squares step on sum r_fit^2 + sum w f^2; ``residuals`` are those of
    the frozen problem: r_fit, then sqrt(w_h) f_h and sqrt(w_v) f_v.  The weight
    is w = (p/2) (f^2 + eps^2)^((p-2)/2): the paper's f^(p-2) for a sum of l_p
    terms alone, with eps keeping it finite at f = 0 and the factor p/2 making
    an IRLS fixed point a stationary point of Phi when an l_2 term is present
    (its gradient matches Phi's there).  Row order: fit, h, v."""
    n_chan = 1

    def __init__(self, W, H, A, w_fit, w_reg, p, eps):
        self.W, self.H = W, H
        self.A = np.asarray(A, float).reshape(H, W)
        self.w_fit, self.w_reg = float(w_fit), float(w_reg)
        self.p, self.eps = float(p), float(eps)
        self.active = np.ones(W * H, bool)
        self.wh = np.ones((H, W))
        self.wv = np.ones((H, W))

    def edge_terms(self, x):
        """(f_h, in-grid mask, f_v, in-grid mask) at x."""
        X = np.asarray(x).reshape(self.H, self.W)
        Xr, inr = _shift(X, 1, 0)
        Xd, ind = _shift(X, 0, 1)
        return (np.where(inr, self.w_reg * (X - Xr), 0), inr, np.where(ind, self.w_reg * (X - Xd), 0), ind)

    def weight(self, f):
        return 0.5 * self.p * (f * f + self.eps ** 2) ** (0.5 * (self.p - 2.0))

    def freeze(self, x):
        """Fix the IRLS weights at x (real)."""
        fh, _, fv, _ = self.edge_terms(np.asarray(x, float))
        self.wh, self.wv = self.weight(fh), self.weight(fv)

    def objective(self, x):
        """Phi(x), FP64."""
        X = np.asarray(x, float).reshape(self.H, self.W)
        fh, inr, fv, ind = self.edge_terms(X)
        smooth = lambda f, m: np.where(m, (f * f + self.eps ** 2) ** (0.5 * self.p), 0.0).sum()
        return float((self.w_fit * (X - self.A)) .ravel() @ (self.w_fit * (X - self.A)).ravel()
                     + smooth(fh, inr) + smooth(fv, ind))

    def residuals(self, x):
        X = self._x(x)[0]
        fh, _, fv, _ = self.edge_terms(X)
        return np.concatenate([(self.w_fit * (X - self.A)).ravel(), (np.sqrt(self.wh) * fh).ravel(),
                               (np.sqrt(self.wv) * fv).ravel()])

    def row_sites(self):
        W, H = self.W, self.H
        return np.concatenate([_pad_cols(_grid_sites(W, H, [(0, 0)]), 2),
                               _grid_sites(W, H, [(0, 0), (1, 0)]),
                               _grid_sites(W, H, [(0, 0), (0, 1)])])


class IntrinsicImage(_Grid):
    """Intrinsic image decomposition (A.2.4, Fig. 33), solved by IRLS (Sec. 7):
    per pixel a reflectance r (3 channels) and a shading s, channel order
    (r0, r1, r2, s).  For each pixel and each of its four stencil neighbours q
    on the grid (+x, -x, +y, -y), a reflectance term f = w_a (r - r_q) (a
    3-vector) entering as (|f|^2 + eps^2)^(p/2) and a shading term w_s (s - s_q)
    (squared); a fit w_fit (r_c + s - I_c) per channel (squared):

        Phi(x) = sum fit^2 + sum_(pixel, q) [(|f|^2 + eps^2)^(p/2) + (w_s (s - s_q))^2].

    Each edge appears once from each end.  IRLS freezes, per edge, the weight
    w = (p/2) (|f|^2 + eps^2)^((p-2)/2) at the current x (both ends share it)
    and takes a least-squares step on the frozen problem; ``residuals`` are
    those of the frozen problem: the fits, then per direction the three
    components of sqrt(w) f, then per direction the shading term.  The weight
    reads as for LpSmoothGrid (eps, and the factor p/2 beside the l_2 fit).
    Row order: fit (3 channels), reflectance (4 directions x 3 components),
    shading (4 directions)."""
    n_chan = 4
    DIRS = ((1, 0), (-1, 0), (0, 1), (0, -1))

    def __init__(self, W, H, I, w_fit, w_a, w_s, p, eps):
        self.W, self.H = W, H
        self.I = np.asarray(I, float).reshape(3, H, W)
        self.w_fit, self.w_a, self.w_s = float(w_fit), float(w_a), float(w_s)
        self.p, self.eps = float(p), float(eps)
        self.active = np.ones(W * H, bool)
        self.wh = np.ones((H, W))  # weight of the edge to the right of a pixel (0 past the grid)
        self.wv = np.ones((H, W))  # of the edge below

    def weight(self, f2):
        """w for |f|^2 = f2."""
        return 0.5 * self.p * (f2 + self.eps ** 2) ** (0.5 * (self.p - 2.0))

    def dir_weights(self):
        """The frozen weight of each direction's edge at every pixel (0 off the grid)."""
        wl, _ = _shift(self.wh, -1, 0)
        wu, _ = _shift(self.wv, 0, -1)
        return (self.wh, wl, self.wv, wu)

    def freeze(self, x):
        X = np.asarray(x, float).reshape(4, self.H, self.W)
        R = X[:3]
        for k, (di, dj) in ((0, (1, 0)), (2, (0, 1))):
            Rq, inb = _shift(R, di, dj)
            f2 = (self.w_a ** 2) * ((R - Rq) ** 2).sum(0)
            w = np.where(inb, self.weight(f2), 0.0)
            if k == 0:
                self.wh = w
            else:
                self.wv = w

    def objective(self, x):
        X = np.asarray(x, float).reshape(4, self.H, self.W)
        R, S = X[:3], X[3]
        fit = self.w_fit * (R + S[None] - self.I)
        e = float((fit * fit).sum())
        for di, dj in self.DIRS:
            Rq, inb = _shift(R, di, dj)
            Sq, _ = _shift(S, di, dj)
            f2 = (self.w_a ** 2) * ((R - Rq) ** 2).sum(0)
            e += float(np.where(inb, (f2 + self.eps ** 2) ** (0.5 * self.p), 0.0).sum())
            e += float(np.where(inb, (self.w_s * (S - Sq)) ** 2, 0.0).sum())
        return e

    def residuals(self, x):
        X = self._x(x)
        R, S = X[:3], X[3]
        out = [(self.w_fit * (R[c] + S - self.I[c])).ravel() for c in range(3)]
        for (di, dj), w in zip(self.DIRS, self.dir_weights()):
            Rq, inb = _shift(R, di, dj)
            for c in range(3):
                out.append(np.where(inb, np.sqrt(w) * self.w_a * (R[c] - Rq[c]), 0).ravel())
        for di, dj in self.DIRS:
            Sq, inb = _shift(S, di, dj)
            out.append(np.where(inb, self.w_s * (S - Sq), 0).ravel())
        return np.concatenate(out)

    def row_sites(self):
        W, H = self.W, self.H
        fit = _pad_cols(_grid_sites(W, H, [(0, 0)]), 2)
        rows = [fit] * 3
        for di, dj in self.DIRS:
            rows += [_grid_sites(W, H, [(0, 0), (di, dj)])] * 3
        for di, dj in self.DIRS:
            rows.append(_grid_sites(W, H, [(0, 0), (di, dj)]))
        return np.concatenate(rows)


class LaplacianGraph(_Graph):
    """Laplacian smoothing on a graph (Fig. 5), float3 per vertex:
    r_fit = w_fit (X_v - A_v); r_e = w_reg (X_v0 - X_v1) for each listed edge.
    Row order: fit x,y,z; edge x,y,z."""
    n_chan = 3

    def __init__(self, V, edges, A, w_fit, w_reg):
        self.V = V
        self.e = np.asarray(edges, np.int64)
        self.A = np.asarray(A, float)
        self.w_fit, self.w_reg = float(w_fit), float(w_reg)
        self.active = np.ones(V, bool)

    @property
    def n_sites(self):
        return self.V

    def residuals(self, x):
        X = np.asarray(x).reshape(3, self.V)
        out = [self.w_fit * (X[c] - self.A[c]) for c in range(3)]
        out += [self.w_reg * (X[c, self.e[:, 0]] - X[c, self.e[:, 1]]) for c in range(3)]
        return np.concatenate(out)

    def row_sites(self):
        v = np.arange(self.V)
        f = np.stack([v, -np.ones_like(v)], 1)
        return np.concatenate([f, f, f, self.e, self.e, self.e])


def make_energy(w):
    """Build the oracle energy for a workload dict from the ``workloads`` package."""
    kind = w["energy"]
    p = w["params"]
    if kind == "arap_warp":
        return ArapWarp(w["W"], w["H"], w["U"], w["C"], w["mask"], p["w_fit"], p["w_reg"])
    if kind == "poisson":
        return Poisson(w["W"], w["H"], w["T"], w["mask"])
    if kind == "flow":
        return OpticalFlow(w["W"], w["H"], w["I"], w["Ihat"], w["Ihat_dx"], w["Ihat_dy"],
                           p["w_fit"], p["w_reg"])
    if kind == "sfs":
        return ShapeFromShading(w["W"], w["H"], w["D"], w["Im"], w["edge_r"], w["edge_c"],
                                p["w_p"], p["w_s"], p["w_g"], p["f_x"], p["f_y"], p["u_x"],
                                p["u_y"], p["L"])
    if kind == "arap_mesh":
        return ArapMesh(w["V"], w["edges"], w["U"], w["C"], p["w_fit"], p["w_reg"])
    if kind == "arap_volume":
        return ArapVolume(w["W"], w["H"], w["D"], w["U"], w["C"], p["w_fit"], p["w_reg"])
    if kind == "laplacian":
        return LaplacianGrid(w["W"], w["H"], w["A"], p["w_fit"], p["w_reg"])
    if kind == "laplacian_graph":
        return LaplacianGraph(w["V"], w["edges"], w["A"], p["w_fit"], p["w_reg"])
    if kind == "lp_smooth":
        return LpSmoothGrid(w["W"], w["H"], w["A"], p["w_fit"], p["w_reg"], p["p"], p["eps"])
    if kind == "intrinsic":
        return IntrinsicImage(w["W"], w["H"], w["I"], p["w_fit"], p["w_a"], p["w_s"], p["p"], p["eps"])
    raise ValueError(kind)
