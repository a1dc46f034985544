"""Explicit sparse Jacobian of an oracle energy.

J[r, ch*n + s] = d F_r / d x[ch, s], taken by complex-step forward
differentiation: F(x + i*h*e) = F(x) + i*h*(J e) + O(h^2), so Im F / h is J e to
rounding for h = 1e-20 (no subtractive cancellation, unlike finite differences).
All sites of one colour are perturbed together; the colouring guarantees a row
reads at most one of them, so each entry of J e belongs to exactly one column.
A row that reads none of the perturbed sites must come out with an imaginary
part of exactly zero; anything else means ``row_sites`` is incomplete and raises.

Columns of excluded sites (``active`` False) are dropped, as Exclude makes those
unknowns constants.
"""
import numpy as np
import scipy.sparse as sp

H_STEP = 1e-20


def jacobian(energy, x, h=H_STEP):
    """J(x) as scipy CSR, shape (rows of F, n_chan * n_sites)."""
    x = np.asarray(x, float).ravel()
    n, nc = energy.n_sites, energy.n_chan
    rs = energy.row_sites()
    color, ncolors = energy.site_colors()
    rc = np.where(rs >= 0, color[np.maximum(rs, 0)], -1)
    R = rs.shape[0]
    rows, cols, vals = [], [], []
    for c in range(ncolors):
        match = rc == c
        cnt = match.sum(1)
        if np.any(cnt > 1):
            raise AssertionError("colouring: a residual reads two sites of one colour")
        has = cnt == 1
        hrows = np.nonzero(has)[0]
        hsite = rs[hrows, np.argmax(match[hrows], 1)]
        sites = np.nonzero(color == c)[0]
        keep_site = energy.active[hsite]
        for ch in range(nc):
            xc = x.astype(complex)
            xc[ch * n + sites] += 1j * h
            d = np.imag(energy.residuals(xc)) / h
            if d.shape[0] != R:
                raise AssertionError("row_sites and residuals disagree on the row count")
            if np.any(d[~has] != 0):
                raise AssertionError("a residual reads a site missing from row_sites")
            v = d[hrows]
            nz = (v != 0) & keep_site
            rows.append(hrows[nz])
            cols.append(ch * n + hsite[nz])
            vals.append(v[nz])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(R, nc * n))


def jacobian_dense_bruteforce(energy, x, h=H_STEP):
    """Dense J by perturbing one unknown at a time (complex step); no colouring
    and no use of ``row_sites``.  Small problems only."""
    x = np.asarray(x, float).ravel()
    N = x.size
    cols = []
    act = np.tile(energy.active, energy.n_chan)
    for k in range(N):
        xc = x.astype(complex)
        xc[k] += 1j * h
        col = np.imag(energy.residuals(xc)) / h
        cols.append(col if act[k] else np.zeros_like(col))
    return np.stack(cols, 1)


def fd_jacobian(energy, x, rel=1e-6):
    """Dense J by central finite differences in real arithmetic, step
    rel*max(1, |x_k|).  Small problems only; accurate to about 1e-8 relative."""
    x = np.asarray(x, float).ravel()
    act = np.tile(energy.active, energy.n_chan)
    cols = []
    for k in range(x.size):
        hk = rel * max(1.0, abs(x[k]))
        xp = x.copy()
        xm = x.copy()
        xp[k] += hk
        xm[k] -= hk
        col = (np.real(energy.residuals(xp)) - np.real(energy.residuals(xm))) / (2 * hk)
        cols.append(col if act[k] else np.zeros_like(col))
    return np.stack(cols, 1)
