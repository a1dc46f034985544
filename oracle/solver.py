"""Gauss-Newton and Levenberg-Marquardt with a Jacobi-PCG inner solve (Sec. 4, 4.1).

Readings of the paper taken here (each is also listed in the design notes):

* The normal equations 2 J^T J d = -2 J^T F (Sec. 4) are solved without the
  factor 2: PCG iterates do not change when A and b are scaled together.  The
  cost is E = sum of squared residuals, with no 1/2.
* PCG is the standard preconditioned conjugate gradient started from d = 0
  (Sec. 4.1; the figure with its kernels is not reproduced in the text).  It runs
  a fixed number of iterations; it stops early only if p.q is not positive
  (breakdown, or the residual reached exactly zero).
* Jacobi preconditioner: M = diag(J^T J) (Sec. 4.2, evalJTF); an unknown with a
  zero diagonal gets M^-1 = 0, so it does not move.  Without the preconditioner
  M^-1 = 1 on every unknown that is not excluded.
* LM (Sec. 4): (J^T J + lambda D) d = -J^T F with D = diag(J^T J) clamped to
  [diag_min, diag_max] and lambda = 1/radius.  The step is taken iff the model
  decrease m > 0 and the gain ratio rho = (E(x) - E(x+d))/m exceeds min_rel_decrease;
  then radius /= max(1/3, 1 - (2 rho - 1)^3) (capped at radius_max) and nu = 2;
  otherwise radius /= nu, nu *= 2, and the solve ends once radius < radius_min.
  This is the Nielsen trust-region rule that the paper's Ceres-derived strategy
  follows; the defaults are Ceres' documented defaults.  The damped system uses
  the Jacobi preconditioner 1/(d + lambda D).  Rejected steps count as iterations.
"""
from dataclasses import dataclass, field

import numpy as np

from .assemble import jacobian


def cost(energy, x):
    """E(x) = sum_r f_r(x)^2 in FP64."""
    F = np.real(energy.residuals(np.asarray(x, float).ravel()))
    return float(F @ F)


class Linearization:
    """F, J and the derived quantities of one outer iteration at x."""

    def __init__(self, energy, x):
        self.energy = energy
        self.x = np.asarray(x, float).ravel().copy()
        self.F = np.real(energy.residuals(self.x))
        self.J = jacobian(energy, self.x)
        self.JT = self.J.T.tocsr()
        self.E = float(self.F @ self.F)
        self.diag = np.asarray(self.J.multiply(self.J).sum(0)).ravel()
        self.active = np.tile(energy.active, energy.n_chan)

    def jtf(self):
        """b = -J^T F."""
        return -(self.JT @ self.F)

    def damping(self, diag_min=1e-6, diag_max=1e32):
        """D = clamp(diag(J^T J), diag_min, diag_max) on active unknowns, 0 elsewhere."""
        return np.where(self.active, np.clip(self.diag, diag_min, diag_max), 0.0)

    def apply(self, p, lam=0.0, D=None):
        """(J^T J + lam D) p."""
        q = self.JT @ (self.J @ p)
        if lam != 0.0:
            q = q + lam * D * p
        return q

    def minv(self, use_precond=True, lam=0.0, D=None):
        if not use_precond:
            return np.where(self.active, 1.0, 0.0)
        d = self.diag + (lam * D if lam != 0.0 else 0.0)
        out = np.zeros_like(d)
        ok = self.active & (d > 0)
        out[ok] = 1.0 / d[ok]
        return out


@dataclass
class PCGInfo:
    iterations: int = 0
    stopped: bool = False
    rz: list = field(default_factory=list)


def pcg(apply_A, b, minv, L):
    """Preconditioned CG for A d = b from d = 0, at most L iterations."""
    d = np.zeros_like(b)
    r = b.copy()
    z = minv * r
    p = z.copy()
    rz = float(r @ z)
    info = PCGInfo(rz=[rz])
    for _ in range(L):
        q = apply_A(p)
        pq = float(p @ q)
        if not pq > 0:
            info.stopped = True
            break
        alpha = rz / pq
        d += alpha * p
        r -= alpha * q
        z = minv * r
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
        info.iterations += 1
        info.rz.append(rz)
    return d, info


def gauss_newton(energy, x0, outer, inner, use_precond=True, callback=None):
    """Returns (x, costs) with costs[k] = E(x_k), k = 0..outer.  If ``callback``
    is given it is called after every outer iteration as callback(k, x), k the
    iterations done and x the new iterate (to follow a long solve; it must not
    modify x)."""
    x = np.asarray(x0, float).ravel().copy()
    costs = []
    for k in range(outer):
        lin = Linearization(energy, x)
        costs.append(lin.E)
        delta, _ = pcg(lin.apply, lin.jtf(), lin.minv(use_precond), inner)
        x = x + delta
        if callback is not None:
            callback(k + 1, x)
    costs.append(cost(energy, x))
    return x, costs


def irls(energy, x0, outer, inner, use_precond=True, callback=None):
    """Iteratively reweighted least squares (Sec. 7, variants of GN/LM): each
    outer iteration fixes the energy's weights at the current x
    (energy.freeze), then takes one Gauss-Newton step, inner PCG iterations, on
    the fixed-weight least-squares problem.  Returns (x, objectives) with
    objectives[k] = energy.objective(x_k), k = 0..outer.  ``callback`` as for
    gauss_newton."""
    x = np.asarray(x0, float).ravel().copy()
    objs = []
    for _ in range(outer):
        energy.freeze(x)
        objs.append(energy.objective(x))
        lin = Linearization(energy, x)
        delta, _ = pcg(lin.apply, lin.jtf(), lin.minv(use_precond), inner)
        x = x + delta
        if callback is not None:
            callback(len(objs), x)
    objs.append(energy.objective(x))
    return x, objs


@dataclass
class LMParams:
    radius0: float = 1e4
    radius_min: float = 1e-32
    radius_max: float = 1e16
    diag_min: float = 1e-6
    diag_max: float = 1e32
    min_rel_decrease: float = 1e-3


def levenberg_marquardt(energy, x0, outer, inner, prm=LMParams(), use_precond=True, history=None,
                        callback=None):
    """Returns (x, costs, accepted): costs[k] = E at the start of iteration k, plus
    the final cost; accepted[k] tells whether iteration k took its step.  If
    ``history`` is a list, one dict per iteration is appended to it: the radius
    the iteration used, its gain ratio rho and model decrease m, whether it
    accepted, and the radius and nu it left.  ``callback``, if given, is called
    after every iteration as callback(k, x) (k iterations done, x the current
    iterate; it must not modify x)."""
    x = np.asarray(x0, float).ravel().copy()
    radius, nu = prm.radius0, 2.0
    costs, accepted = [], []
    lin = None
    for _ in range(outer):
        if radius < prm.radius_min:
            break
        if lin is None:
            lin = Linearization(energy, x)
        costs.append(lin.E)
        lam = 1.0 / radius
        D = lin.damping(prm.diag_min, prm.diag_max)
        delta, _ = pcg(lambda p: lin.apply(p, lam, D), lin.jtf(),
                       lin.minv(use_precond, lam, D), inner)
        Jd = lin.J @ delta
        m = -float(Jd @ (2.0 * lin.F + Jd))
        E1 = cost(energy, x + delta)
        rho = (lin.E - E1) / m if m != 0 else -np.inf
        if m > 0 and rho > prm.min_rel_decrease:
            x = x + delta
            radius = min(radius / max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3), prm.radius_max)
            nu = 2.0
            lin = None
            accepted.append(True)
        else:
            radius = radius / nu
            nu = 2.0 * nu
            accepted.append(False)
        if history is not None:
            history.append(dict(radius_used=1.0 / lam, lam=lam, rho=rho, m=m, accepted=accepted[-1],
                                radius=radius, nu=nu))
        if callback is not None:
            callback(len(accepted), x)
    costs.append(cost(energy, x))
    return x, costs, accepted
