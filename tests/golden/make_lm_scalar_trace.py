"""Write lm_scalar_trace.json: a Levenberg-Marquardt trace of one scalar
residual, derived by hand in closed form (no solver code is used).

Problem: one unknown x, one residual f(x) = x^2 - c with c = -1 (no root: the
minimum E = 1 is at x = 0), from x0 = 2.  Gauss-Newton steps on it jump around
0, so the trace holds accepted steps of gain ratio well inside (0, 1), where the
radius update is not clamped, and rejected ones.

Each iteration, with J = f'(x) = 2x and F = f(x) (Sec. 4, lambda = 1/radius and
D the diagonal of J^T J clamped to [1e-6, 1e32]):
  A = J^2 + lambda * clamp(J^2);  the damped normal equation A d = -J F has one
  unknown, so one Jacobi-preconditioned CG iteration solves it exactly: d = -J F / A;
  E0 = F^2;  E1 = f(x + d)^2;  m = -(J d)(2F + J d)   (model decrease);
  rho = (E0 - E1) / m.
Step control (the Nielsen trust-region rule, Madsen, Nielsen and Tingleff 2004,
with Ceres' documented defaults: radius0 = 1e4, bounds [1e-32, 1e16],
acceptance threshold 1e-3):
  accept iff m > 0 and rho > 1e-3:  x += d; radius /= max(1/3, 1 - (2 rho - 1)^3),
    capped at 1e16; nu = 2;
  else: radius /= nu; nu *= 2.

    python tests/golden/make_lm_scalar_trace.py
"""
import json
import os

C, X0, RADIUS0, ITERS = -1.0, 2.0, 1e4, 16


def trace():
    x, radius, nu = X0, RADIUS0, 2.0
    rows = []
    for _ in range(ITERS):
        J, F = 2.0 * x, x * x - C
        lam = 1.0 / radius
        A = J * J + lam * min(max(J * J, 1e-6), 1e32)
        d = -J * F / A
        E0, E1 = F * F, ((x + d) ** 2 - C) ** 2
        Jd = J * d
        m = -Jd * (2.0 * F + Jd)
        rho = (E0 - E1) / m
        row = dict(x=x, radius_used=radius, rho=rho, m=m, E0=E0)
        if m > 0 and rho > 1e-3:
            x = x + d
            radius = min(radius / max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3), 1e16)
            nu = 2.0
            row["accepted"] = True
        else:
            radius, nu = radius / nu, 2.0 * nu
            row["accepted"] = False
        row["radius"] = radius
        rows.append(row)
    return rows, x


if __name__ == "__main__":
    rows, x = trace()
    out = {"source": "Levenberg-Marquardt of Sec. 4 with the trust-region rule read as the Nielsen update "
                     "(Madsen, Nielsen and Tingleff 2004) and Ceres' documented defaults; derivation in "
                     "make_lm_scalar_trace.py",
           "problem": "one unknown x, residual f(x) = x^2 + 1, x0 = 2, radius0 = 1e4, 16 iterations",
           "c": C, "x0": X0, "radius0": RADIUS0, "iters": ITERS, "steps": rows, "x_final": x}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lm_scalar_trace.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    for r in rows:
        print(f"x={r['x']:.6f} radius={r['radius_used']:.4g} rho={r['rho']:.4f} acc={r['accepted']}")
