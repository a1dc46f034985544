"""FP64 CPU oracle for the matrix-free Gauss-Newton / Levenberg-Marquardt PCG path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library may import, call or link this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP path.

What it computes (Opt, arXiv 1604.06525):

* residual vectors F(x) of each energy, written from the energies defined in
  Appendix C (Figs. 24-27, 30, 31; Laplacian of Figs. 3 and 5), in plain vectorised
  numpy, FP64 (``energies``);
* an explicit sparse Jacobian J(x) (scipy CSR).  Entries come from complex-step
  forward differentiation of F, exact to rounding, with columns grouped by a
  colouring so that each residual row sees at most one perturbed site
  (``assemble``).  The paper derives J symbolically (Sec. 5.2); any exact
  derivative gives the same J;
* the solver of Sec. 4: Gauss-Newton on the normal equations J^T J d = -J^T F
  (the common factor 2 cancels), a Jacobi-preconditioned conjugate gradient inner
  solve started from d = 0 (Sec. 4.1), and Levenberg-Marquardt with the damping
  lambda*diag(J^T J) of Sec. 4 and a trust-region radius update (``solver``).

Everything is double precision.  It is a correctness reference, not a tuned CPU
solver.
"""
from .energies import (ArapWarp, Poisson, ShapeFromShading, OpticalFlow, ArapMesh, ArapVolume,
                       LaplacianGrid, LaplacianGraph, LpSmoothGrid, IntrinsicImage, make_energy)
from .assemble import jacobian, jacobian_dense_bruteforce, fd_jacobian
from .solver import (Linearization, pcg, gauss_newton, levenberg_marquardt, irls, cost,
                     LMParams)

__all__ = ["ArapWarp", "Poisson", "ShapeFromShading", "OpticalFlow", "ArapMesh", "ArapVolume",
           "LaplacianGrid", "LaplacianGraph", "LpSmoothGrid", "IntrinsicImage", "make_energy", "jacobian",
           "jacobian_dense_bruteforce", "fd_jacobian", "Linearization", "pcg",
           "gauss_newton", "levenberg_marquardt", "irls", "cost", "LMParams"]
