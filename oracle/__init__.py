"""CPU oracle for the bake-off problems BP1-BP6 (TEST INFRASTRUCTURE ONLY).

A plain, slow, FP64 NumPy/SciPy statement of what the GPU path computes,
written from the paper (Fischer et al., "Scalability of high-performance PDE
solvers", sections 3-5 and Appendix A1), and used only by the tests, by the
smoke check and by the benchmark's CPU-baseline leg. The product path never
imports, calls or links anything here, and nothing here imports the product.

Contents:
  quadrature  GLL / GL rules, Lagrange interpolation and derivative matrices
  geometry    isoparametric derivatives, geometric factors G and B~ (eq. (gij), (mass))
  operators   sum-factorised mass / stiffness application with gather, scatter
              and Dirichlet mask (eq. (bk5x), (tens1), (mass), Q^T A_L Q)
  assembled   brute-force element matrices via Kronecker products, assembled
              in scipy.sparse (tiny meshes only)
  pcg         Jacobi-preconditioned CG (section 3), fixed-iteration and
              tolerance modes, independent scalars per component
  mixed       single-precision inner PCG inside FP64 defect correction
  adjoint     variable-coefficient Poisson, loss, adjoint solve and dL/dkappa

Pins (tests/test_oracle_*.py) tie every function to something other than
itself: quadrature exactness and library rules, closed-form geometric
factors, the 7-point Laplacian at p=1, Kronecker consistent mass at p=1,
volume, null space, energy identity, patch test, brute-force assembly, a
direct sparse solve, spectral convergence, and finite differences.
"""
