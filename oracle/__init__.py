"""Plain, slow, FP64 CPU oracle for the LDG multigrid solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never calls it and
shares no code with it.

Every function follows a passage of the paper (Saye, "A comparative study of
efficient multigrid solvers for high-order local discontinuous Galerkin
methods", arXiv:2412.12506) and cites the section, equation, algorithm or table.
Where the paper defers to earlier work that is not available (penalty
constants, pressure-penalty form), the reading taken is stated in the function
that uses it; those constants are "parity unpinned" in absolute terms.

Modules:
  basis      1-D basis, quadrature, reference and transfer matrices
  ldg        scalar LDG operator A = sum_k G_k^T M_mu G_k + E and its RHS
  stokes     Stokes saddle-point LDG operator (eq:components)
  hierarchy  factor coarsening and the level list
  smoothers  block Jacobi, multi-coloured Gauss-Seidel, balanced block SAI
  vcycle     Algorithm 1 (V-cycle) and the bottom pseudo-inverse
  krylov     preconditioned CG, left-preconditioned GMRES, eta estimate
  solver     convenience: build everything for a workload
"""
