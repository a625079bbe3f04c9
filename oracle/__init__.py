"""FP64 CPU oracle for the Calderon-preconditioned PMCHWT path.

TEST INFRASTRUCTURE ONLY.  Plain, slow, direct implementations of what the
GPU library computes, written from the paper (Kleanthous et al., "Accelerated
Calderon preconditioning for Maxwell transmission problems") and from the
published mathematics it relies on (RWG and Buffa-Christiansen functions,
symmetric triangle rules, Sauter-Schwab singular quadrature).  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the GPU library: it has its own topology, dual-basis
construction, quadrature tables and linear algebra.

Modules
  quadrature  triangle rules, Gauss-Legendre, Sauter-Schwab transformations
  mesh        edge topology, RWG orientation, barycentric refinement, BC functions
  operators   Galerkin matrices of S and C (direct quadrature sums), mass matrices
  pmchwt      PMCHWT blocks, preconditioners, right-hand side, solves,
              far field and cross sections, the matvec cost model
"""
