"""Plain FP64 CPU oracle for ADMM-BB robust proton planning (TEST INFRASTRUCTURE).

This package is the slow, obviously-correct reference that the GPU library is
judged against.  It is test infrastructure only: the tests, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
(the C-ABI library and its Python binding) never does, and this package never
imports the product.  The two share no code; both read the same seeded inputs
from the `synth` module.

Contents, each following the paper's own statement:

  wls      the objective f(x) = sum_s sum_i c_s w_i (a_{s,i}^T x - p_i)^2
           (Sec. 2.1, eq. for f_s and the robust problem), its gradient
           (Sec. 2.1, eq. for grad f_s), the closed quadratic form
           (1/2 x^T H x - g0^T x + const), the KKT residual of the box-constrained
           problem, and FP64 sparse products used as SpMV references.
  exact    exact minimisers: brute-force enumeration of active sets (n <= 12)
           and a projected-Newton active-set polish for any n.
  admm     ADMM-BB exactly as Sec. 2.2 and Appendix A state it: per-scenario
           x-update through a cached Cholesky factor of B_s, z-update, dual update
           with the Barzilai-Borwein step, and the residual stopping test.
  pgd      projected gradient descent with Armijo backtracking (Sec. 2.1).
  mlp      FP64 reference of the small warm-start network (forward, backward,
           Adam), used to check the GPU training kernels.

Everything is float64.  Parity status of each function is stated in its
docstring: "pinned" functions are checked by the CPU test suite against facts
that do not come from this package (closed forms, brute force, library
solvers, finite differences, invariances).
"""
