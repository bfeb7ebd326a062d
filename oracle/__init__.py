"""FP64 CPU oracle for FD-preconditioned flexible GMRES on spline collocation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
link anything in this package; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP path
(no kernels, headers, helpers or table generators).  Inputs it needs (right-hand
sides, seeds) are passed in by the caller.

Paper: M. Tani, "A preconditioning strategy for linear systems arising from
nonsymmetric schemes in isogeometric analysis" (arXiv 1705.04384).

Modules (each function cites the passage it follows):

* ``bspline``  -- open uniform knot vectors, Greville abscissae (Sec. 2.1-2.2,
  eq. 2.4), B-spline values and first/second derivatives by the Cox-de Boor
  recursion.
* ``colloc``   -- univariate collocation factors M, K (eq. 2.8), the
  unit-domain Kronecker operator (eq. 2.7 / 2.9), manufactured right-hand
  sides, and the collocation operator on a smoothly deformed cube (Sec. 2.2,
  whose general form the paper does not write out; derived here by the chain
  rule).
* ``fd``       -- generalized eigendecomposition of the pencils (eq. 4.6),
  V = (M U)^{-T}, and the fast-diagonalization solve (eq. 4.7 / 4.9).
* ``galerkin`` -- Gauss-quadrature Galerkin factors M, K (eq. 3.8) and the
  convection factor H (after eq. 3.9), symmetric FD factors (V = U), and the
  Galerkin convection-diffusion matrix on the deformed cube (Sec. 3.2).
* ``bicgstab`` -- right-preconditioned BiCGStab (the Krylov method of the
  experiments, Sec. 5) with the k + 0.5 half-step count.
* ``fgmres``   -- flexible GMRES(m) with classical Gram-Schmidt and one
  reorthogonalisation, Givens least squares, true-residual restarts (the paper
  names GMRES as the Krylov method for the nonsymmetric system, Sec. 3).

Parity status: every function here is pinned by a test in
``tests/test_oracle_*.py`` against something other than itself (library
routines, closed forms, brute-force dense solves, convergence orders);
none is "parity unpinned".
"""
