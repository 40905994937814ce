"""FP64 CPU oracle for the fast Birkhoff products and the Birkhoff-preconditioned solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or calls anything in this package; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark do.

Every function here is the plain, slow definition of what the GPU path computes:

* ``birkhoff``  -- the CGL grid, the dense Birkhoff matrix B^a built two independent
  ways, the Clenshaw-Curtis weights, the lower-triangular approximation B~^a, and the
  closed-form Chebyshev antiderivatives used to check products at any N.
* ``system``    -- the dense linear system [I - B^a df] dX = x^a b, the dense Birkhoff
  preconditioner P = I - B~^a df, its forward substitution, dense LU solves, and a
  plain right-preconditioned GMRES used only to compare iteration counts.
* ``newton``    -- the two-body right-hand side and its Jacobian, the residual
  X - x^a b - B^a f(X) of the nonlinear IVP, and Newton's method on it with dense
  linear solves and Armijo backtracking.
* ``kkt``       -- the symmetric saddle-point (KKT) form of the collocated system, the
  backward substitution P^{-T}, the block-diagonal SPD preconditioner, and a plain
  preconditioned MINRES.

It shares no code with the HIP path.  Arithmetic is float64 throughout; library
primitives (LAPACK solves, matrix products, scipy's DCT, Gauss-Legendre nodes) serve
as single steps only.
"""

from . import birkhoff, kkt, newton, system  # noqa: F401
