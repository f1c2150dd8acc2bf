"""Plain CPU float64 oracle for the ParaDiag-II all-at-once solve.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product
library never calls it, and it shares no code with the GPU path (it imports
numpy and scipy only).

What it computes, all in float64, each function citing the passage it follows:

* ``operators``  spatial matrices (eq2.2b, eq3.1), Toeplitz time matrices
  (eq2.5b, eq3.2b), their alpha-circulant versions (eq2.11b, eq3.4) and the
  time symbols of Lemma 1.
* ``rhs``        the all-at-once right-hand side and its transpose.
* ``solve``      the solution of A u = b three ways: sequential time stepping,
  a sparse all-at-once solve and a dense Kronecker solve (eq1.1).
* ``precond``    P_alpha^{-1} r two ways: sparse solve with the assembled
  alpha-circulant matrix (eq1.2) and the three FFT steps (eq1.3 / eq2.12).
* ``krylov``     flexible GMRES and the stationary iteration (eq5.1).
* ``adjoint``    the transposed solve and the gradient of a tracking cost.
* ``hybrid``     ParaDiag-I with the hybrid midpoint / backward Euler time
  discretisation (Section 2.1.2): its time matrices, the closed-form
  eigendecomposition and exact all-at-once solves.
* ``parareal``   classical parareal and the ParaDiag-II parareal variant with
  the alpha-periodic coarse-grid correction (Section 2.2.2).
* ``nonlinear``  nonlinear ParaDiag with the averaged Jacobian (eq1.4, eq1.5)
  and windowing.
* ``ocwave``     the optimality system of the optimal control of the wave
  equation and its block-circulant preconditioner (Section 4, Thm the4).

Parity status of every function is stated in its module docstring.
"""

from .problem import Problem  # noqa: F401
from . import operators, rhs, solve, precond, krylov, adjoint, hybrid, parareal, nonlinear, ocwave  # noqa: F401
