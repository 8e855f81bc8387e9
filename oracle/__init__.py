"""CPU FP64 oracle for the equality-constrained LQ optimal-control KKT system.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the
product path never does, and this package imports nothing from it.

Contents (each function cites the passage of the paper it follows):

* ``kkt``      -- explicit assembly of the KKT matrix and right-hand side of the
                  optimality conditions (eq. opt-cond-ocp-eq), dense and banded
                  direct solves, and the KKT residual.
* ``riccati``  -- the textbook (non-factorised) Riccati recursion for the
                  cost-to-go P_k (eq. riccati-recursion-P) with its vector
                  recursion and forward rollout; reference factors derived from P_k.
* ``condense`` -- an independent condensing solve (states eliminated through
                  the dynamics), used only to pin the other routes.
* ``adjoint``  -- gradients of a loss of the solution through the KKT system,
                  and central finite differences.
* ``closed``   -- closed forms (scalar discrete algebraic Riccati equation).
* ``blocktri`` -- symmetric positive definite block-tridiagonal systems: dense definition, the
                  cyclic-reduction factor as the Cholesky factor of the valuation-ordered
                  matrix, the written-out CR and PCR recursions, preconditioned CG.
* ``update``   -- the stage Hessians changed by constraint-penalty changes (low-rank terms) and
                  the factors of the modified problem.
* ``qp``       -- box-constrained LQ QPs: the optimality certificate, the augmented-Lagrangian merit
                  function and its exact line search (sorted breakpoints), the proximal ALM with
                  semismooth Newton inner solves.

All arithmetic is float64 with numpy / scipy (LAPACK).  Nothing here is blocked,
fused or reordered beyond the definitions.
"""
from . import adjoint, blocktri, closed, condense, kkt, qp, riccati, update  # noqa: F401
