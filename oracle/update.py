"""Low-rank modification of the stage Hessians by changes of constraint penalties, and the factors
of the modified problem.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. "Factorization updates": the stage Hessian of the augmented-Lagrangian Newton system is the
cost Hessian plus [D_j^T; C_j^T] Sigma_j [D_j C_j] over the active constraint rows
(eq. qpalm-ocp-hessians), so a change Delta Sigma_j of the (diagonal) penalty factors changes it by
the symmetric term of eq. low-rank-update-Hj:

    R_j <- R_j + D_j^T dSigma_j D_j,   S_j <- S_j + D_j^T dSigma_j C_j,   Q_j <- Q_j + C_j^T dSigma_j C_j

(S_j is the u-x block in the order (u_j, x_j) of eq. ocp-eq).  Rows with a zero change contribute
nothing; negative changes (constraints leaving the active set) are downdates.  The terminal stage
has only state rows (C_N); stage 0's rows reach S_0, which multiplies the fixed initial state.

* ``modified_problem``: the problem with R_j, S_j, Q_j so modified -- the plain definition of
  what an update of the stored factors represents.
* ``updated_factors``: the Cholesky factors of the modified problem's recursion
  (``riccati.reference_factors``).  Factors with positive diagonals are unique, so these are what
  any factorisation update (Alg. "fact-mod-riccati-update", hyperbolic Householder
  transformations) must reproduce.

Array shapes for one instance with m rows per stage: C [N+1, m, nx] (stages 0..N),
D [N, m, nu] (stages 0..N-1), dsig [N+1, m].
float64 numpy throughout.
"""
from __future__ import annotations

import copy

import numpy as np

from . import riccati


def modified_problem(prob, C, D, dsig):
    """The instance with its stage Hessians changed by the penalty changes (eq. low-rank-update-Hj)."""
    N, nx, nu = prob.N, prob.nx, prob.nu
    C = np.asarray(C, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    dsig = np.asarray(dsig, dtype=np.float64)
    assert C.shape[0] == N + 1 and C.shape[2] == nx
    assert D.shape[0] == N and D.shape[2] == nu
    assert dsig.shape == (N + 1, C.shape[1]) and D.shape[1] == C.shape[1]
    out = copy.copy(prob)
    out.R = np.array(prob.R, dtype=np.float64, copy=True)
    out.Q = np.array(prob.Q, dtype=np.float64, copy=True)
    out.S = np.zeros((N, nu, nx)) if prob.S is None else np.array(prob.S, dtype=np.float64, copy=True)
    for j in range(N + 1):
        W = np.diag(dsig[j])
        out.Q[j] = out.Q[j] + C[j].T @ W @ C[j]
        if j < N:
            out.R[j] = out.R[j] + D[j].T @ W @ D[j]
            out.S[j] = out.S[j] + D[j].T @ W @ C[j]
    return out


def updated_factors(prob, C, D, dsig):
    """(LQ, LR, LS) of the modified problem, as ``riccati.reference_factors`` returns them."""
    return riccati.reference_factors(modified_problem(prob, C, D, dsig))
