"""Textbook Riccati recursion (backward dynamic programming), FP64.

Cost-to-go recursion of Sec. "Riccati recursion" (eq. riccati-recursion-P):

    P_N = Q_N
    P_k = Q_k + A_k^T P_{k+1} A_k
          - (S_k^T + A_k^T P_{k+1} B_k) (R_k + B_k^T P_{k+1} B_k)^{-1} (S_k + B_k^T P_{k+1} A_k)

written out with explicit (asymmetric) products and a linear solve; this is the
non-factorised form the paper contrasts with the factorised one.  The affine
terms follow from the same dynamic-programming step with value function
V_k(x) = 1/2 x^T P_k x + p_k^T x + const:

    w_k   = P_{k+1} f_k + p_{k+1}
    K_k   = -(R_k + B_k^T P_{k+1} B_k)^{-1} (S_k + B_k^T P_{k+1} A_k)
    d_k   = -(R_k + B_k^T P_{k+1} B_k)^{-1} (r_k + B_k^T w_k)
    p_k   = q_k + A_k^T w_k + (S_k^T + A_k^T P_{k+1} B_k) d_k,    p_N = q_N

and the forward rollout x_0 = x_init, u_k = K_k x_k + d_k,
x_{k+1} = A_k x_k + B_k u_k + f_k, with the multipliers of the dynamics
lam_k = P_{k+1} x_{k+1} + p_{k+1} (the gradient of V_{k+1} at x_{k+1}, which is
what the x_{k+1} rows of eq. opt-cond-ocp-eq give).

P_0 is formed with Q_0 and is only a diagnostic: x_0 is fixed.
"""
from __future__ import annotations

import numpy as np

from .kkt import sym


def _S(prob, k):
    return np.zeros((prob.nu, prob.nx)) if prob.S is None else prob.S[k]


def _f(prob, k):
    return np.zeros(prob.nx) if prob.f is None else prob.f[k]


def recursion(prob):
    """Backward pass.  Returns dict with P [N+1], K [N], d [N], p [N+1], Rhat [N], Shat [N]."""
    N = prob.N
    P = [None] * (N + 1)
    p = [None] * (N + 1)
    Kg = [None] * N
    d = [None] * N
    Rh = [None] * N
    Sh = [None] * N
    P[N] = sym(prob.Q[N])
    p[N] = prob.q[N].copy()
    for k in range(N - 1, -1, -1):
        A, B = prob.A[k], prob.B[k]
        Pn = P[k + 1]
        Rhat = sym(prob.R[k]) + B.T @ Pn @ B
        Shat = _S(prob, k) + B.T @ Pn @ A
        Kg[k] = -np.linalg.solve(Rhat, Shat)
        P[k] = sym(prob.Q[k]) + A.T @ Pn @ A - (_S(prob, k).T + A.T @ Pn @ B) @ np.linalg.solve(Rhat, Shat)
        w = Pn @ _f(prob, k) + p[k + 1]
        d[k] = -np.linalg.solve(Rhat, prob.r[k] + B.T @ w)
        p[k] = prob.q[k] + A.T @ w + (_S(prob, k).T + A.T @ Pn @ B) @ d[k]
        Rh[k], Sh[k] = Rhat, Shat
    return {"P": P, "K": Kg, "d": d, "p": p, "Rhat": Rh, "Shat": Sh}


def solve(prob, rec=None):
    """Textbook Riccati solve: returns (x [N, nx] for k = 1..N, u [N, nu], lam [N, nx])."""
    rec = recursion(prob) if rec is None else rec
    N = prob.N
    x = np.zeros((N, prob.nx))
    u = np.zeros((N, prob.nu))
    lam = np.zeros((N, prob.nx))
    xk = prob.x0.copy()
    for k in range(N):
        u[k] = rec["K"][k] @ xk + rec["d"][k]
        xn = prob.A[k] @ xk + prob.B[k] @ u[k] + _f(prob, k)
        lam[k] = rec["P"][k + 1] @ xn + rec["p"][k + 1]
        x[k] = xn
        xk = xn
    return x, u, lam


def reference_factors(prob, rec=None):
    """Cholesky factors implied by the textbook quantities.

    LQ[k] = chol(P_k) for k = 1..N (index 0 unused), LR[k] = chol(R_k + B_k^T P_{k+1} B_k),
    LS[k] = (S_k + B_k^T P_{k+1} A_k)^T LR[k]^{-T} for k = 0..N-1.  Cholesky factors
    with positive diagonals are unique, so these are what any factorised
    recursion must produce.
    """
    rec = recursion(prob) if rec is None else rec
    N = prob.N
    LQ = [None] + [np.linalg.cholesky(sym(rec["P"][k])) for k in range(1, N + 1)]
    LR = [np.linalg.cholesky(sym(rec["Rhat"][k])) for k in range(N)]
    LS = [np.linalg.solve(LR[k], rec["Shat"][k]).T for k in range(N)]
    return LQ, LR, LS
