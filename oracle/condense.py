"""Condensing solve: an independent route to the same solution, used only as a pin.

The states are eliminated through the dynamics (eq. ocp-eq with E_j = I),
x = Gamma U + e with U = (u_0, ..., u_{N-1}) and e the free response from x_init
and f; the objective becomes a dense quadratic in U whose minimiser solves the
normal equations.  The multipliers then follow from the state rows of the
optimality conditions (eq. opt-cond-ocp-eq), swept backward from
lam_{N-1} = Q_N x_N + q_N.
"""
from __future__ import annotations

import numpy as np

from .kkt import sym


def solve(prob):
    N, nx, nu = prob.N, prob.nx, prob.nu
    S = np.zeros((N, nu, nx)) if prob.S is None else prob.S
    f = np.zeros((N, nx)) if prob.f is None else prob.f
    # x_k = Phi_k x0 + sum_j Gam[k][j] u_j + c_k, k = 1..N  (row block k-1)
    Gam = np.zeros((N * nx, N * nu))
    e = np.zeros(N * nx)
    Phi = np.eye(nx)
    c = np.zeros(nx)
    prev_rows = None
    for k in range(1, N + 1):
        A, B = prob.A[k - 1], prob.B[k - 1]
        rows = slice((k - 1) * nx, k * nx)
        if prev_rows is not None:
            Gam[rows, :] = A @ Gam[prev_rows, :]
        Gam[rows, (k - 1) * nu:k * nu] = B
        Phi = A @ Phi
        c = A @ c + f[k - 1]
        e[rows] = Phi @ prob.x0 + c
        prev_rows = rows
    Qx = np.zeros((N * nx, N * nx))
    Ru = np.zeros((N * nu, N * nu))
    Sux = np.zeros((N * nu, N * nx))
    qv = np.zeros(N * nx)
    rv = np.zeros(N * nu)
    for k in range(N):
        Ru[k * nu:(k + 1) * nu, k * nu:(k + 1) * nu] = sym(prob.R[k])
        rv[k * nu:(k + 1) * nu] = prob.r[k]
        if k >= 1:
            Sux[k * nu:(k + 1) * nu, (k - 1) * nx:k * nx] = S[k]
    rv[0:nu] += S[0] @ prob.x0
    for k in range(1, N + 1):
        Qx[(k - 1) * nx:k * nx, (k - 1) * nx:k * nx] = sym(prob.Q[k])
        qv[(k - 1) * nx:k * nx] = prob.q[k]
    Hc = Ru + Sux @ Gam + Gam.T @ Sux.T + Gam.T @ Qx @ Gam
    g = rv + Sux @ e + Gam.T @ (Qx @ e + qv)
    U = np.linalg.solve(sym(Hc), -g)
    X = Gam @ U + e
    x = X.reshape(N, nx)
    u = U.reshape(N, nu)
    lam = np.zeros((N, nx))
    lam[N - 1] = sym(prob.Q[N]) @ x[N - 1] + prob.q[N]
    for k in range(N - 1, 0, -1):
        # S_k^T u_k + Q_k x_k + A_k^T lam_k - lam_{k-1} = -q_k
        lam[k - 1] = S[k].T @ u[k] + sym(prob.Q[k]) @ x[k - 1] + prob.A[k].T @ lam[k] + prob.q[k]
    return x, u, lam
