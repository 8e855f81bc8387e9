"""Gradients of a loss of the KKT solution, and central finite differences.

The solution z of K(theta) z = b(theta) (eq. opt-cond-ocp-eq) has, for a loss
l(z), dl/dtheta = zbar^T (db/dtheta - dK/dtheta z) with K zbar = grad_z l
(K is symmetric).  Writing zbar = (ubar, xbar, lambar) with xbar_0 = 0 and
x_0 = x_init, the entries of K and b give, stage by stage:

    dl/dA_k = -(lambar_k x_k^T + lam_k xbar_k^T)
    dl/dB_k = -(lambar_k u_k^T + lam_k ubar_k^T)
    dl/dS_k = -(ubar_k x_k^T + u_k xbar_k^T)
    dl/dQ_k = -1/2 (xbar_k x_k^T + x_k xbar_k^T)   (Q enters through its symmetric part)
    dl/dR_k = -1/2 (ubar_k u_k^T + u_k ubar_k^T)
    dl/dq_k = -xbar_k,  dl/dr_k = -ubar_k,  dl/df_k = -lambar_k
    dl/dx_init = -(A_0^T lambar_0 + S_0^T ubar_0)
    dl/dQ_0 = 0, dl/dq_0 = 0.
"""
from __future__ import annotations

import copy

import numpy as np

from . import kkt


def adjoint_grad(prob, gx, gu):
    """Gradients for upstream gradients gx = dl/dx_k (k = 1..N) and gu = dl/du_k (k = 0..N-1)."""
    K, b, L = kkt.assemble(prob)
    Kd = K.toarray()
    z = np.linalg.solve(Kd, b)
    x, u, lam = kkt.split(z, L)
    g = kkt.join(np.asarray(gx, np.float64), np.asarray(gu, np.float64), np.zeros_like(lam), L)
    zb = np.linalg.solve(Kd, g)
    xb, ub, lb = kkt.split(zb, L)
    return grads_from(prob, x, u, lam, xb, ub, lb), (x, u, lam), (xb, ub, lb)


def adjoint_grad_banded(prob, gx, gu):
    """``adjoint_grad`` with both solves (z and zbar) in banded storage, for horizons where the
    dense K does not fit or is too slow; the same equations."""
    K, b, L = kkt.assemble(prob)
    z = kkt.banded_solve(K, b, L)
    x, u, lam = kkt.split(z, L)
    g = kkt.join(np.asarray(gx, np.float64), np.asarray(gu, np.float64), np.zeros_like(lam), L)
    zb = kkt.banded_solve(K, g, L)
    xb, ub, lb = kkt.split(zb, L)
    return grads_from(prob, x, u, lam, xb, ub, lb), (x, u, lam), (xb, ub, lb)


def grads_from(prob, x, u, lam, xb, ub, lb):
    N, nx, nu = prob.N, prob.nx, prob.nu
    xs = np.vstack([prob.x0[None, :], x])           # x_0 .. x_N
    xbs = np.vstack([np.zeros((1, nx)), xb])        # xbar_0 = 0
    out = {k: np.zeros_like(getattr(prob, k)) for k in ("A", "B", "Q", "R", "q", "r", "x0")}
    out["S"] = np.zeros((N, nu, nx))
    out["f"] = np.zeros((N, nx))
    for k in range(N):
        out["A"][k] = -(np.outer(lb[k], xs[k]) + np.outer(lam[k], xbs[k]))
        out["B"][k] = -(np.outer(lb[k], u[k]) + np.outer(lam[k], ub[k]))
        out["S"][k] = -(np.outer(ub[k], xs[k]) + np.outer(u[k], xbs[k]))
        out["R"][k] = -0.5 * (np.outer(ub[k], u[k]) + np.outer(u[k], ub[k]))
        out["r"][k] = -ub[k]
        out["f"][k] = -lb[k]
    for k in range(1, N + 1):
        out["Q"][k] = -0.5 * (np.outer(xbs[k], xs[k]) + np.outer(xs[k], xbs[k]))
        out["q"][k] = -xbs[k]
    S0 = np.zeros((nu, nx)) if prob.S is None else prob.S[0]
    out["x0"] = -(prob.A[0].T @ lb[0] + S0.T @ ub[0])
    return out


def quad_loss(x, u):
    """l = 1/2 sum_k (||x_k||^2 + ||u_k||^2) over x_1..x_N and u_0..u_{N-1}; returns (l, gx, gu)."""
    return 0.5 * (np.sum(x * x) + np.sum(u * u)), x.copy(), u.copy()


def fd_grad(prob, name, entries, loss=quad_loss, h=1e-6):
    """Central differences of loss(solve_dense(prob)) w.r.t. the listed entries of array ``name``."""
    out = []
    for idx in entries:
        vals = []
        for s in (+1.0, -1.0):
            p = copy.deepcopy(prob)
            arr = getattr(p, name)
            if arr is None:
                shape = {"S": (p.N, p.nu, p.nx), "f": (p.N, p.nx)}[name]
                arr = np.zeros(shape)
                setattr(p, name, arr)
            arr[idx] += s * h
            x, u, _ = kkt.solve_dense(p)
            vals.append(loss(x, u)[0])
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.asarray(out)
