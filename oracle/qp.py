"""Box-constrained LQ optimal-control QPs and their solution by the proximal augmented Lagrangian
method with semismooth Newton inner solves.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem (eq. ocp with inequality constraints): the LQ problem of eq. ocp-eq plus, per stage j,
    bl_j <= C_j x_j + D_j u_j <= bu_j   (j = 0..N-1; x_0 is the fixed initial state)
    bl_N <= C_N x_N <= bu_N
with +-inf allowed for one-sided rows.  Arrays for one instance with m rows per stage:
C [N+1, m, nx], D [N, m, nu], bl, bu [N+1, m]; multipliers y [N+1, m] (positive where an upper bound
is active, negative where a lower one is), lam [N, nx] for the dynamics as in eq. opt-cond-ocp-eq.

* ``certificate``: the QP's optimality conditions, the plain definition of the solution:
  stationarity of the Lagrangian (the rows of eq. opt-cond-ocp-eq plus G^T y), the dynamics, and
  ||Gz - Pi_[bl, bu](Gz + y)||_inf, which is zero exactly when Gz is feasible, y has the right sign
  on the active bounds and is zero elsewhere.
* ``merit`` / ``merit_slope``: the Gamma-proximal Sigma-augmented Lagrangian of eq. ocp-al-funcs
  along a direction, psi(tau), and its derivative in the form of eq. psi-prime.
* ``exact_step``: the minimiser of psi by sorting the breakpoints t_i = alpha_i / delta_i and
  walking the segments of the piecewise-linear psi' (the sort-based method the paper improves on).
* ``solve``: the method's steps in the paper's notation: semismooth Newton on the inner problem
  eq. ocp-al (generalised Hessians eq. qpalm-ocp-hessians, Newton system eq. newton-sys-with-x0 with
  x_0 eliminated as in eq. elim-x0, solved densely by ``kkt.solve_dense``), the exact line search,
  and the outer updates y <- yhat, proximal centre <- z, penalties raised on rows whose violation did
  not shrink enough.  The outer rules come from the QPALM papers the method cites (not printed in
  this paper); the constants are stated in ``solve``.

float64 numpy throughout.
"""
from __future__ import annotations

import copy

import numpy as np

from . import kkt


def _proj(v, lo, hi):
    return np.minimum(np.maximum(v, lo), hi)


def constraint_values(prob, C, D, x, u):
    """w_j = C_j x_j + D_j u_j for j = 0..N (x_0 = x_init; x given for stages 1..N)."""
    N = prob.N
    xs = np.vstack([prob.x0[None, :], x])
    w = np.einsum("jmn,jn->jm", C, xs)
    w[:N] += np.einsum("jmn,jn->jm", D, u)
    return w


def certificate(prob, C, D, bl, bu, x, u, lam, y):
    """(stationarity, dynamics, complementarity) residuals in the infinity norm."""
    K, b, L = kkt.assemble(prob)
    z = kkt.join(x, u, lam, L)
    r = K @ z - b                              # eq. opt-cond-ocp-eq rows: stationarity and dynamics
    gty = np.zeros(L.n)
    for j in range(prob.N + 1):
        if j < prob.N:
            gty[L.u(j)] += D[j].T @ y[j]
        if j >= 1:
            gty[L.x(j)] += C[j].T @ y[j]
    stat = r[:L.nw] + gty[:L.nw]
    dyn = r[L.nw:]
    w = constraint_values(prob, C, D, x, u)
    comp = w - _proj(w + y, bl, bu)
    return float(np.abs(stat).max()), float(np.abs(dyn).max()), float(np.abs(comp).max())


def _stage_cost(prob, x, u):
    """The LQ objective of eq. ocp-eq (x_0 = x_init)."""
    return kkt.cost(prob, x, u)


def merit(prob, C, D, bl, bu, y, sigma, ginv, xbar, ubar, x, u):
    """Gamma-proximal Sigma-augmented Lagrangian (eq. ocp-al-funcs) at (x, u); ginv = 1/gamma."""
    w = constraint_values(prob, C, D, x, u)
    v = w + y / sigma
    dist2 = np.sum(sigma * (v - _proj(v, bl, bu)) ** 2)
    prox = np.sum((x - xbar) ** 2) + np.sum((u - ubar) ** 2)
    return _stage_cost(prob, x, u) + 0.5 * dist2 + 0.5 * ginv * prox


def line_coefficients(prob, C, D, bl, bu, y, sigma, ginv, xbar, ubar, x, u, dx, du):
    """eta, beta, delta, alpha of eq. psi-prime along (dx, du), from their definitions: eta and beta
    from the stage costs of eq. ocp-eq (symmetric parts of Q, R; cross term S), the proximal term and
    the direction (x_0 is fixed, so its step is 0)."""
    N, nx, nu = prob.N, prob.nx, prob.nu
    S = np.zeros((N, nu, nx)) if prob.S is None else prob.S
    xs = np.vstack([prob.x0[None, :], x])
    dxs = np.vstack([np.zeros((1, nx)), dx])
    eta = ginv * (np.sum(dx * dx) + np.sum(du * du))
    beta = ginv * (np.sum(dx * (x - xbar)) + np.sum(du * (u - ubar)))
    for j in range(N + 1):
        Qs = kkt.sym(prob.Q[j])
        if j >= 1:
            eta += dxs[j] @ Qs @ dxs[j]
            beta += dxs[j] @ (Qs @ xs[j] + prob.q[j])
        if j < N:
            Rs = kkt.sym(prob.R[j])
            eta += du[j] @ Rs @ du[j] + 2.0 * du[j] @ S[j] @ dxs[j]
            beta += du[j] @ (Rs @ u[j] + S[j] @ xs[j] + prob.r[j]) + dxs[j] @ (S[j].T @ u[j])
    w = constraint_values(prob, C, D, x, u).reshape(-1)
    gd = np.einsum("jmn,jn->jm", C, dxs)
    gd[:N] += np.einsum("jmn,jn->jm", D, du)
    gd = gd.reshape(-1)
    s = sigma.reshape(-1)
    yy = y.reshape(-1)
    lo, hi = bl.reshape(-1), bu.reshape(-1)
    rs = np.sqrt(s)
    delta = np.concatenate([-rs * gd, rs * gd])
    with np.errstate(invalid="ignore"):
        alpha = np.concatenate([(yy + s * (w - lo)) / rs, -(yy + s * (w - hi)) / rs])
    return eta, beta, delta, alpha


def merit_slope(eta, beta, delta, alpha, tau):
    """psi'(tau) of eq. psi-prime (rows with infinite alpha, i.e. absent bounds, contribute 0)."""
    ok = np.isfinite(alpha)
    return eta * tau + beta + np.sum(delta[ok] * np.maximum(delta[ok] * tau - alpha[ok], 0.0))


def exact_step(eta, beta, delta, alpha):
    """Root of psi' over tau > 0 by sorting the breakpoints and walking the segments."""
    ok = np.isfinite(alpha) & (delta != 0.0)
    d, a = delta[ok], alpha[ok]
    t = a / d
    order = np.argsort(t, kind="stable")
    t, d, a = t[order], d[order], a[order]
    # at tau just above 0: active rows are those with delta tau - alpha > 0
    def slope_intercept(tau):
        act = d * tau - a > 0.0
        return eta + np.sum(d[act] ** 2), beta - np.sum(d[act] * a[act])
    lo = 0.0
    for k in range(len(t) + 1):
        hi = t[k] if k < len(t) else np.inf
        if hi <= lo:
            continue
        mid = lo + 1.0 if not np.isfinite(hi) else 0.5 * (lo + hi)
        sl, ic = slope_intercept(mid)
        tau = -ic / sl
        if tau <= hi or not np.isfinite(hi):
            return max(tau, lo)
        lo = hi
    raise AssertionError("psi' has no root")


def newton_problem(prob, C, D, bl, bu, y, sigma, ginv, xbar, ubar, x, u):
    """The Newton system at (x, u) as an LQ problem of eq. opt-cond-ocp-eq (x_0 eliminated: its step
    is 0): generalised Hessians eq. qpalm-ocp-hessians, gradients of eq. ocp-al-funcs as linear
    terms, the dynamics residuals c_j (0 at dynamics-feasible iterates) as f.  Also returns yhat and
    the active set."""
    N, nx, nu = prob.N, prob.nx, prob.nu
    w = constraint_values(prob, C, D, x, u)
    v = w + y / sigma
    act = (v < bl) | (v > bu)
    yhat = y + sigma * (w - _proj(v, bl, bu))
    sj = np.where(act, sigma, 0.0)
    S = np.zeros((N, nu, nx)) if prob.S is None else prob.S
    f = np.zeros((N, nx)) if prob.f is None else prob.f
    xs = np.vstack([prob.x0[None, :], x])
    q = copy.copy(prob)
    q.Q = np.empty_like(prob.Q)
    q.R = np.empty_like(prob.R)
    q.S = np.empty((N, nu, nx))
    q.q = np.empty_like(prob.q)
    q.r = np.empty_like(prob.r)
    q.f = np.empty((N, nx))
    q.x0 = np.zeros(nx)
    for j in range(N + 1):
        W = np.diag(sj[j])
        Qs = kkt.sym(prob.Q[j])
        q.Q[j] = Qs + C[j].T @ W @ C[j] + ginv * np.eye(nx)
        gx = Qs @ xs[j] + prob.q[j] + C[j].T @ yhat[j] + (ginv * (xs[j] - xbar[j - 1]) if j >= 1 else 0.0)
        if j < N:
            Rs = kkt.sym(prob.R[j])
            q.R[j] = Rs + D[j].T @ W @ D[j] + ginv * np.eye(nu)
            q.S[j] = S[j] + D[j].T @ W @ C[j]
            gx = gx + S[j].T @ u[j]
            q.r[j] = Rs @ u[j] + S[j] @ xs[j] + prob.r[j] + D[j].T @ yhat[j] + ginv * (u[j] - ubar[j])
            # the iterate satisfies the dynamics (it starts feasible and every direction stays in
            # the null space of the dynamics), so the constraint residual c_j of the Newton
            # right-hand side is 0; its rounding-level value is not fed back (it would tilt the
            # direction away from descent once the direction is that small)
            q.f[j] = 0.0
        q.q[j] = gx
    return q, yhat, act


def inner_residual(prob, npb, lam):
    """||grad l^Sigma(z) + M^T lam||_inf: the stationarity residual of the inner problem eq. ocp-al at the
    point the Newton problem npb was formed at, with dynamics multipliers lam (the rows of
    eq. opt-cond-ocp-eq for a zero step)."""
    N = prob.N
    r = 0.0
    for k in range(N):
        r = max(r, np.abs(npb.r[k] + prob.B[k].T @ lam[k]).max())
        if k >= 1:
            r = max(r, np.abs(npb.q[k] + prob.A[k].T @ lam[k] - lam[k - 1]).max())
    return max(r, np.abs(npb.q[N] - lam[N - 1]).max())


def rollout(prob, u):
    """States x_1..x_N of the dynamics from x_init under inputs u."""
    N = prob.N
    f = np.zeros((N, prob.nx)) if prob.f is None else prob.f
    x = np.empty((N, prob.nx))
    xk = prob.x0
    for k in range(N):
        xk = prob.A[k] @ xk + prob.B[k] @ u[k] + f[k]
        x[k] = xk
    return x


def solve(prob, C, D, bl, bu, sigma0=1e2, gamma=1e7, eps=1e-9, theta=0.25, sigma_up=10.0, sigma_max=1e9,
          max_outer=100, max_inner=50, inner_tol=1e-11, u0=None, y0=None, linear="dense"):
    """Proximal ALM with semismooth Newton inner solves.  Returns (x, u, lam, y, stats).

    The Newton systems are solved by ``kkt.solve_dense`` (linear="dense") or ``kkt.solve_banded``.
    Start: u = u0 (0), x by the dynamics; after every step x is simulated again from the new u (the
    same point in exact arithmetic; the dynamics stay exact, which the line search assumes),
    y = y0 (0), Sigma = sigma0, Gamma = gamma I, proximal centre = the start.  Inner loop: Newton
    direction (dense solve of the Newton system), exact step; it ends when the full step is taken
    without any row changing activity (z is then the inner minimiser: the model is exact), when the
    inner stationarity residual (``inner_residual`` with the Newton multipliers) is below
    inner_tol max(1, ||z||_inf, ||yhat||_inf), when the direction is at rounding level (an exact step
    along it would only amplify the dynamics' rounding residual), or after max_inner steps.  Where psi'(0) is not negative in floating point although d is a Newton
    direction (its decrease is below the rounding of psi'), the full step is taken.  Outer: y <- yhat, stop when ||Gz - Pi(Gz + y / Sigma)||_inf <= eps and
    ||(z - zbar) / gamma||_inf <= eps; otherwise Sigma_i <- min(sigma_max, sigma_up Sigma_i) on rows
    whose violation did not shrink below theta times the previous one, and the centre moves to z.
    """
    N, nu = prob.N, prob.nu
    m = C.shape[1]
    ginv = 1.0 / gamma
    u = np.zeros((N, nu)) if u0 is None else np.array(u0, dtype=np.float64)
    x = rollout(prob, u)
    y = np.zeros((N + 1, m)) if y0 is None else np.array(y0, dtype=np.float64)
    sigma = np.full((N + 1, m), float(sigma0))
    xbar, ubar = x.copy(), u.copy()
    e_prev = np.full((N + 1, m), np.inf)
    lam = np.zeros((N, prob.nx))
    stats = {"outer": 0, "inner": 0}
    for outer in range(max_outer):
        stats["outer"] = outer + 1
        for inner in range(max_inner):
            stats["inner"] += 1
            npb, yhat, act = newton_problem(prob, C, D, bl, bu, y, sigma, ginv, xbar, ubar, x, u)
            dx, du, lam = kkt.solve_dense(npb) if linear == "dense" else kkt.solve_banded(npb)
            scale = max(1.0, np.abs(x).max(), np.abs(u).max(), np.abs(yhat).max())
            if inner_residual(prob, npb, lam) <= inner_tol * scale:
                break                      # inner minimiser to tolerance: no step
            if max(np.abs(dx).max(), np.abs(du).max()) <= 1e-15 * scale:
                break                      # no step at rounding level

            eta, beta, delta, alpha = line_coefficients(prob, C, D, bl, bu, y, sigma, ginv, xbar, ubar, x, u, dx, du)
            if merit_slope(eta, beta, delta, alpha, 0.0) < 0.0:
                tau = exact_step(eta, beta, delta, alpha)
            else:
                tau = 1.0                  # descent below the rounding of psi': the full Newton step
            u = u + tau * du
            x = rollout(prob, u)           # = x + tau dx in exact arithmetic; keeps the dynamics exact

            _, _, act2 = newton_problem(prob, C, D, bl, bu, y, sigma, ginv, xbar, ubar, x, u)
            if abs(tau - 1.0) <= 1e-8 and np.array_equal(act, act2):
                break
        _, yhat, _ = newton_problem(prob, C, D, bl, bu, y, sigma, ginv, xbar, ubar, x, u)
        e = (yhat - y) / sigma
        y = yhat
        dual = ginv * max(np.abs(x - xbar).max(), np.abs(u - ubar).max())
        if np.abs(e).max() <= eps and dual <= eps:
            break
        grow = np.abs(e) > theta * e_prev
        sigma = np.where(grow, np.minimum(sigma_max, sigma_up * sigma), sigma)
        e_prev = np.abs(e)
        xbar, ubar = x.copy(), u.copy()
    return x, u, lam, y, stats
