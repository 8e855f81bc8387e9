"""Explicit KKT system of the LQ optimal-control problem, and direct solves.

Follows the paper's problem statement (eq. ocp-eq, with E_j = I) and its
optimality conditions after elimination of the fixed initial state
(eq. opt-cond-ocp-eq):

    Q_N x_N - lam_{N-1}                              = -q_N
    R_k u_k + S_k x_k + B_k^T lam_k                  = -r_k        (0 < k < N)
    S_k^T u_k + Q_k x_k + A_k^T lam_k - lam_{k-1}    = -q_k        (0 < k < N)
    R_0 u_0 + B_0^T lam_0                            = -(r_0 + S_0 x_init)
    B_k u_k + A_k x_k - x_{k+1}                      = -f_k        (0 < k < N)
    B_0 u_0 - x_1                                    = -(f_0 + A_0 x_init)

Unknown ordering of z: primal w = [u_0, x_1, u_1, x_2, ..., u_{N-1}, x_N],
then the multipliers lam_0, ..., lam_{N-1}.  K = [[H, G^T], [G, 0]] with the
block-diagonal cost Hessian H and the dynamics Jacobian G.

Q and R enter through their symmetric parts 1/2 (M + M^T): only those appear in
the cost.  Q_0 and q_0 multiply the fixed x_0 and drop out.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp


def sym(m):
    return 0.5 * (m + np.swapaxes(m, -1, -2))


class Layout:
    """Offsets of u_k, x_k (k >= 1) and lam_k inside z."""

    def __init__(self, N, nx, nu):
        self.N, self.nx, self.nu = N, nx, nu
        self.nw = N * (nx + nu)
        self.n = self.nw + N * nx

    def u(self, k):  # k = 0..N-1
        s = 0 if k == 0 else self.nu + (k - 1) * (self.nx + self.nu) + self.nx
        return slice(s, s + self.nu)

    def x(self, k):  # k = 1..N
        s = self.nu + (k - 1) * (self.nx + self.nu)
        return slice(s, s + self.nx)

    def lam(self, k):  # k = 0..N-1
        s = self.nw + k * self.nx
        return slice(s, s + self.nx)


def _get(prob, name, k, shape):
    a = getattr(prob, name)
    return np.zeros(shape) if a is None else a[k]


def assemble(prob):
    """Return (K as scipy CSR, b, layout) for one instance (eq. opt-cond-ocp-eq)."""
    N, nx, nu = prob.N, prob.nx, prob.nu
    L = Layout(N, nx, nu)
    rows, cols, vals = [], [], []

    def put(rs, cs, M):
        M = np.asarray(M, dtype=np.float64)
        ii, jj = np.meshgrid(np.arange(rs.start, rs.stop), np.arange(cs.start, cs.stop), indexing="ij")
        rows.append(ii.ravel()); cols.append(jj.ravel()); vals.append(M.ravel())

    b = np.zeros(L.n)
    x0 = prob.x0
    eye = np.eye(nx)
    # cost Hessian H (symmetric), stage by stage
    for k in range(N):
        Rk = sym(prob.R[k])
        put(L.u(k), L.u(k), Rk)
        Sk = _get(prob, "S", k, (nu, nx))
        if k >= 1:
            put(L.u(k), L.x(k), Sk)
            put(L.x(k), L.u(k), Sk.T)
            put(L.x(k), L.x(k), sym(prob.Q[k]))
            b[L.x(k)] = -prob.q[k]
            b[L.u(k)] = -prob.r[k]
        else:
            b[L.u(0)] = -(prob.r[0] + Sk @ x0)
    put(L.x(N), L.x(N), sym(prob.Q[N]))
    b[L.x(N)] = -prob.q[N]
    # dynamics Jacobian G and its transpose
    for k in range(N):
        Ak, Bk = prob.A[k], prob.B[k]
        fk = _get(prob, "f", k, (nx,))
        put(L.lam(k), L.u(k), Bk)
        put(L.u(k), L.lam(k), Bk.T)
        put(L.lam(k), L.x(k + 1), -eye)
        put(L.x(k + 1), L.lam(k), -eye)
        if k >= 1:
            put(L.lam(k), L.x(k), Ak)
            put(L.x(k), L.lam(k), Ak.T)
            b[L.lam(k)] = -fk
        else:
            b[L.lam(0)] = -(fk + Ak @ x0)
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(L.n, L.n))
    K.sum_duplicates()
    return K, b, L


def split(z, L):
    """z -> (x [N, nx] for k = 1..N, u [N, nu], lam [N, nx])."""
    x = np.stack([z[L.x(k)] for k in range(1, L.N + 1)])
    u = np.stack([z[L.u(k)] for k in range(L.N)])
    lam = np.stack([z[L.lam(k)] for k in range(L.N)])
    return x, u, lam


def join(x, u, lam, L):
    z = np.zeros(L.n)
    for k in range(L.N):
        z[L.u(k)] = u[k]
        z[L.x(k + 1)] = x[k]
        z[L.lam(k)] = lam[k]
    return z


def solve_dense(prob):
    """Assemble K densely and solve K z = b with LAPACK LU (partial pivoting)."""
    K, b, L = assemble(prob)
    z = np.linalg.solve(K.toarray(), b)
    return split(z, L)


def _interleave_perm(L):
    """Stage-interleaved order u_0, lam_0, x_1, u_1, lam_1, x_2, ..., which gives K a narrow band."""
    idx = []
    for k in range(L.N):
        idx.extend(range(L.u(k).start, L.u(k).stop))
        idx.extend(range(L.lam(k).start, L.lam(k).stop))
        idx.extend(range(L.x(k + 1).start, L.x(k + 1).stop))
    return np.asarray(idx)


def banded_solve(K, rhs, L):
    """Solve K z = rhs for the assembled K of one instance in banded storage.

    The unknowns are permuted stage-interleaved so that K has bandwidth below
    2 (nu + 2 nx); the banded matrix is solved by LAPACK's banded LU.
    """
    perm = _interleave_perm(L)
    Kp = K[perm][:, perm].tocoo()
    lo = int(max(0, (Kp.row - Kp.col).max()))
    up = int(max(0, (Kp.col - Kp.row).max()))
    ab = np.zeros((lo + up + 1, L.n))
    ab[up + Kp.row - Kp.col, Kp.col] = Kp.data
    zp = scipy.linalg.solve_banded((lo, up), ab, rhs[perm], check_finite=True)
    z = np.empty(L.n)
    z[perm] = zp
    return z


def solve_banded(prob):
    """Same system as ``solve_dense`` in banded storage (for horizons where dense K does not fit)."""
    K, b, L = assemble(prob)
    return split(banded_solve(K, b, L), L)


def residual(prob, x, u, lam):
    """KKT residual rho = b - K z and the relative residual ||rho||_inf / ||b||_inf.

    This is the row-wise check of eq. opt-cond-ocp-eq: stationarity in u_k and
    x_k, and the dynamics.  If b = 0 the absolute residual is returned as the
    relative one.
    """
    K, b, L = assemble(prob)
    z = join(np.asarray(x, np.float64), np.asarray(u, np.float64), np.asarray(lam, np.float64), L)
    rho = b - K @ z
    nb = np.abs(b).max()
    rel = np.abs(rho).max() / nb if nb > 0 else np.abs(rho).max()
    return rho, rel


def backward_error(prob, x, u, lam):
    """Normwise backward error ||b - K z||_inf / (||K||_inf ||z||_inf + ||b||_inf)."""
    K, b, L = assemble(prob)
    z = join(x, u, lam, L)
    rho = b - K @ z
    knorm = np.abs(K).sum(axis=1).max()
    return np.abs(rho).max() / (knorm * np.abs(z).max() + np.abs(b).max())


def cost(prob, x, u):
    """Objective of eq. ocp-eq at (x_1..x_N, u_0..u_{N-1}) with x_0 = x_init, without the Q_0/q_0 constants."""
    N = prob.N
    xs = np.vstack([prob.x0[None, :], x])
    J = 0.0
    for k in range(N):
        Sk = _get(prob, "S", k, (prob.nu, prob.nx))
        J += 0.5 * u[k] @ sym(prob.R[k]) @ u[k] + u[k] @ Sk @ xs[k] + prob.r[k] @ u[k]
        if k >= 1:
            J += 0.5 * xs[k] @ sym(prob.Q[k]) @ xs[k] + prob.q[k] @ xs[k]
    J += 0.5 * xs[N] @ sym(prob.Q[N]) @ xs[N] + prob.q[N] @ xs[N]
    return J


def dynamics_violation(prob, x, u):
    """max_k ||A_k x_k + B_k u_k + f_k - x_{k+1}||_inf (x_0 = x_init)."""
    xs = np.vstack([prob.x0[None, :], x])
    worst = 0.0
    for k in range(prob.N):
        fk = _get(prob, "f", k, (prob.nx,))
        worst = max(worst, np.abs(prob.A[k] @ xs[k] + prob.B[k] @ u[k] + fk - xs[k + 1]).max())
    return worst
