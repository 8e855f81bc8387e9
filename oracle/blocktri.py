"""Symmetric positive definite block-tridiagonal systems: cyclic reduction (CR), parallel cyclic
reduction (PCR) and preconditioned conjugate gradients (PCG).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The system of Sec. "Cyclic reduction of block-tridiagonal linear systems" (eq. block-tri):
diagonal blocks M_k (k = 0..Nb-1, n x n, SPD), subdiagonal blocks K_k (block row k+1, block
column k; k = 0..Nb-2) and right-hand side b_k.  Arrays: M [Nb, n, n], K [Nb-1, n, n], b [Nb, n].

* ``assemble`` / ``solve``: the dense matrix and its LAPACK solve -- the plain definition of what
  CR, PCR and PCG compute.
* ``valuation`` / ``cr_order``: the 2-adic valuation nu_2 (index 0 last) and the ordering of the
  block rows by increasing valuation (Sec. "Cyclic reduction as block Cholesky factorization").
* ``cr_factors``: the block Cholesky factor of the matrix permuted into that order.  CR *is* this
  factorisation (same section), so its blocks are the definition of the CR factors:
  L_k = diagonal block of column k, U_k = block (row k - 2^l, column k), Y_k = block
  (row k + 2^l, column k) for nu_2(k) = l.
* ``cr_recursive``: the elimination of the odd equations written out level by level
  (eq. cr-updated-odd, eq. cr-even, eq. cr-odd) -- a second route, used to pin the others.
* ``pcr``: the steps of Alg. "pcr" (both odd and even equations eliminated at every level), with
  neighbours outside 0..Nb-1 taken as absent (the non-periodic system).
* ``stair_apply`` / ``jacobi_apply`` / ``pcg``: the symmetric stair preconditioner in the
  factored form of the section "Handling of the final scalar levels"
  (Phi^{-1} = L^{-T} L^{-1} (I - K L^{-T} L^{-1}) with L = blkdiag(chol M_k) and K the
  off-diagonal part), the block-Jacobi one (L^{-T} L^{-1}), and textbook preconditioned conjugate
  gradients from x = 0, stopped when ||b - M x||_inf <= tol ||b||_inf.

float64 numpy / LAPACK throughout.
"""
from __future__ import annotations

import numpy as np


def assemble(M, K):
    Nb, n = M.shape[0], M.shape[1]
    A = np.zeros((Nb * n, Nb * n))
    for k in range(Nb):
        A[k * n:(k + 1) * n, k * n:(k + 1) * n] = M[k]
    for k in range(Nb - 1):
        A[(k + 1) * n:(k + 2) * n, k * n:(k + 1) * n] = K[k]
        A[k * n:(k + 1) * n, (k + 1) * n:(k + 2) * n] = K[k].T
    return A


def solve(M, K, b):
    """x = M^{-1} b for the assembled block-tridiagonal matrix (LAPACK LU)."""
    Nb, n = M.shape[0], M.shape[1]
    return np.linalg.solve(assemble(M, K), b.reshape(-1)).reshape(Nb, n)


def valuation(i, Nb):
    """nu_2(i), with index 0 given a valuation above every other index of 0..Nb-1 (it is last)."""
    if i == 0:
        return max(1, (Nb - 1).bit_length())
    v = 0
    while i % 2 == 0:
        i //= 2
        v += 1
    return v


def cr_order(Nb):
    """Block row indices ordered by increasing valuation, ties by index."""
    return sorted(range(Nb), key=lambda i: (valuation(i, Nb), i))


def cr_factors(M, K):
    """Blocks of the Cholesky factor of the matrix permuted into ``cr_order``.

    Returns (L, U, Y, level): L[k] lower n x n; U[k] / Y[k] the blocks of column k in the rows of
    k - 2^l / k + 2^l (None where that row does not exist), level[k] = nu_2(k) (index 0: the last
    level)."""
    Nb, n = M.shape[0], M.shape[1]
    order = cr_order(Nb)
    pos = {k: i for i, k in enumerate(order)}
    A = assemble(M, K)
    idx = np.concatenate([np.arange(k * n, (k + 1) * n) for k in order])
    Lf = np.linalg.cholesky(A[np.ix_(idx, idx)])

    def blk(r, c):
        return Lf[pos[r] * n:(pos[r] + 1) * n, pos[c] * n:(pos[c] + 1) * n]

    L, U, Y, level = [None] * Nb, [None] * Nb, [None] * Nb, [0] * Nb
    for k in range(Nb):
        lv = valuation(k, Nb)
        level[k] = lv
        L[k] = blk(k, k).copy()
        if k > 0:
            s = 1 << lv
            if k - s >= 0:
                U[k] = blk(k - s, k).copy()
            if k + s < Nb:
                Y[k] = blk(k + s, k).copy()
    return L, U, Y, level


def cr_recursive(M, K, b):
    """Cyclic reduction written out: at level l (stride s = 2^l) eliminate the equations k with
    nu_2(k) = l from their neighbours k - s, k + s (eq. cr-updated-odd, eq. cr-even), recurse on
    the rest, then recover the eliminated unknowns (eq. cr-odd)."""
    Nb, n = M.shape[0], M.shape[1]
    Mw = {k: M[k].copy() for k in range(Nb)}
    # coupling of the current reduced system: C[(i, j)] = block (row j, column i), i < j
    C = {(k, k + 1): K[k].copy() for k in range(Nb - 1)}
    bw = {k: b[k].copy() for k in range(Nb)}
    saved = []
    active = list(range(Nb))
    while len(active) > 1:
        odd = active[1::2]
        even = active[0::2]
        lev = []
        for k in odd:
            L = np.linalg.cholesky(Mw[k])
            i = active.index(k)
            prv, nxt = active[i - 1], (active[i + 1] if i + 1 < len(active) else None)
            Ui = np.linalg.solve(L, C[(prv, k)]).T            # U = K_bwd L^{-T}, K_bwd = block (row prv, col k)
            Yi = np.linalg.solve(L, C[(k, nxt)].T).T if nxt is not None else None
            bt = np.linalg.solve(L, bw[k])
            lev.append((k, prv, nxt, L, Ui, Yi, bt))
        for k, prv, nxt, L, Ui, Yi, bt in lev:
            Mw[prv] = Mw[prv] - Ui @ Ui.T
            bw[prv] = bw[prv] - Ui @ bt
            if nxt is not None:
                Mw[nxt] = Mw[nxt] - Yi @ Yi.T
                bw[nxt] = bw[nxt] - Yi @ bt
                C[(prv, nxt)] = -(Yi @ Ui.T)
        saved.append(lev)
        active = even
    x = {0: np.linalg.solve(Mw[0], bw[0])}
    for lev in reversed(saved):
        for k, prv, nxt, L, Ui, Yi, bt in lev:
            rhs = bt - Ui.T @ x[prv] - (Yi.T @ x[nxt] if nxt is not None else 0.0)
            x[k] = np.linalg.solve(L.T, rhs)
    return np.stack([x[k] for k in range(Nb)])


def pcr(M, K, b):
    """Parallel cyclic reduction: every level factors every block, eliminates both neighbours at
    distance s = 2^l from every equation, until no coupling is left (Alg. "pcr")."""
    Nb, n = M.shape[0], M.shape[1]
    Mw = [M[k].copy() for k in range(Nb)]
    Kw = [K[k].copy() for k in range(Nb - 1)] + [np.zeros((n, n))]   # Kw[k]: row k + s, column k
    bw = [b[k].copy() for k in range(Nb)]
    s = 1
    while s < Nb:
        L = [np.linalg.cholesky(Mw[k]) for k in range(Nb)]
        Y = [np.linalg.solve(L[k], Kw[k].T).T if k + s < Nb else None for k in range(Nb)]
        U = [np.linalg.solve(L[k], Kw[k - s]).T if k - s >= 0 else None for k in range(Nb)]
        bt = [np.linalg.solve(L[k], bw[k]) for k in range(Nb)]
        M2, K2, b2 = [], [], []
        for k in range(Nb):
            m, r = Mw[k].copy(), bw[k].copy()
            if k - s >= 0:
                m -= Y[k - s] @ Y[k - s].T
                r -= Y[k - s] @ bt[k - s]
            if k + s < Nb:
                m -= U[k + s] @ U[k + s].T
                r -= U[k + s] @ bt[k + s]
            M2.append(m)
            b2.append(r)
            K2.append(-(Y[k + s] @ U[k + s].T) if k + 2 * s < Nb else np.zeros((n, n)))
        Mw, Kw, bw = M2, K2, b2
        s *= 2
    return np.stack([np.linalg.solve(Mw[k], bw[k]) for k in range(Nb)])


def matvec(M, K, x):
    y = np.einsum("kij,kj->ki", M, x)
    y[1:] += np.einsum("kij,kj->ki", K, x[:-1])
    y[:-1] += np.einsum("kji,kj->ki", K, x[1:])
    return y


def jacobi_apply(M, K, r):
    return np.stack([np.linalg.solve(M[k], r[k]) for k in range(M.shape[0])])


def stair_apply(M, K, r):
    """Phi^{-1} r = D^{-1} (r - Koff D^{-1} r), D = blkdiag(M_k) = L L^T, Koff the off-diagonal part."""
    t = jacobi_apply(M, K, r)
    u = matvec(np.zeros_like(M), K, t)
    return jacobi_apply(M, K, r - u)


def pcg(M, K, b, precond="stair", tol=1e-12, max_it=1000):
    """Textbook preconditioned CG from x = 0.  Returns (x, iterations, ||b - M x||_inf / ||b||_inf)."""
    P = stair_apply if precond == "stair" else jacobi_apply
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.abs(b).max()
    if nb == 0:
        return x, 0, 0.0
    z = P(M, K, r)
    p = z.copy()
    rz = np.sum(r * z)
    it = 0
    while np.abs(r).max() > tol * nb and it < max_it:
        q = matvec(M, K, p)
        alpha = rz / np.sum(p * q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        z = P(M, K, r)
        rz2 = np.sum(r * z)
        p = z + (rz2 / rz) * p
        rz = rz2
    return x, it, float(np.abs(b - matvec(M, K, x)).max() / nb)
