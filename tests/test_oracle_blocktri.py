"""Pins of the block-tridiagonal oracle (CR / PCR / PCG) against facts that do not come from it.

* a scalar system worked by hand in exact fractions (tests/golden/blocktri_hand.json);
* three routes agreeing with LAPACK's dense solve: the CR factor (Cholesky of the permuted
  matrix), the written-out CR recursion and PCR, over sizes including non-powers of two;
* the CR factor blocks reproduce the permuted matrix and match the recursion's pivots;
* the stair preconditioner's factored form against the explicit block matrix printed beside it;
* PCG reaches its stopping tolerance and the dense solution within the implied bound;
* planted mistakes are caught.
"""
import inspect
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import blocktri as bt

GOLD = os.path.join(os.path.dirname(__file__), "golden", "blocktri_hand.json")


def _f(v):
    return float(Fraction(v))


def _random(seed, Nb, n, dominance=4.0):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((Nb, n, n))
    M = G @ np.swapaxes(G, 1, 2) + dominance * n * np.eye(n)
    K = rng.standard_normal((max(Nb - 1, 0), n, n))
    b = rng.standard_normal((Nb, n))
    return M, K, b


def _hand():
    g = json.load(open(GOLD))
    M = np.array([[[_f(v)]] for v in g["M"]])
    K = np.array([[[_f(v)]] for v in g["K"]])
    b = np.array([[_f(v)] for v in g["b"]])
    return g, M, K, b


def test_hand_example_solution_all_routes():
    g, M, K, b = _hand()
    x = np.array([_f(v) for v in g["x"]])
    for fn in (bt.solve, bt.cr_recursive, bt.pcr):
        np.testing.assert_allclose(fn(M, K, b)[:, 0], x, rtol=0, atol=1e-15)
    xg, it, rel = bt.pcg(M, K, b, tol=1e-15)
    np.testing.assert_allclose(xg[:, 0], x, rtol=0, atol=1e-14)


def test_hand_example_cr_factors():
    g, M, K, b = _hand()
    L, U, Y, level = bt.cr_factors(M, K)
    assert level[1] == level[3] == 0 and level[2] == 1 and level[0] == 2
    for k, v in g["pivots_squared"].items():
        assert L[int(k)][0, 0] ** 2 == pytest.approx(_f(v), rel=1e-15)
    assert U[1][0, 0] == pytest.approx(0.5, rel=1e-15) and U[3][0, 0] == pytest.approx(0.5, rel=1e-15)
    assert U[2][0, 0] < 0 and U[2][0, 0] ** 2 == pytest.approx(1 / 56, rel=1e-14)
    assert Y[1][0, 0] == pytest.approx(0.5, rel=1e-15)
    assert Y[3] is None and Y[2] is None and U[0] is None and Y[0] is None


@pytest.mark.parametrize("Nb", [1, 2, 3, 4, 5, 7, 8, 12, 16, 33])
@pytest.mark.parametrize("n", [1, 3, 6])
def test_routes_agree_with_dense(Nb, n):
    M, K, b = _random(Nb * 10 + n, Nb, n)
    x = bt.solve(M, K, b)
    scale = np.abs(x).max()
    for fn in (bt.cr_recursive, bt.pcr):
        assert np.abs(fn(M, K, b) - x).max() <= 1e-12 * scale, fn.__name__


@pytest.mark.parametrize("Nb,n", [(4, 2), (8, 3), (11, 4), (16, 2)])
def test_cr_factor_reproduces_permuted_matrix(Nb, n):
    M, K, _ = _random(Nb + 100 * n, Nb, n)
    L, U, Y, level = bt.cr_factors(M, K)
    A = bt.assemble(M, K)
    order = bt.cr_order(Nb)
    # rebuild the block factor from its blocks and compare L L^T with the permuted matrix
    pos = {k: i for i, k in enumerate(order)}
    F = np.zeros_like(A)
    for k in range(Nb):
        c = pos[k]
        F[c * n:(c + 1) * n, c * n:(c + 1) * n] = L[k]
        s = 1 << level[k]
        if U[k] is not None:
            r = pos[k - s]
            F[r * n:(r + 1) * n, c * n:(c + 1) * n] = U[k]
        if Y[k] is not None:
            r = pos[k + s]
            F[r * n:(r + 1) * n, c * n:(c + 1) * n] = Y[k]
    idx = np.concatenate([np.arange(k * n, (k + 1) * n) for k in order])
    np.testing.assert_allclose(F @ F.T, A[np.ix_(idx, idx)], rtol=0, atol=1e-11 * np.abs(A).max())
    # the factor has no other nonzero blocks: each column couples only to k -+ 2^l
    assert all(np.all(np.diag(L[k]) > 0) for k in range(Nb))


def test_stair_preconditioner_explicit_form():
    """The factored form L^{-T} L^{-1} (I - K L^{-T} L^{-1}) equals the explicit block matrix
    with M_i^{-1} on the diagonal and -M_i^{-1} K_i^T M_{i+1}^{-1} above it,
    -M_{i+1}^{-1} K_i M_i^{-1} below it."""
    Nb, n = 5, 3
    M, K, _ = _random(7, Nb, n)
    Mi = [np.linalg.inv(M[k]) for k in range(Nb)]
    P = np.zeros((Nb * n, Nb * n))
    for i in range(Nb):
        P[i * n:(i + 1) * n, i * n:(i + 1) * n] = Mi[i]
    for i in range(Nb - 1):
        P[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] = -Mi[i] @ K[i].T @ Mi[i + 1]
        P[(i + 1) * n:(i + 2) * n, i * n:(i + 1) * n] = -Mi[i + 1] @ K[i] @ Mi[i]
    rng = np.random.default_rng(3)
    for _ in range(3):
        r = rng.standard_normal((Nb, n))
        np.testing.assert_allclose(bt.stair_apply(M, K, r).reshape(-1), P @ r.reshape(-1), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(bt.jacobi_apply(M, K, r).reshape(-1),
                                   np.concatenate([Mi[k] @ r[k] for k in range(Nb)]), rtol=1e-12)


@pytest.mark.parametrize("precond", ["stair", "jacobi"])
def test_pcg_reaches_tolerance(precond):
    M, K, b = _random(11, 24, 4)
    x = bt.solve(M, K, b)
    for tol in (1e-6, 1e-10, 1e-13):
        xg, it, rel = bt.pcg(M, K, b, precond=precond, tol=tol)
        assert rel <= tol and it < 100
        # ||x - x*|| <= ||M^{-1}|| ||r||
        A = bt.assemble(M, K)
        bound = np.linalg.norm(np.linalg.inv(A), np.inf) * tol * np.abs(b).max()
        assert np.abs(xg - x).max() <= 1.01 * bound + 1e-15


def test_pcg_stair_not_slower_than_jacobi():
    M, K, b = _random(12, 32, 4, dominance=2.0)
    _, it_s, _ = bt.pcg(M, K, b, precond="stair", tol=1e-12)
    _, it_j, _ = bt.pcg(M, K, b, precond="jacobi", tol=1e-12)
    assert it_s <= it_j


MUTATIONS = [
    ("cr_recursive", "Mw[nxt] = Mw[nxt] - Yi @ Yi.T", "Mw[nxt] = Mw[nxt] + Yi @ Yi.T"),
    ("cr_recursive", "C[(prv, nxt)] = -(Yi @ Ui.T)", "C[(prv, nxt)] = -(Ui @ Yi.T)"),
    ("cr_recursive", "rhs = bt - Ui.T @ x[prv]", "rhs = bt + Ui.T @ x[prv]"),
    ("pcr", "K2.append(-(Y[k + s] @ U[k + s].T) if k + 2 * s < Nb", "K2.append(-(U[k + s] @ Y[k + s].T) if k + 2 * s < Nb"),
    ("pcr", "r -= U[k + s] @ bt[k + s]", "r -= U[k + s] @ bt[k]"),
    ("cr_factors", "order = cr_order(Nb)", "order = list(range(Nb))"),
    ("stair_apply", "return jacobi_apply(M, K, r - u)", "return jacobi_apply(M, K, r + u)"),
]


@pytest.mark.parametrize("fname,old,new", MUTATIONS)
def test_planted_mistake_is_caught(fname, old, new, monkeypatch):
    src = inspect.getsource(getattr(bt, fname))
    assert old in src
    ns = dict(vars(bt))
    exec(compile(src.replace(old, new, 1), f"<mutant {fname}>", "exec"), ns)
    monkeypatch.setattr(bt, fname, ns[fname])
    caught = False
    for check in (test_hand_example_solution_all_routes, test_hand_example_cr_factors,
                  lambda: test_routes_agree_with_dense(12, 3), test_stair_preconditioner_explicit_form):
        try:
            check()
        except (AssertionError, np.linalg.LinAlgError, TypeError):
            caught = True
            break
    assert caught, f"mutation in {fname} not detected"
