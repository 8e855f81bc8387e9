"""Pins of the factorisation-update oracle (oracle/update.py) against facts that do not come from it.

* a scalar instance worked by hand in exact fractions (tests/golden/update_hand.json);
* a second route through the dense KKT matrix: the modified problem's KKT matrix minus the
  original one equals G^T dSigma G for the explicit constraint-row matrix G built here from the
  unknown layout (x_0 terms move to the right-hand side of the u_0 rows);
* an update followed by its downdate gives the original problem back; updates add up;
* the modified problem's factors reproduce the modified stage Hessians' recursion;
* planted mistakes in a copy of the modification fail the dense route.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import kkt, riccati, update

GOLD = os.path.join(os.path.dirname(__file__), "golden", "update_hand.json")


def _f(v):
    return float(Fraction(v))


def test_hand_example():
    g = json.load(open(GOLD))
    e = g["expected"]
    p = synth.LQProblem(A=np.array([[[_f(g["A"])]]]), B=np.array([[[_f(g["B"])]]]),
                        Q=np.array([[[_f(g["Q0"])]], [[_f(g["Q1"])]]]), R=np.array([[[_f(g["R0"])]]]),
                        q=np.zeros((2, 1)), r=np.zeros((1, 1)), x0=np.ones(1), S=np.array([[[_f(g["S0"])]]]))
    C = np.array([[[_f(g["C0"])]], [[_f(g["C1"])]]])
    D = np.array([[[_f(g["D0"])]]])
    dsig = np.array([[_f(g["dsig0"])], [_f(g["dsig1"])]])
    m = update.modified_problem(p, C, D, dsig)
    assert m.R[0, 0, 0] == pytest.approx(_f(e["R0"]), abs=1e-15)
    assert m.S[0, 0, 0] == pytest.approx(_f(e["S0"]), abs=1e-15)
    assert m.Q[0, 0, 0] == pytest.approx(_f(e["Q0"]), abs=1e-15)
    assert m.Q[1, 0, 0] == pytest.approx(_f(e["Q1"]), abs=1e-15)
    LQ, LR, LS = update.updated_factors(p, C, D, dsig)
    assert LR[0][0, 0] ** 2 == pytest.approx(_f(e["LR0_sq"]), rel=1e-14)
    assert LS[0][0, 0] ** 2 == pytest.approx(_f(e["LS0_sq"]), rel=1e-14)
    assert LQ[1][0, 0] ** 2 == pytest.approx(_f(e["LQ1_sq"]), rel=1e-14)
    # the input problem is left alone
    assert p.R[0, 0, 0] == _f(g["R0"]) and p.S[0, 0, 0] == _f(g["S0"])


def _rows_matrix(prob, C, D):
    """G: one row per (stage j, row i) acting on z = [u_0, x_1, u_1, ..., x_N, lam]; the x_0 part
    (known) is returned separately as the constant of each stage-0 row."""
    L = kkt.Layout(prob.N, prob.nx, prob.nu)
    N, m = prob.N, C.shape[1]
    G = np.zeros(((N + 1) * m, L.n))
    const = np.zeros((N + 1) * m)
    for j in range(N + 1):
        for i in range(m):
            row = j * m + i
            if j < N:
                G[row, L.u(j)] = D[j, i]
            if j >= 1:
                G[row, L.x(j)] = C[j, i]
            else:
                const[row] = C[j, i] @ prob.x0
    return G, const


def _dense_route_error(prob, mod, C, D, dsig):
    K0, b0, L = kkt.assemble(prob)
    K1, b1, _ = kkt.assemble(mod)
    G, const = _rows_matrix(prob, C, D)
    w = dsig.reshape(-1)
    dK = (K1 - K0).toarray()
    want = G.T @ (w[:, None] * G)
    # the penalty's linear part at the fixed x_0: -(D_0^T dSigma_0 C_0 x_0) in the u_0 rows
    db = np.zeros(L.n)
    db -= G.T @ (w * const)
    scale = max(1.0, np.abs(want).max())
    return max(np.abs(dK - want).max(), np.abs((b1 - b0) - db).max()) / scale


CASES = [(3, 2, 1, 1, True, True), (4, 3, 2, 2, False, True), (5, 4, 3, 3, True, False), (2, 5, 2, 4, False, False)]


@pytest.mark.parametrize("N,nx,nu,m,box,with_S", CASES)
def test_dense_kkt_route(N, nx, nu, m, box, with_S):
    p = synth.random_problem(31 + N, N, nx, nu, with_S=with_S)
    C, D, dsig = (a[0] for a in synth.random_update_rows(N, 1, N, nx, nu, m, density=0.7, box=box))
    dsig = dsig * np.where(np.arange(dsig.size).reshape(dsig.shape) % 3 == 0, -0.1, 1.0)
    mod = update.modified_problem(p, C, D, dsig)
    assert _dense_route_error(p, mod, C, D, dsig) < 1e-13


def test_update_then_downdate_and_additivity():
    N, nx, nu, m = 6, 4, 2, 3
    p = synth.random_problem(5, N, nx, nu)
    C, D, s = (a[0] for a in synth.random_update_rows(5, 1, N, nx, nu, m, box=False))
    C2, D2, s2 = (a[0] for a in synth.random_update_rows(6, 1, N, nx, nu, m, box=True))
    back = update.modified_problem(update.modified_problem(p, C, D, s), C, D, -s)
    for name in ("R", "S", "Q"):
        assert np.allclose(getattr(back, name), getattr(p, name), rtol=0, atol=1e-13)
    two = update.modified_problem(update.modified_problem(p, C, D, s), C2, D2, s2)
    one = update.modified_problem(p, np.concatenate([C, C2], 1), np.concatenate([D, D2], 1),
                                  np.concatenate([s, s2], 1))
    for name in ("R", "S", "Q"):
        assert np.allclose(getattr(two, name), getattr(one, name), rtol=0, atol=1e-13)


def test_factors_of_modified_problem():
    N, nx, nu, m = 7, 3, 2, 2
    p = synth.random_problem(9, N, nx, nu)
    C, D, s = (a[0] for a in synth.random_update_rows(9, 1, N, nx, nu, m, box=False))
    mod = update.modified_problem(p, C, D, s)
    LQ, LR, LS = update.updated_factors(p, C, D, s)
    rec = riccati.recursion(mod)
    for k in range(N):
        assert np.allclose(LR[k] @ LR[k].T, kkt.sym(rec["Rhat"][k]), atol=1e-11)
        assert np.allclose(LS[k] @ LR[k].T, rec["Shat"][k].T, atol=1e-11)
    for k in range(1, N + 1):
        assert np.allclose(LQ[k] @ LQ[k].T, rec["P"][k], atol=1e-11)
    # with every change zero the factors are the original ones
    LQ0, LR0, LS0 = update.updated_factors(p, C, D, 0 * s)
    LQr, LRr, LSr = riccati.reference_factors(p)
    assert all(np.array_equal(a, b) for a, b in zip(LR0, LRr))


def _mutant(kind):
    def f(prob, C, D, dsig):
        out = update.modified_problem(prob, 0 * C, 0 * D, 0 * dsig)
        for j in range(prob.N + 1):
            W = np.diag(dsig[j])
            if not (kind == "no_terminal" and j == prob.N):
                out.Q[j] = out.Q[j] + C[j].T @ W @ C[j]
            if j < prob.N:
                sgn = -1.0 if kind == "sign_R" else 1.0
                out.R[j] = out.R[j] + sgn * D[j].T @ W @ D[j]
                if kind == "S_from_C_only":
                    out.S[j] = out.S[j] + (C[j].T @ W @ C[j])[:prob.nu]
                elif kind == "S_without_weights":
                    out.S[j] = out.S[j] + D[j].T @ C[j]
                else:
                    out.S[j] = out.S[j] + D[j].T @ W @ C[j]
        return out
    return f


@pytest.mark.parametrize("kind", ["no_terminal", "sign_R", "S_from_C_only", "S_without_weights"])
def test_planted_mistakes_fail_dense_route(kind):
    N, nx, nu, m = 4, 3, 2, 2
    p = synth.random_problem(17, N, nx, nu)
    C, D, s = (a[0] for a in synth.random_update_rows(17, 1, N, nx, nu, m, density=1.0, box=False))
    good = update.modified_problem(p, C, D, s)
    assert _dense_route_error(p, good, C, D, s) < 1e-13
    bad = _mutant(kind)(p, C, D, s)
    assert _dense_route_error(p, bad, C, D, s) > 1e-6
