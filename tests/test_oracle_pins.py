"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* hand-solved KKT systems in exact fractions (tests/golden/hand_examples.json);
* three independent solution routes agreeing: dense KKT (eq. opt-cond-ocp-eq),
  textbook Riccati (eq. riccati-recursion-P) and condensing;
* the scalar DARE closed form at a long horizon and scipy's DARE solver;
* invariants of the cost-to-go, the optimal-cost identity, padding invariance
  (Sec. 'Remainders and padding');
* the adjoint gradient against central finite differences;
* planted mistakes in the oracle source are caught by these pins.
"""
import copy
import inspect
import json
import os
import types
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import adjoint, closed, condense, kkt, riccati

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _prob_from_json(ex):
    arr = lambda k: np.asarray(ex[k], dtype=np.float64)  # noqa: E731
    return synth.LQProblem(A=arr("A"), B=arr("B"), Q=arr("Q"), R=arr("R"), q=arr("q"), r=arr("r"),
                           x0=arr("x0"), S=arr("S"), f=arr("f"))


def _frac(a):
    return np.asarray([[float(Fraction(v)) for v in row] for row in a])


@pytest.mark.parametrize("route", ["dense", "banded", "riccati", "condense"])
def test_hand_examples(route):
    data = json.load(open(GOLD))
    fn = {"dense": kkt.solve_dense, "banded": kkt.solve_banded, "riccati": riccati.solve,
          "condense": condense.solve}[route]
    for ex in data["examples"]:
        p = _prob_from_json(ex)
        x, u, lam = fn(p)
        sol = ex["solution"]
        np.testing.assert_allclose(u, _frac(sol["u"]), rtol=0, atol=1e-13)
        np.testing.assert_allclose(x, _frac(sol["x"]), rtol=0, atol=1e-13)
        np.testing.assert_allclose(lam, _frac(sol["lam"]), rtol=0, atol=1e-13)


CASES = [(1, 1, 1), (1, 3, 2), (2, 2, 1), (3, 3, 2), (5, 4, 3), (7, 2, 5), (12, 6, 2)]


@pytest.mark.parametrize("N,nx,nu", CASES)
@pytest.mark.parametrize("withS,withf", [(True, True), (False, False), (True, False)])
def test_three_routes_agree(N, nx, nu, withS, withf):
    p = synth.random_problem(N * 100 + nx * 10 + nu, N, nx, nu, with_S=withS, with_f=withf)
    xd, ud, ld = kkt.solve_dense(p)
    for fn in (riccati.solve, condense.solve, kkt.solve_banded):
        x, u, lam = fn(p)
        scale = max(np.abs(xd).max(), np.abs(ud).max(), np.abs(ld).max())
        assert np.abs(x - xd).max() <= 1e-11 * scale
        assert np.abs(u - ud).max() <= 1e-11 * scale
        assert np.abs(lam - ld).max() <= 1e-11 * scale


def test_residual_small_at_independent_solutions():
    p = synth.random_problem(7, 9, 5, 3)
    for fn in (riccati.solve, condense.solve):
        _, rel = kkt.residual(p, *fn(p))
        assert rel < 1e-13


def test_residual_sees_each_block():
    """Perturbing one unknown shows up exactly in the rows the KKT conditions couple it to."""
    p = synth.random_problem(8, 4, 3, 2)
    x, u, lam = kkt.solve_dense(p)
    _, b, L = kkt.assemble(p)
    d = np.array([1e-3, -2e-3])
    u2 = u.copy(); u2[2] += d
    rho, rel = kkt.residual(p, x, u2, lam)
    assert rel > 1e-5
    # dynamics row of stage 2: B_2 u_2 + A_2 x_2 - x_3 = -f_2  -> residual changes by -B_2 d
    np.testing.assert_allclose(rho[L.lam(2)], -p.B[2] @ d, atol=1e-12)
    # u_2 stationarity row: R_2 u_2 + ... -> residual changes by -sym(R_2) d
    np.testing.assert_allclose(rho[L.u(2)], -kkt.sym(p.R[2]) @ d, atol=1e-12)
    # x_2 row: S_2^T u_2 ... -> -S_2^T d
    np.testing.assert_allclose(rho[L.x(2)], -p.S[2].T @ d, atol=1e-12)
    others = np.ones(L.n, bool)
    for s in (L.lam(2), L.u(2), L.x(2)):
        others[s] = False
    assert np.abs(rho[others]).max() < 1e-12


ERRGOLD = os.path.join(os.path.dirname(__file__), "golden", "error_measures.json")


def test_error_measures_hand_values():
    """Backward error, relative residual and dynamics violation of perturbed iterates of the hand
    examples against values computed by hand in exact fractions (tests/golden/error_measures.json)."""
    exs = {e["name"]: e for e in json.load(open(GOLD))["examples"]}
    for case in json.load(open(ERRGOLD))["cases"]:
        p = _prob_from_json(exs[case["example"]])
        it = case["iterate"]
        x, u, lam = _frac(it["x"]), _frac(it["u"]), _frac(it["lam"])
        assert kkt.backward_error(p, x, u, lam) == pytest.approx(float(Fraction(case["backward_error"])), rel=1e-15)
        assert kkt.residual(p, x, u, lam)[1] == pytest.approx(float(Fraction(case["rel_res"])), rel=1e-15)
        assert kkt.dynamics_violation(p, x, u) == pytest.approx(float(Fraction(case["dynamics_violation"])),
                                                                abs=1e-15)


def test_error_measures_bound_each_other():
    """For any iterate the backward error is at most the relative residual (its denominator is
    larger), and both vanish at the exact solution; the dynamics violation is at most the
    residual's largest dynamics row."""
    p = synth.random_problem(31, 7, 4, 3)
    x, u, lam = kkt.solve_dense(p)
    assert kkt.backward_error(p, x, u, lam) < 1e-15
    assert kkt.dynamics_violation(p, x, u) < 1e-13
    rng = np.random.default_rng(3)
    for _ in range(5):
        xp = x + 1e-3 * rng.standard_normal(x.shape)
        up = u + 1e-3 * rng.standard_normal(u.shape)
        rho, rel = kkt.residual(p, xp, up, lam)
        be = kkt.backward_error(p, xp, up, lam)
        _, b, L = kkt.assemble(p)
        assert 0 < be <= rel
        dyn = max(np.abs(rho[L.lam(k)]).max() for k in range(p.N))
        assert kkt.dynamics_violation(p, xp, up) == pytest.approx(dyn, rel=1e-12)


def test_banded_adjoint_matches_dense():
    """The banded adjoint route (used at horizons where the dense one is too slow) gives the dense
    route's gradients, which are pinned to finite differences below."""
    p = synth.random_problem(41, 9, 5, 3)
    x, u, _ = kkt.solve_dense(p)
    _, gx, gu = adjoint.quad_loss(x, u)
    gd, _, _ = adjoint.adjoint_grad(p, gx, gu)
    gb, _, _ = adjoint.adjoint_grad_banded(p, gx, gu)
    for k in gd:
        assert np.abs(gd[k] - gb[k]).max() <= 1e-12 * max(1.0, np.abs(gd[k]).max()), k


@pytest.mark.parametrize("a,b,q,r", [(0.9, 0.5, 1.0, 0.1), (1.2, 1.0, 2.0, 0.5), (0.3, 2.0, 0.7, 3.0)])
def test_scalar_dare_closed_form(a, b, q, r):
    N = 1000
    one = np.ones((N, 1, 1))
    p = synth.LQProblem(A=a * one, B=b * one, Q=q * np.ones((N + 1, 1, 1)), R=r * one,
                        q=np.zeros((N + 1, 1)), r=np.zeros((N, 1)), x0=np.ones(1))
    P = riccati.recursion(p)["P"]
    Pinf = closed.scalar_dare(a, b, q, r)
    assert abs(P[1][0, 0] - Pinf) <= 1e-14 * Pinf
    assert abs(P[N][0, 0] - q) == 0.0


def test_dare_matches_scipy():
    rng = np.random.default_rng(5)
    nx, nu, N = 4, 2, 400
    A = 0.9 * np.eye(nx) + 0.2 * rng.standard_normal((nx, nx))
    B = rng.standard_normal((nx, nu))
    W = rng.standard_normal((nx + nu, nx + nu))
    H = W @ W.T + np.eye(nx + nu)
    R, S, Q = H[:nu, :nu], H[:nu, nu:], H[nu:, nu:]
    p = synth.LQProblem(A=np.broadcast_to(A, (N, nx, nx)).copy(), B=np.broadcast_to(B, (N, nx, nu)).copy(),
                        Q=np.broadcast_to(Q, (N + 1, nx, nx)).copy(), R=np.broadcast_to(R, (N, nu, nu)).copy(),
                        S=np.broadcast_to(S, (N, nu, nx)).copy(), q=np.zeros((N + 1, nx)), r=np.zeros((N, nu)),
                        x0=np.ones(nx))
    P1 = riccati.recursion(p)["P"][1]
    X = scipy.linalg.solve_discrete_are(A, B, Q, R, s=S.T)
    assert np.abs(P1 - X).max() <= 1e-10 * np.abs(X).max()


def test_cost_to_go_invariants():
    b = synth.make_batch(2, batch=3, N=20)
    for i in range(3):
        p = b.instance(i)
        P = riccati.recursion(p)["P"]
        for k in range(1, p.N + 1):
            assert np.abs(P[k] - P[k].T).max() <= 1e-12 * np.abs(P[k]).max()
            assert np.linalg.eigvalsh(kkt.sym(P[k])).min() > 0
            # with S = 0: P_k - Q_k = A^T (P_{k+1}^{-1} + B R^{-1} B^T)^{-1} A is PSD
            assert np.linalg.eigvalsh(kkt.sym(P[k] - p.Q[k])).min() > -1e-10 * np.abs(P[k]).max()


def test_optimal_cost_identity():
    p = synth.random_problem(11, 8, 4, 3, with_f=False)
    p.q[:] = 0.0
    p.r[:] = 0.0
    x, u, _ = kkt.solve_dense(p)
    J = kkt.cost(p, x, u)
    rec = riccati.recursion(p)
    A0 = p.A[0]
    Rh, Sh = rec["Rhat"][0], rec["Shat"][0]
    P0t = A0.T @ rec["P"][1] @ A0 - Sh.T @ np.linalg.solve(Rh, Sh)
    assert abs(J - 0.5 * p.x0 @ P0t @ p.x0) <= 1e-12 * abs(J)


def test_reference_factors_reproduce_P():
    p = synth.random_problem(12, 6, 4, 2)
    rec = riccati.recursion(p)
    LQ, LR, LS = riccati.reference_factors(p, rec)
    for k in range(1, p.N + 1):
        np.testing.assert_allclose(LQ[k] @ LQ[k].T, rec["P"][k], rtol=1e-12, atol=1e-12)
    for k in range(p.N):
        np.testing.assert_allclose(LR[k] @ LR[k].T, rec["Rhat"][k], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(LS[k] @ LR[k].T, rec["Shat"][k].T, rtol=1e-12, atol=1e-12)
        # the closed-loop gain K = -Rhat^{-1} Shat = -LR^{-T} LS^T
        np.testing.assert_allclose(-np.linalg.solve(LR[k].T, LS[k].T), rec["K"][k], rtol=1e-10, atol=1e-12)


def test_padding_invariance():
    """Padding stages with Q = I, R = I, S = 0, A = 0, B = 0 leaves the original solution unchanged."""
    p = synth.random_problem(13, 5, 3, 2)
    N, nx, nu, pad = p.N, p.nx, p.nu, 3
    pp = copy.deepcopy(p)
    pp.A = np.concatenate([p.A, np.zeros((pad, nx, nx))])
    pp.B = np.concatenate([p.B, np.zeros((pad, nx, nu))])
    pp.R = np.concatenate([p.R, np.broadcast_to(np.eye(nu), (pad, nu, nu))])
    pp.S = np.concatenate([p.S, np.zeros((pad, nu, nx))])
    pp.Q = np.concatenate([p.Q, np.broadcast_to(np.eye(nx), (pad, nx, nx))])
    pp.q = np.concatenate([p.q, np.zeros((pad, nx))])
    pp.r = np.concatenate([p.r, np.zeros((pad, nu))])
    pp.f = np.concatenate([p.f, np.zeros((pad, nx))])
    x, u, lam = kkt.solve_dense(p)
    xp, up, lp = kkt.solve_dense(pp)
    np.testing.assert_allclose(xp[:N], x, atol=1e-12)
    np.testing.assert_allclose(up[:N], u, atol=1e-12)
    np.testing.assert_allclose(lp[:N], lam, atol=1e-12)
    assert np.abs(up[N:]).max() < 1e-12 and np.abs(xp[N:]).max() < 1e-12


@pytest.mark.parametrize("withS,withf", [(True, True), (False, False)])
def test_adjoint_matches_finite_differences(withS, withf):
    p = synth.random_problem(21, 3, 3, 2, with_S=withS, with_f=withf)
    x, u, _ = kkt.solve_dense(p)
    _, gx, gu = adjoint.quad_loss(x, u)
    g, _, _ = adjoint.adjoint_grad(p, gx, gu)
    rng = np.random.default_rng(0)
    names = ["A", "B", "Q", "R", "q", "r", "x0"] + (["S"] if withS else []) + (["f"] if withf else [])
    for name in names:
        arr = getattr(p, name)
        entries = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]
        fd = adjoint.fd_grad(p, name, entries)
        an = np.array([g[name][e] for e in entries])
        assert np.abs(fd - an).max() <= 1e-7 * max(1.0, np.abs(an).max()), name
    # Q_0 and q_0 do not influence the solution
    assert np.all(g["Q"][0] == 0) and np.all(g["q"][0] == 0)


def test_generators_are_seeded_and_shaped():
    a = synth.make_batch(2, batch=2)
    b = synth.make_instance(2, 1)
    assert a.A.shape == (2, 50, 12, 12) and a.Q.shape == (2, 51, 12, 12) and a.R.shape == (2, 50, 4, 4)
    np.testing.assert_array_equal(a.A[1], b.A)
    np.testing.assert_array_equal(a.Q[1], a.Q[1].swapaxes(-1, -2))
    d = np.diagonal(a.R, axis1=-2, axis2=-1)
    assert d.min() >= 0.1 and d.max() <= 1.1
    # workload 4: A_k = 0.99 * Haar orthogonal + 0.01 * G, so its singular values stay near 0.99
    c4 = synth.make_instance(4, 0, N=3, nx=16, nu=4)
    assert np.abs(np.linalg.svd(c4.A[0], compute_uv=False) - 0.99).max() < 0.1
    rag = synth.make_ragged(16)
    assert all(6 <= p.nx <= 64 and 2 <= p.nu <= 16 and 10 <= p.N <= 200 for p in rag)


# ---------------------------------------------------------------------------
# Planted mistakes: each mutated copy of an oracle function must fail a pin.

def _mutant(module, fname, old, new):
    src = inspect.getsource(getattr(module, fname))
    assert old in src, (fname, old)
    ns = dict(vars(module))
    exec(compile(src.replace(old, new, 1), f"<mutant {fname}>", "exec"), ns)
    return ns[fname]


MUTATIONS = [
    (kkt, "assemble", "put(L.x(k + 1), L.lam(k), -eye)", "put(L.x(k + 1), L.lam(k), eye)"),
    (kkt, "assemble", "b[L.u(0)] = -(prob.r[0] + Sk @ x0)", "b[L.u(0)] = -(prob.r[0])"),
    (kkt, "assemble", "put(L.x(k), L.lam(k), Ak.T)", "put(L.x(k), L.lam(k), Ak)"),
    (kkt, "assemble", "b[L.lam(0)] = -(fk + Ak @ x0)", "b[L.lam(0)] = -(fk)"),
    (riccati, "recursion", "Shat = _S(prob, k) + B.T @ Pn @ A", "Shat = B.T @ Pn @ A"),
    (riccati, "recursion", "w = Pn @ _f(prob, k) + p[k + 1]", "w = p[k + 1]"),
    (riccati, "recursion", "Rhat = sym(prob.R[k]) + B.T @ Pn @ B", "Rhat = sym(prob.R[k]) + B.T @ B"),
    (riccati, "solve", "lam[k] = rec[\"P\"][k + 1] @ xn + rec[\"p\"][k + 1]", "lam[k] = rec[\"P\"][k] @ xn + rec[\"p\"][k + 1]"),
    (condense, "solve", "rv[0:nu] += S[0] @ prob.x0", "rv[0:nu] -= S[0] @ prob.x0"),
    (kkt, "backward_error", "(knorm * np.abs(z).max() + np.abs(b).max())", "(knorm * np.abs(z).max())"),
    (kkt, "backward_error", "knorm = np.abs(K).sum(axis=1).max()", "knorm = np.abs(K).max()"),
    (kkt, "dynamics_violation", "fk - xs[k + 1]", "fk - xs[k]"),
    (kkt, "dynamics_violation", "prob.B[k] @ u[k]", "prob.B[k] @ u[max(k - 1, 0)]"),
]


@pytest.mark.parametrize("mod,fname,old,new", MUTATIONS)
def test_planted_mistake_is_caught(mod, fname, old, new, monkeypatch):
    bad = _mutant(mod, fname, old, new)
    monkeypatch.setattr(mod, fname, bad)
    caught = False
    if fname in ("backward_error", "dynamics_violation"):
        try:
            test_error_measures_hand_values()
        except AssertionError:
            caught = True
        assert caught, f"mutation in {mod.__name__}.{fname} not detected"
        return
    try:
        test_hand_examples("dense" if mod is kkt else ("riccati" if mod is riccati else "condense"))
    except AssertionError:
        caught = True
    if not caught:
        try:
            test_three_routes_agree(5, 4, 3, True, True)
        except AssertionError:
            caught = True
    assert caught, f"mutation in {mod.__name__}.{fname} not detected"
