"""Pins of the QP oracle (oracle/qp.py) against facts that do not come from it.

* the optimality certificate on a QP solved by hand in exact fractions (tests/golden/qp_hand.json);
* psi'(tau) of eq. psi-prime (line_coefficients + merit_slope) against central differences of the
  merit function itself (eq. ocp-al-funcs evaluated directly), at points on both sides of
  activity changes;
* the exact step against a brute-force minimisation of the merit function along the line;
* the solver's result against brute-force enumeration of active sets on tiny QPs (each row
  inactive, at its lower or at its upper bound: the equality-constrained KKT solve whose point is
  feasible with multipliers of the right signs), and against the LQ solve when no bound is active;
* the certificate of the solver's result on the mass-spring benchmark;
* planted mistakes in copies of the slope and the step are caught.
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import kkt, qp

GOLD = os.path.join(os.path.dirname(__file__), "golden", "qp_hand.json")


def _f(v):
    return float(Fraction(v))


def _hand_problem():
    p = synth.LQProblem(A=np.ones((1, 1, 1)), B=np.ones((1, 1, 1)), Q=np.zeros((2, 1, 1)), R=np.ones((1, 1, 1)),
                        q=np.zeros((2, 1)), r=-np.ones((1, 1)), x0=np.zeros(1), S=np.zeros((1, 1, 1)),
                        f=np.zeros((1, 1)))
    C = np.zeros((2, 1, 1))
    D = np.ones((1, 1, 1))
    bl = np.array([[-np.inf], [-np.inf]])
    bu = np.array([[0.5], [np.inf]])
    return p, C, D, bl, bu


def test_certificate_hand_example():
    g = json.load(open(GOLD))
    p, C, D, bl, bu = _hand_problem()
    x = np.array([[_f(g["x1"])]])
    u = np.array([[_f(g["u0"])]])
    lam = np.array([[_f(g["lam0"])]])
    y = np.array([[_f(g["y0"])], [0.0]])
    st, dy, co = qp.certificate(p, C, D, bl, bu, x, u, lam, y)
    assert st == 0.0 and dy == 0.0 and co == 0.0
    y2 = np.array([[_f(g["perturbed_y0"])], [0.0]])
    st2, _, _ = qp.certificate(p, C, D, bl, bu, x, u, lam, y2)
    assert st2 == pytest.approx(_f(g["perturbed_stationarity"]), abs=1e-15)
    # and the solver reaches it
    xs, us, lams, ys, _ = qp.solve(p, C, D, bl, bu)
    assert abs(us[0, 0] - 0.5) < 1e-9 and abs(ys[0, 0] - 0.5) < 1e-8 and abs(lams[0, 0]) < 1e-8


def _random_qp(seed, N, nx, nu, m):
    p = synth.random_problem(seed, N, nx, nu)
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((N + 1, m, nx))
    D = rng.standard_normal((N, m, nu))
    bl = -rng.uniform(0.2, 1.0, (N + 1, m))
    bu = rng.uniform(0.2, 1.0, (N + 1, m))
    bl[rng.uniform(size=bl.shape) < 0.2] = -np.inf
    return p, C, D, bl, bu


def _state(seed, p, m):
    rng = np.random.default_rng(seed + 1)
    N, nx, nu = p.N, p.nx, p.nu
    u = rng.standard_normal((N, nu))
    x = qp.rollout(p, u)
    y = rng.standard_normal((N + 1, m))
    sigma = rng.uniform(1.0, 10.0, (N + 1, m))
    du = rng.standard_normal((N, nu))
    dx = qp.rollout(synth.LQProblem(A=p.A, B=p.B, Q=p.Q, R=p.R, q=p.q, r=p.r, x0=np.zeros(nx), S=p.S,
                                    f=np.zeros((N, nx))), du)
    return x, u, y, sigma, x + 0.1, u - 0.1, dx, du


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_slope_against_differences_of_the_merit(seed):
    p, C, D, bl, bu = _random_qp(seed, 5, 3, 2, 3)
    x, u, y, sigma, xb, ub, dx, du = _state(seed, p, 3)
    ginv = 0.3
    co = qp.line_coefficients(p, C, D, bl, bu, y, sigma, ginv, xb, ub, x, u, dx, du)
    psi = lambda t: qp.merit(p, C, D, bl, bu, y, sigma, ginv, xb, ub, x + t * dx, u + t * du)  # noqa: E731
    eta, beta, delta, alpha = co
    ok = np.isfinite(alpha) & (delta != 0)
    tb = np.sort((alpha[ok] / delta[ok]))
    for t in [-0.7, 0.0, 0.13, 0.5, 1.0, 2.5] + list(tb[:3] + 1e-4) + list(tb[:3] - 1e-4):
        h = 1e-6
        num = (psi(t + h) - psi(t - h)) / (2 * h)
        assert qp.merit_slope(*co, t) == pytest.approx(num, rel=1e-6, abs=1e-6), t


@pytest.mark.parametrize("seed", [4, 5, 6, 7])
def test_exact_step_against_brute_force(seed):
    p, C, D, bl, bu = _random_qp(seed, 4, 3, 2, 3)
    x, u, y, sigma, xb, ub, dx, du = _state(seed, p, 3)
    ginv = 0.5
    co = qp.line_coefficients(p, C, D, bl, bu, y, sigma, ginv, xb, ub, x, u, dx, du)
    if qp.merit_slope(*co, 0.0) > 0:   # make it a descent direction
        dx, du = -dx, -du
        co = qp.line_coefficients(p, C, D, bl, bu, y, sigma, ginv, xb, ub, x, u, dx, du)
    tau = qp.exact_step(*co)
    psi = lambda t: qp.merit(p, C, D, bl, bu, y, sigma, ginv, xb, ub, x + t * dx, u + t * du)  # noqa: E731
    grid = np.linspace(0.0, 4.0 * max(tau, 1.0), 20001)
    vals = np.array([psi(t) for t in grid])
    k = int(np.argmin(vals))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    for _ in range(100):                 # golden-section refinement of the grid minimiser
        a, b = lo + 0.382 * (hi - lo), lo + 0.618 * (hi - lo)
        if psi(a) < psi(b):
            hi = b
        else:
            lo = a
    # a minimiser located from function values is good to about sqrt(eps) of the scale
    assert tau == pytest.approx(0.5 * (lo + hi), rel=1e-5, abs=1e-7)
    assert abs(qp.merit_slope(*co, tau)) <= 1e-9 * max(1.0, abs(co[1]))


def _enumerate(p, C, D, bl, bu):
    """The QP solution by trying every activity pattern (tiny problems)."""
    K, b, L = kkt.assemble(p)
    Kd = K.toarray()
    N, m = p.N, C.shape[1]
    rows = []
    for j in range(N + 1):
        for i in range(m):
            g = np.zeros(L.n)
            const = 0.0
            if j < N:
                g[L.u(j)] = D[j, i]
            if j >= 1:
                g[L.x(j)] = C[j, i]
            else:
                const = C[0, i] @ p.x0
            rows.append((j, i, g, const))
    best = []
    for pat in itertools.product((0, -1, 1), repeat=len(rows)):
        act = [(r, s) for r, s in zip(rows, pat) if s != 0]
        if any((s == -1 and not np.isfinite(bl[r[0], r[1]])) or (s == 1 and not np.isfinite(bu[r[0], r[1]]))
               for r, s in act):
            continue
        na = len(act)
        M = np.zeros((L.n + na, L.n + na))
        rhs = np.zeros(L.n + na)
        M[:L.n, :L.n] = Kd
        rhs[:L.n] = b
        for a_, (r, s) in enumerate(act):
            g = r[2]
            M[:L.nw, L.n + a_] = g[:L.nw]
            M[L.n + a_, :L.nw] = g[:L.nw]
            rhs[L.n + a_] = (bl if s == -1 else bu)[r[0], r[1]] - r[3]
        try:
            sol = np.linalg.solve(M, rhs)
        except np.linalg.LinAlgError:
            continue
        z, ya = sol[:L.n], sol[L.n:]
        y = np.zeros((N + 1, m))
        for a_, (r, s) in enumerate(act):
            y[r[0], r[1]] = ya[a_]
        x, u, lam = kkt.split(z, L)
        w = qp.constraint_values(p, C, D, x, u)
        feas = np.all(w >= bl - 1e-9) and np.all(w <= bu + 1e-9)
        signs = all((s == 1 and y[r[0], r[1]] >= -1e-9) or (s == -1 and y[r[0], r[1]] <= 1e-9) for r, s in act)
        if feas and signs:
            best.append((x, u, lam, y))
    assert len(best) >= 1
    return best[0]


@pytest.mark.parametrize("seed", [11, 12, 13, 14])
def test_solver_against_active_set_enumeration(seed):
    p, C, D, bl, bu = _random_qp(seed, 2, 2, 1, 1)
    # bounds around a dynamics-feasible point (so the QP is feasible), tight enough that some are
    # active at the solution
    rng = np.random.default_rng(seed + 100)
    uf = rng.standard_normal((p.N, p.nu))
    wf = qp.constraint_values(p, C, D, qp.rollout(p, uf), uf)
    bl = wf - rng.uniform(0.05, 0.3, wf.shape)
    bu = wf + rng.uniform(0.05, 0.3, wf.shape)
    x, u, lam, y, _ = qp.solve(p, C, D, bl, bu)
    xe, ue, lame, ye = _enumerate(p, C, D, bl, bu)
    for a, b in ((x, xe), (u, ue), (lam, lame), (y, ye)):
        assert np.abs(a - b).max() <= 1e-7 * max(1.0, np.abs(b).max())
    st, dy, co = qp.certificate(p, C, D, bl, bu, x, u, lam, y)
    assert st <= 1e-8 and dy <= 1e-12 and co <= 1e-8


def test_inactive_bounds_reduce_to_the_lq_solve():
    p, C, D, bl, bu = _random_qp(21, 6, 3, 2, 2)
    bl[:] = -1e6
    bu[:] = 1e6
    x, u, lam, y, _ = qp.solve(p, C, D, bl, bu)
    xr, ur, lr = kkt.solve_dense(p)
    assert np.abs(y).max() == 0.0
    for a, b in ((x, xr), (u, ur), (lam, lr)):
        assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(b).max())


def test_mass_spring_certificate():
    prob, C, D, bl, bu = synth.mass_spring(6, 8, 2, seed=3)
    for i in range(2):
        p = prob.instance(i)
        x, u, lam, y, _ = qp.solve(p, C, D, bl, bu)
        st, dy, co = qp.certificate(p, C, D, bl, bu, x, u, lam, y)
        assert st <= 1e-9 and dy <= 1e-12 and co <= 1e-8
        assert np.abs(u).max() <= 0.5 + 1e-8 and np.abs(x[:, :6]).max() <= 4 + 1e-8
        assert np.abs(y).max() > 0        # some bounds are active (the benchmark is constrained)


def test_planted_mistakes():
    p, C, D, bl, bu = _random_qp(31, 4, 3, 2, 3)
    x, u, y, sigma, xb, ub, dx, du = _state(31, p, 3)
    ginv = 0.3
    eta, beta, delta, alpha = qp.line_coefficients(p, C, D, bl, bu, y, sigma, ginv, xb, ub, x, u, dx, du)
    psi = lambda t: qp.merit(p, C, D, bl, bu, y, sigma, ginv, xb, ub, x + t * dx, u + t * du)  # noqa: E731
    t, h = 0.37, 1e-6
    num = (psi(t + h) - psi(t - h)) / (2 * h)
    half = len(delta) // 2
    bad_delta = np.concatenate([-delta[:half], delta[half:]])       # lower-bound part with the wrong sign
    assert abs(qp.merit_slope(eta, beta, bad_delta, alpha, t) - num) > 1e-4
    assert abs(qp.merit_slope(eta, beta + ginv, delta, alpha, t) - num) > 1e-4   # a stray proximal term
    assert abs(qp.merit_slope(eta, beta, delta, alpha, t) - num) < 1e-5


def test_banded_newton_solves_match_dense():
    prob, C, D, bl, bu = synth.mass_spring(6, 6, 1, seed=4)
    p = prob.instance(0)
    a = qp.solve(p, C, D, bl, bu)
    b = qp.solve(p, C, D, bl, bu, linear="banded")
    for u, v in zip(a[:4], b[:4]):
        assert np.abs(u - v).max() <= 1e-8 * max(1.0, np.abs(v).max())
