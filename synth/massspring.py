"""The mass-spring MPC benchmark of the paper's experiments (Sec. "Problem description"): M masses
(M a multiple of 6) in a chain between two walls, nu = M / 2 actuators between pairs of masses (the
6-mass pattern W repeated), unit masses and springs, no friction, the walls at distance 0 so the
steady state is the origin; zero-order hold with T_s = 15 s / N; cost Q = Q_N = I, R = I; bounds
|position| <= 4 and |u| <= 0.5.  Initial states: velocities 0, positions uniform in [-3, 3].

Only the problem definition (the discretisation by the matrix exponential is part of it): no solver
arithmetic.  Constraint rows per stage (m = M + nu): the M positions (C = [I 0]) and the nu inputs
(D = I); the terminal stage has the position rows and inactive input rows (bounds +-inf).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .problems import LQProblem, SEED_ROOT


def _continuous(M):
    if M % 6 != 0:
        raise ValueError("M must be a multiple of 6")
    k = m_ = 1.0
    V = (np.diag(-2.0 * k * np.ones(M)) + np.diag(k * np.ones(M - 1), 1) + np.diag(k * np.ones(M - 1), -1)) / m_
    Ac = np.block([[np.zeros((M, M)), np.eye(M)], [V, np.zeros((M, M))]])
    W = np.zeros((6, 3))
    W[0, 0], W[1, 0] = 1.0, -1.0
    W[2, 1], W[4, 1] = 1.0, -1.0
    W[3, 2], W[5, 2] = 1.0, -1.0
    W /= m_
    Bc = np.vstack([np.zeros((M, M // 2)), scipy.linalg.block_diag(*([W] * (M // 6)))])
    return Ac, Bc


def discretise(M, N):
    """(A, B) of the zero-order hold with T_s = 15 / N."""
    Ac, Bc = _continuous(M)
    nx, nu = Ac.shape[0], Bc.shape[1]
    E = np.zeros((nx + nu, nx + nu))
    E[:nx, :nx], E[:nx, nx:] = Ac, Bc
    F = scipy.linalg.expm(E * (15.0 / N))
    return F[:nx, :nx], F[:nx, nx:]


def mass_spring(M, N, count, seed=0):
    """(LQProblem batch of `count` initial states, C [N+1, m, nx], D [N, m, nu], bl, bu [N+1, m])."""
    A, B = discretise(M, N)
    nx, nu = A.shape[0], B.shape[1]
    m = M + nu
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 13, M, N, seed]))
    x0 = np.zeros((count, nx))
    x0[:, :M] = rng.uniform(-3.0, 3.0, size=(count, M))
    rep = lambda a, n: np.broadcast_to(a, (count, n) + a.shape).copy()  # noqa: E731
    prob = LQProblem(A=rep(A, N), B=rep(B, N), Q=rep(np.eye(nx), N + 1), R=rep(np.eye(nu), N),
                     q=np.zeros((count, N + 1, nx)), r=np.zeros((count, N, nu)), x0=x0,
                     S=np.zeros((count, N, nu, nx)), f=np.zeros((count, N, nx)),
                     meta={"workload": "mass-spring", "M": M})
    C = np.zeros((N + 1, m, nx))
    C[:, :M, :M] = np.eye(M)
    D = np.zeros((N, m, nu))
    D[:, M:, :] = np.eye(nu)
    bl = np.concatenate([np.full((N + 1, M), -4.0), np.full((N + 1, nu), -0.5)], axis=1)
    bu = -bl
    bl[N, M:], bu[N, M:] = -np.inf, np.inf
    return prob, C, D, bl, bu
