"""Seeded constraint rows and penalty changes for factorisation updates (the changes of the
active-set penalties of eq. low-rank-update-Hj).  Only draws numbers: no solver arithmetic.

Per instance and stage j there are m rows (D_j u_j + C_j x_j).  With ``box`` each row is a bound
on one variable of the stage, as in the box-constrained problems of the paper's experiments: a
unit row e_i of C_j (a state bound) or of D_j (an input bound), the variable drawn uniformly from
the stage's nx + nu (the terminal stage from its nx states); otherwise the rows have N(0, 1)
entries.  Each row's penalty change is nonzero with probability ``density``, drawn uniformly from
``sigma``; zero rows leave the stage unchanged.
"""
from __future__ import annotations

import numpy as np

from .problems import SEED_ROOT


def random_update_rows(seed: int, batch: int, N: int, nx: int, nu: int, m: int, density: float = 0.5,
                       sigma=(0.5, 2.0), box: bool = True):
    """(C [batch, N+1, m, nx], D [batch, N, m, nu], dsig [batch, N+1, m]) from
    default_rng(SeedSequence([SEED_ROOT, 11, seed]))."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 11, seed]))
    C = np.zeros((batch, N + 1, m, nx))
    D = np.zeros((batch, N, m, nu))
    if box:
        pick = rng.integers(0, nx + nu, size=(batch, N + 1, m))
        pick[:, N] = nu + rng.integers(0, nx, size=(batch, m))
        b, j, i = np.nonzero(pick >= nu)
        C[b, j, i, pick[b, j, i] - nu] = 1.0
        b, j, i = np.nonzero(pick[:, :N] < nu)
        D[b, j, i, pick[b, j, i]] = 1.0
    else:
        C[:] = rng.standard_normal(C.shape)
        D[:] = rng.standard_normal(D.shape)
    on = rng.uniform(size=(batch, N + 1, m)) < density
    dsig = np.where(on, rng.uniform(sigma[0], sigma[1], size=(batch, N + 1, m)), 0.0)
    return C, D, dsig
