"""Seeded symmetric positive definite block-tridiagonal systems (eq. block-tri): diagonal blocks
M_k = G_k G_k^T + dominance n I, subdiagonal blocks K_k and right-hand sides b_k with N(0, 1)
entries.  Only draws numbers: no solver arithmetic."""
from __future__ import annotations

import numpy as np

from .problems import SEED_ROOT


def random_blocktri(seed: int, batch: int, Nb: int, n: int, dominance: float = 4.0):
    """(M [batch, Nb, n, n], K [batch, Nb-1, n, n], b [batch, Nb, n]) from
    default_rng(SeedSequence([SEED_ROOT, 7, seed]))."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 7, seed]))
    G = rng.standard_normal((batch, Nb, n, n))
    M = G @ np.swapaxes(G, -1, -2) + dominance * n * np.eye(n)
    M = 0.5 * (M + np.swapaxes(M, -1, -2))
    K = rng.standard_normal((batch, max(Nb - 1, 0), n, n))
    b = rng.standard_normal((batch, Nb, n))
    return M, K, b
