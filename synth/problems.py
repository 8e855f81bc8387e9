"""Seeded generators for the five benchmark workloads and for random test problems.

The problem class is the equality-constrained LQ optimal-control problem of the
paper's problem statement (eq. ocp-eq): dynamics x_{k+1} = A_k x_k + B_k u_k + f_k,
stage cost 1/2 [u;x]^T [[R_k, S_k],[S_k^T, Q_k]] [u;x] + [u;x]^T [r_k; q_k],
terminal cost 1/2 x_N^T Q_N x_N + q_N^T x_N, fixed initial state x_init.

Array conventions (row-major, float64):
    A  [N, nx, nx]      k = 0..N-1
    B  [N, nx, nu]      k = 0..N-1
    Q  [N+1, nx, nx]    k = 0..N   (Q_0 only multiplies the fixed x_0: it does not affect the solution)
    R  [N, nu, nu]      k = 0..N-1
    S  [N, nu, nx]      k = 0..N-1, or None for zero
    q  [N+1, nx]        k = 0..N   (q_0 likewise irrelevant)
    r  [N, nu]          k = 0..N-1
    f  [N, nx]          k = 0..N-1, or None for zero
    x0 [nx]

A batch of equally sized instances stacks these along a leading axis.

Seeds: instance i of workload c draws from
``default_rng(SeedSequence([SEED_ROOT, c, 1, i]))``, so any subset of a batch can
be regenerated on its own.  The ragged workload draws its sizes first from
``SeedSequence([SEED_ROOT, 3, 0])``.  Within an instance the draw order is
A (all k), B, M (for Q, k = 0..N), R, q (k = 0..N), r, x0.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_ROOT = 2512090580


@dataclass
class LQProblem:
    """One instance (arrays without batch axis) or a uniform batch (leading axis)."""

    A: np.ndarray
    B: np.ndarray
    Q: np.ndarray
    R: np.ndarray
    q: np.ndarray
    r: np.ndarray
    x0: np.ndarray
    S: Optional[np.ndarray] = None
    f: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def batched(self) -> bool:
        return self.A.ndim == 4

    @property
    def N(self) -> int:
        return self.A.shape[-3]

    @property
    def nx(self) -> int:
        return self.A.shape[-1]

    @property
    def nu(self) -> int:
        return self.B.shape[-1]

    @property
    def batch(self) -> int:
        return self.A.shape[0] if self.batched else 1

    def instance(self, i: int) -> "LQProblem":
        if not self.batched:
            if i != 0:
                raise IndexError(i)
            return self
        g = lambda a: None if a is None else a[i]  # noqa: E731
        return LQProblem(A=self.A[i], B=self.B[i], Q=self.Q[i], R=self.R[i], q=self.q[i],
                         r=self.r[i], x0=self.x0[i], S=g(self.S), f=g(self.f), meta=dict(self.meta))

    def subset(self, idx) -> "LQProblem":
        idx = np.asarray(idx)
        g = lambda a: None if a is None else a[idx]  # noqa: E731
        return LQProblem(A=self.A[idx], B=self.B[idx], Q=self.Q[idx], R=self.R[idx], q=self.q[idx],
                         r=self.r[idx], x0=self.x0[idx], S=g(self.S), f=g(self.f), meta=dict(self.meta))


def stack(insts: List[LQProblem]) -> LQProblem:
    """Stack equally sized instances into a batch."""
    def st(name):
        vals = [getattr(p, name) for p in insts]
        if all(v is None for v in vals):
            return None
        ref = next(v for v in vals if v is not None)
        return np.stack([np.zeros_like(ref) if v is None else v for v in vals])
    return LQProblem(A=st("A"), B=st("B"), Q=st("Q"), R=st("R"), q=st("q"), r=st("r"),
                     x0=st("x0"), S=st("S"), f=st("f"), meta=dict(insts[0].meta))


def _sym(m):
    return 0.5 * (m + np.swapaxes(m, -1, -2))


def _rng(cfg: int, i: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, cfg, 1, i]))


def _haar(rng, n, count):
    """`count` Haar-orthogonal n x n matrices: QR of N(0,1) matrices with the signs of diag(R)
    moved into Q.  The normals are drawn in one call (the same stream as `count` successive
    n x n draws) and factored as a stack (the same LAPACK routine per matrix)."""
    g = rng.standard_normal((count, n, n))
    qm, rm = np.linalg.qr(g)
    return qm * np.sign(np.diagonal(rm, axis1=-2, axis2=-1))[:, None, :]


def config_sizes(cfg: int):
    """(batch, N, nx, nu) of the uniform workloads."""
    return {1: (1, 20, 4, 2), 2: (4096, 50, 12, 4), 4: (64, 1000, 128, 32), 5: (1024, 100, 32, 8)}[cfg]


def _draw(rng, cfg, N, nx, nu, N_override=None):
    eye_x = np.eye(nx)
    if cfg == 1:
        A = eye_x + 0.1 * rng.standard_normal((N, nx, nx))
        B = rng.standard_normal((N, nx, nu))
        M = rng.standard_normal((N + 1, nx, nx))
        Q = _sym(M @ np.swapaxes(M, -1, -2)) + eye_x
        R = np.eye(nu) + 0.1 * np.einsum("ki,ij->kij", rng.uniform(size=(N, nu)), np.eye(nu))
    elif cfg in (2, 3, 5):
        A = eye_x + 0.05 * rng.standard_normal((N, nx, nx))
        B = 0.5 * rng.standard_normal((N, nx, nu))
        M = rng.standard_normal((N + 1, nx, nx))
        Q = _sym(M @ np.swapaxes(M, -1, -2)) + 0.1 * eye_x
        R = 0.1 * np.eye(nu) + np.einsum("ki,ij->kij", rng.uniform(size=(N, nu)), np.eye(nu))
    elif cfg == 4:
        A = 0.99 * _haar(rng, nx, N) + 0.01 * rng.standard_normal((N, nx, nx))
        B = rng.standard_normal((N, nx, nu)) / np.sqrt(nx)
        M = rng.standard_normal((N + 1, nx, nx))
        Q = _sym(M @ np.swapaxes(M, -1, -2)) + eye_x
        R = np.broadcast_to(np.eye(nu), (N, nu, nu)).copy()
    else:
        raise ValueError(f"unknown workload {cfg}")
    q = rng.standard_normal((N + 1, nx))
    r = rng.standard_normal((N, nu))
    x0 = rng.standard_normal(nx)
    return LQProblem(A=A, B=B, Q=Q, R=R, q=q, r=r, x0=x0, meta={"cfg": cfg})


def make_instance(cfg: int, i: int, N=None, nx=None, nu=None) -> LQProblem:
    """Instance i of workload ``cfg`` (sizes may be overridden for reduced tests)."""
    if cfg == 3:
        Ns, nxs, nus = _ragged_sizes(max(i + 1, 2048))
        N0, nx0, nu0 = int(Ns[i]), int(nxs[i]), int(nus[i])
    else:
        _, N0, nx0, nu0 = config_sizes(cfg)
    N = N0 if N is None else N
    nx = nx0 if nx is None else nx
    nu = nu0 if nu is None else nu
    p = _draw(_rng(cfg, i), cfg, N, nx, nu)
    p.meta.update({"index": i})
    return p


def make_batch(cfg: int, batch=None, N=None, nx=None, nu=None, start=0) -> LQProblem:
    """A uniform batch of workload ``cfg`` (instances start..start+batch-1)."""
    b0, N0, nx0, nu0 = config_sizes(cfg)
    batch = b0 if batch is None else batch
    insts = [make_instance(cfg, start + i, N=N or N0, nx=nx or nx0, nu=nu or nu0) for i in range(batch)]
    out = stack(insts)
    out.meta = {"cfg": cfg, "start": start}
    return out


def _instance_worker(args):
    cfg, i, N, nx, nu = args
    p = make_instance(cfg, i, N=N, nx=nx, nu=nu)
    return i, {k: getattr(p, k) for k in ("A", "B", "Q", "R", "q", "r", "x0")}


def make_batch_parallel(cfg: int, batch=None, workers=8, N=None, nx=None, nu=None, progress=None) -> LQProblem:
    """``make_batch`` with the instances drawn in `workers` processes (each instance has its own
    seed, so the result is identical), written into preallocated batch arrays as they arrive;
    for the workloads whose instances take seconds to draw.  progress(done, total) is called
    every few instances."""
    import multiprocessing as mp
    b0, N0, nx0, nu0 = config_sizes(cfg)
    batch = b0 if batch is None else batch
    N, nx, nu = N or N0, nx or nx0, nu or nu0
    shapes = {"A": (N, nx, nx), "B": (N, nx, nu), "Q": (N + 1, nx, nx), "R": (N, nu, nu), "q": (N + 1, nx),
              "r": (N, nu), "x0": (nx,)}
    arrs = {k: np.empty((batch,) + s_) for k, s_ in shapes.items()}
    jobs = [(cfg, i, N, nx, nu) for i in range(batch)]
    done = 0
    # one BLAS thread per worker process (the workers inherit the environment at their start)
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "1" for k in keys})
    try:
        with mp.get_context("spawn").Pool(max(1, min(workers, batch))) as pool:
            for i, d in pool.imap_unordered(_instance_worker, jobs):
                for k, v in d.items():
                    arrs[k][i] = v
                done += 1
                if progress and (done % 8 == 0 or done == batch):
                    progress(done, batch)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    out = LQProblem(**arrs)
    out.meta = {"cfg": cfg, "start": 0}
    return out


def _ragged_sizes(batch: int):
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 3, 0]))
    nx = rng.integers(6, 65, size=batch)
    nu = rng.integers(2, 17, size=batch)
    N = rng.integers(10, 201, size=batch)
    return N, nx, nu


def make_ragged(batch: int = 2048, idx=None) -> List[LQProblem]:
    """The uneven workload: nx ~ U{6..64}, nu ~ U{2..16}, N ~ U{10..200}, config-2 generators."""
    Ns, nxs, nus = _ragged_sizes(max(batch, 2048))
    idx = range(batch) if idx is None else idx
    out = []
    for i in idx:
        p = _draw(_rng(3, int(i)), 3, int(Ns[i]), int(nxs[i]), int(nus[i]))
        p.meta.update({"index": int(i)})
        out.append(p)
    return out


def random_problem(seed: int, N: int, nx: int, nu: int, with_S=True, with_f=True, batch=None,
                   scale_q=1.0) -> LQProblem:
    """A general random instance (or batch) with nonzero S and f, for tests.

    The stage Hessians [[R, S],[S^T, Q]] are made positive definite by drawing a
    full (nu+nx)-square factor and adding a multiple of the identity.
    """
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 99, seed]))
    shape = () if batch is None else (batch,)
    nux = nu + nx
    A = np.eye(nx) + 0.3 * rng.standard_normal(shape + (N, nx, nx))
    B = rng.standard_normal(shape + (N, nx, nu))
    W = rng.standard_normal(shape + (N + 1, nux, nux))
    H = _sym(W @ np.swapaxes(W, -1, -2)) / nux + 0.5 * np.eye(nux)
    R = H[..., :N, :nu, :nu].copy()
    S = H[..., :N, :nu, nu:].copy() if with_S else None
    Q = H[..., :, nu:, nu:].copy()
    q = scale_q * rng.standard_normal(shape + (N + 1, nx))
    r = rng.standard_normal(shape + (N, nu))
    f = rng.standard_normal(shape + (N, nx)) if with_f else None
    x0 = rng.standard_normal(shape + (nx,))
    return LQProblem(A=A, B=B, Q=Q, R=R, q=q, r=r, x0=x0, S=S, f=f, meta={"seed": seed})
