"""Parallel-in-time solve (interval recursions, Schur complement of the boundary multipliers,
cyclic reduction, interval sweeps) against the CPU oracle.  The method reaches the same unique
KKT solution as every other route (eq. opt-cond-ocp-eq), so the oracle is the dense / banded /
textbook solve.

Bar: the library's float64 rel_res and the oracle's residual of the GPU solution <= 1e-10;
forward error against the oracle <= 1e-9 (random and workload-1/2 shapes) or <= 1e-7 (the large
workload, condition number ~1e6); edge cases P = 1, P = N, N = 1, intervals of unequal length,
S and f nonzero, nx above one 64-column panel; the stage and Schur status codes."""
import numpy as np
import pytest

import synth
from oracle import kkt, riccati

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from paper_2512_09058_amd import pit  # noqa: E402
from gpu_util import forward_error, oracle_solution  # noqa: E402


def run_pit(b, P):
    plan = pit.PitPlan(b.batch, b.N, b.nx, b.nu, P)
    data = L.pack(b)
    ws = plan.workspace()
    info = torch.full((b.batch,), 99, dtype=torch.int32, device="cuda")
    rel = torch.full((b.batch,), -1.0, dtype=torch.float64, device="cuda")
    x, u, lam = plan.empty_outputs()
    pit.factor(plan, data, ws, info)
    pit.solve(plan, data, ws, x, u, lam, rel, info)
    torch.cuda.synchronize()
    N, nx, nu = b.N, b.nx, b.nu
    xs = x.view(b.batch, N, nx).cpu().numpy()
    us = u.view(b.batch, N, nu).cpu().numpy()
    ls = lam.view(b.batch, N, nx).cpu().numpy()
    return xs, us, ls, rel.cpu().numpy(), info.cpu().numpy()


def check_batch(b, P, tol_fwd=1e-9, sample=None):
    xs, us, ls, rel, info = run_pit(b, P)
    assert np.all(info == 0), info
    assert rel.max() <= 1e-10, rel.max()
    for i in (range(b.batch) if sample is None else sample):
        p = b.instance(i)
        sol = (xs[i], us[i], ls[i])
        assert kkt.residual(p, *sol)[1] <= 1e-10, i
        assert forward_error(sol, oracle_solution(p)) <= tol_fwd, i


def _stable(b, seed):
    """random_problem's batch with stable dynamics (0.9 orthogonal + 0.05 G, B / sqrt(nx)): at
    nx = 70 the generator's I + 0.3 G grows ~3.5x per stage, and even the oracle's dense LU solve
    of such an instance stays above a 1e-10 residual."""
    rng = np.random.default_rng(seed)
    shp = b.A.shape
    b.A = 0.9 * np.linalg.qr(rng.standard_normal(shp))[0] + 0.05 * rng.standard_normal(shp)
    b.B = b.B / np.sqrt(b.nx)
    return b


@pytest.mark.parametrize("N,nx,nu,P", [(1, 3, 2, 1), (2, 2, 1, 2), (5, 4, 3, 1), (5, 4, 3, 2), (5, 4, 3, 5),
                                       (12, 6, 3, 4), (17, 5, 2, 3), (16, 12, 4, 8), (9, 70, 7, 3), (7, 20, 66, 2)])
def test_random_with_S_and_f(N, nx, nu, P):
    print(f"case: pit random N={N} nx={nx} nu={nu} P={P}", flush=True)
    b = synth.random_problem(1200 + N + nx + nu + P, N, nx, nu, batch=3)
    if nx > 64:
        b = _stable(b, N + nx)
    check_batch(b, P)


@pytest.mark.parametrize("P", [1, 2, 4, 5, 10, 20])
def test_workload1_every_interval_count(P):
    print(f"case: pit workload 1 P={P}", flush=True)
    b = synth.make_batch(1)
    check_batch(b, P)


@pytest.mark.parametrize("P", [4, 7, 16])
def test_workload2_shape(P):
    print(f"case: pit workload 2 batch 32 P={P}", flush=True)
    check_batch(synth.make_batch(2, batch=32), P, sample=[0, 31])


def test_one_interval_matches_the_serial_path():
    """P = 1: one interval holding every stage, the wrap stage's coupling as the only boundary:
    the same solution as the serial factorised recursion to rounding."""
    b = synth.random_problem(77, 9, 6, 3, batch=4)
    xs, us, ls, rel, info = run_pit(b, 1)
    from gpu_util import instance_solution, run
    ref = run(b, "f64")
    for i in range(b.batch):
        assert forward_error((xs[i], us[i], ls[i]), instance_solution(ref, i)) <= 1e-12


def test_large_workload_full_size_sampled():
    """Workload 4 at full size (64 distinct instances, N = 1000, nx = 128, nu = 32) split into 8
    intervals per instance (512 workgroups): every instance's library residual, the oracle on a
    sample."""
    import os
    b = synth.make_batch_parallel(4, workers=min(16, os.cpu_count() or 1),
                                  progress=lambda d, t: print(f"  drawn {d}/{t} instances", flush=True))
    print("case: pit workload 4 full size P=8", flush=True)
    check_batch(b, 8, tol_fwd=1e-7, sample=[0, 37, 63])


def test_status_codes():
    b = synth.make_batch(2, batch=3, N=12)
    b.R[1, 5] = -1e4 * np.eye(4)  # stage 5 not positive definite
    b.A[2, 3, 0, 0] = np.nan       # non-finite data
    _, _, _, rel, info = run_pit(b, 3)
    assert info[0] == 0 and info[1] == 5 and info[2] != 0
    assert rel[0] <= 1e-10 and not np.isfinite(rel[2])


def test_rejects_bad_sizes():
    with pytest.raises(ValueError):
        pit.PitPlan(2, 4, 3, 2, 5)   # P > N
    plan = pit.PitPlan(1, 4, 300, 2, 2)  # nx above the kernels' limit: refused by the call
    data = {k: torch.zeros(4, dtype=torch.float64, device="cuda") for k in ("A", "B", "Q", "R", "q", "r", "x0")}
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="status -2"):
        pit.factor(plan, data, torch.empty(256, dtype=torch.uint8, device="cuda"), info)
