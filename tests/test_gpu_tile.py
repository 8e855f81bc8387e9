"""Parity of the matrix-core tile factor kernel with the oracle (float64 and mixed precision).

Bar: as the other parity tests, rel_res <= 1e-10 from the library and from the oracle's residual,
forward error against the oracle's direct solve <= 1e-9; the stored factors against chol(P_k),
chol(R_k + B^T P B) and L^S from the textbook recursion to 1e-12 relative (float64).  Shapes
cover one to ten tile columns, ragged tiles (nx, nu not multiples of 16), several input tiles,
S and f, and the workloads' full sizes (sampled instances).
"""
import numpy as np
import pytest

import synth
from oracle import kkt, riccati

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from gpu_util import forward_error, instance_solution, oracle_solution, run  # noqa: E402

# (N, nx, nu): tile columns T = ceil(nx/16) + ceil(nu/16) from 2 to 10
SHAPES = [(3, 5, 3), (4, 16, 16), (5, 17, 1), (4, 32, 8), (3, 40, 20), (3, 64, 16), (2, 33, 64), (3, 128, 32),
          (2, 100, 40)]


def _plan(insts, mode, variant="tile"):
    plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode=mode)
    plan.set_variant(variant)
    return plan


def _check(res, tol_fwd=1e-9, sample=None):
    insts = res["insts"]
    assert np.all(res["info"] == 0), res["info"]
    assert res["rel"].max() <= 1e-10, res["rel"].max()
    for i in (range(len(insts)) if sample is None else sample):
        sol = instance_solution(res, i)
        assert kkt.residual(insts[i], *sol)[1] <= 1e-10, i
        assert forward_error(sol, oracle_solution(insts[i])) <= tol_fwd, i


def _well_conditioned(seed, N, nx, nu):
    """random_problem's stage data with stable dynamics (spectral radius < 1), so that the KKT
    systems of the larger shapes stay well conditioned."""
    p = synth.random_problem(seed, N, nx, nu)
    rng = np.random.default_rng(seed)
    p.A = 0.9 * np.linalg.qr(rng.standard_normal((N, nx, nx)))[0] + 0.05 * rng.standard_normal((N, nx, nx))
    p.B = p.B / np.sqrt(nx)
    return p


@pytest.mark.parametrize("N,nx,nu", SHAPES)
@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 8), ("mixed_bf16", 40)])
def test_tile_matches_oracle(N, nx, nu, mode, max_it):
    print(f"case: tile N={N} nx={nx} nu={nu} {mode}", flush=True)
    insts = [_well_conditioned(300 + i, N, nx, nu) for i in range(3)]
    res = run(insts, mode, max_it=max_it, plan=_plan(insts, mode))
    assert res["plan"].variant == "tile"
    _check(res)


def test_tile_factors_match_oracle_cost_to_go():
    p = _well_conditioned(41, 5, 21, 18)  # two input tiles, two state tiles, ragged both
    print("case: tile factors", flush=True)
    res = run([p], "f64", plan=_plan([p], "f64"))
    ws = res["ws"].cpu().numpy().view(np.float64)
    nx, nu, N = p.nx, p.nu, p.N
    fs = nu * (nu + 1) // 2 + nu + nx * nu + nx * (nx + 1) // 2 + nx
    LQ, LR, LS = riccati.reference_factors(p)

    def tri(v, n):
        M = np.zeros((n, n))
        M[np.tril_indices(n)] = v
        return M

    for k in range(N + 1):
        blk = ws[k * fs:(k + 1) * fs]
        o = 0
        Lr = tri(blk[o:o + nu * (nu + 1) // 2], nu); o += nu * (nu + 1) // 2
        dR = blk[o:o + nu]; o += nu
        Ls = blk[o:o + nx * nu].reshape(nx, nu); o += nx * nu
        Lq = tri(blk[o:o + nx * (nx + 1) // 2], nx); o += nx * (nx + 1) // 2
        dQ = blk[o:o + nx]
        if k >= 1:
            np.testing.assert_allclose(Lq, LQ[k], rtol=0, atol=1e-12 * np.abs(LQ[k]).max())
            np.testing.assert_allclose(dQ, 1 / np.diag(LQ[k]), rtol=1e-13)
        if k < N:
            np.testing.assert_allclose(Lr, LR[k], rtol=0, atol=1e-12 * np.abs(LR[k]).max())
            np.testing.assert_allclose(Ls, LS[k], rtol=0, atol=1e-12 * max(1, np.abs(LS[k]).max()))
            np.testing.assert_allclose(dR, 1 / np.diag(LR[k]), rtol=1e-13)


@pytest.mark.parametrize("mode", ["f64", "mixed_f32"])
def test_tile_and_generic_agree_on_ragged_batch(mode):
    """A ragged batch of mixed tile counts through both kernels (persistent grid)."""
    insts = [_well_conditioned(500 + i, 3 + i % 4, nx, nu)
             for i, (nx, nu) in enumerate([(6, 2), (31, 9), (47, 16), (64, 3), (12, 14), (50, 30)])]
    print(f"case: tile vs generic ragged {mode}", flush=True)
    mi = 0 if mode == "f64" else 8
    rt = run(insts, mode, max_it=mi, plan=_plan(insts, mode, "tile"))
    rg = run(insts, mode, max_it=mi, plan=_plan(insts, mode, "generic"))
    _check(rt)
    for i in range(len(insts)):
        assert forward_error(instance_solution(rt, i), instance_solution(rg, i)) <= 1e-10, i


def test_tile_indefinite_and_nonfinite_report_info():
    p = _well_conditioned(61, 6, 20, 5)
    p.R[3] = -np.eye(5) * 50.0            # stage 3 not positive definite
    q = _well_conditioned(62, 6, 20, 5)
    q.A[2, 1, 1] = np.nan                 # non-finite data
    r = _well_conditioned(63, 6, 20, 5)
    print("case: tile info codes", flush=True)
    res = run([p, q, r], "f64", max_it=0, plan=_plan([p, q, r], "f64"))
    assert res["info"][0] == 4
    assert res["info"][1] == -1
    assert res["info"][2] == 0


@pytest.mark.parametrize("variant,ckpt", [("tile", 0), ("tile", 2), ("generic", 0)])
def test_solve_without_certificate(variant, ckpt):
    """opts.check = 0 with max_it = 0: the residual is not formed, rel_res reads NaN, info stays 0,
    and x, u, lam are the certified solve's bit for bit (stored and checkpointed tile factors, and
    the generic kernels, which skipped it already)."""
    insts = [_well_conditioned(640 + i, 9, 24, 6) for i in range(3)]
    out = []
    for check in (True, False):
        print(f"case: {variant} ckpt={ckpt} check={check}", flush=True)
        plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode="f64",
                      ckpt_stride=ckpt)
        plan.set_variant(variant)
        out.append(run(insts, "f64", max_it=0, check=check, plan=plan))
    on, off = out
    assert np.all(on["info"] == 0) and np.all(off["info"] == 0), (on["info"], off["info"])
    assert on["rel"].max() <= 1e-10 and np.all(np.isnan(off["rel"])), (on["rel"], off["rel"])
    for key in ("x", "u", "lam"):
        assert on[key].cpu().numpy().tobytes() == off[key].cpu().numpy().tobytes(), key
    for i in range(len(insts)):
        assert forward_error(instance_solution(off, i), oracle_solution(insts[i])) <= 1e-9, i


def test_tile_adjoint_consumes_tile_factors():
    """lq_solve_backward on tile factors: gradients vs the oracle's dense adjoint."""
    from oracle import adjoint
    from paper_2512_09058_amd.autograd import lq_solve
    b = synth.make_batch(5, batch=2, N=12)
    print("case: tile adjoint", flush=True)
    t = {k: torch.tensor(getattr(b, k), dtype=torch.float64, device="cuda", requires_grad=True)
         for k in ("A", "B", "Q", "R", "q", "r", "x0")}
    x, u, _ = lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"], variant="tile")
    (0.5 * (x.pow(2).sum() + u.pow(2).sum())).backward()
    for i in range(b.batch):
        p = b.instance(i)
        xo, uo, _ = kkt.solve_dense(p)
        _, gx, gu = adjoint.quad_loss(xo, uo)
        ref, _, _ = adjoint.adjoint_grad(p, gx, gu)
        for k in ("A", "B", "Q", "R", "q", "r", "x0"):
            g = t[k].grad[i].cpu().numpy()
            assert np.abs(g - ref[k]).max() <= 1e-8 * max(1.0, np.abs(ref[k]).max()), (i, k)


def test_adjoint_workload_full_size_sampled():
    """Workload 5 at its full size (1024 instances, N = 100, nx = 32, nu = 8) through the tile
    kernel: library residual for every instance, the oracle on a sample."""
    b = synth.make_batch(5)
    print("case: workload 5 full size, tile", flush=True)
    for mode, mi in (("f64", 0), ("mixed_f32", 8)):
        plan = L.Plan(b.N, b.nx, b.nu, batch=b.batch, mode=mode)
        assert plan.variant == "tile"
        res = run(b, mode, max_it=mi, plan=plan)
        _check(res, sample=[0, 511, 1023])


def test_large_workload_full_size_sampled():
    """Workload 4 at its full size (64 distinct instances, N = 1000, nx = 128, nu = 32, drawn in
    up to sixteen processes): float64 and mixed, residual of every instance, oracle (textbook Riccati)
    on a sample."""
    import os
    b = synth.make_batch_parallel(4, workers=min(16, os.cpu_count() or 1),
                                  progress=lambda d, t: print(f"  drawn {d}/{t} instances", flush=True))
    assert b.batch == 64 and len({float(b.A[i, 0, 0, 0]) for i in range(64)}) == 64
    insts = [b.instance(i) for i in range(64)]
    print("case: workload 4 full size, tile", flush=True)
    for mode, mi in (("f64", 0), ("mixed_f32", 8), ("mixed_bf16", 30)):
        res = run(b, mode, max_it=mi, plan=L.Plan(b.N, b.nx, b.nu, batch=64, mode=mode))
        assert res["plan"].variant == "tile"
        res["insts"] = insts
        _check(res, sample=[0, 1, 63])


def test_bf16_plans_only_where_the_tile_kernel_runs():
    """The bf16 mode exists only on the matrix-core tile kernels (checkpointed ones included):
    shapes they do not take are refused instead of silently running float32 products."""
    assert L.Plan(20, 12, 4, batch=2, mode="mixed_bf16", ckpt_stride=5).variant == "tile"
    with pytest.raises(RuntimeError, match="status -2"):
        L.Plan(20, 100, 40, batch=2, mode="mixed_bf16", ckpt_stride=5)
    with pytest.raises(RuntimeError, match="status -2"):
        L.Plan(20, 170, 4, batch=2, mode="mixed_bf16")
    plan = L.Plan(20, 12, 4, batch=2, mode="mixed_bf16")
    assert plan.variant == "tile"
    with pytest.raises(RuntimeError, match="status -2"):
        plan.set_variant("generic")
