"""The library's own numbers against the oracle, element by element.

* The float64 KKT residual that drives refinement (eq. opt-cond-ocp-eq, rho = b - K z): the
  library's rel_res and the residual blocks it stores for the correction sweep (rho_u, rho_x and
  -rho_lambda, in each kernel variant's sign convention) against `kkt.residual` of the same
  iterate.  The iterate is the first forward pass (max_it = 1 with tol = 1e30: the residual is
  computed and stored, no correction follows), so in mixed mode it is the unrefined iterate whose
  residual is ~1e-6 ||b||: a dropped or mis-scaled row block would show far above the bar.
  Bar: |rho_lib - rho_oracle| <= 1e-12 ||b||_inf per entry, |rel_lib - rel_oracle| <= 1e-12.
* The stored factors L^R_k, L^S_k, L^Q_k against the textbook recursion's chol(R_k + B_k^T P B_k),
  L^S_k and chol(P_k) (Alg. "factor-block-column-riccati", eq. riccati-recursion-P): relative to
  the matrix's largest entry, <= 1e-12 in float64 and <= 1e-4 with float32 stage products
  (float32 storage).
* x, u, lambda entry by entry: |a_i - b_i| <= rtol |b_i| + atol ||b||_inf (float64: 1e-9 / 1e-11;
  mixed refined to 1e-10: 1e-7 / 1e-9), beside the normwise forward error.
* Q_k and R_k that are not symmetric through the size-specialised kernels (only their symmetric
  parts enter the KKT system).
* The adjoint workload at full size in its reported configuration (1024 x N = 100, nx = 32,
  nu = 8, mixed float32, factors checkpointed every 10 stages): gradients of sampled instances
  against the oracle's adjoint gradient (banded solves), <= 1e-7 relative per array.
"""
import numpy as np
import pytest

import synth
from oracle import adjoint, kkt, riccati

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from gpu_util import (elementwise_ok, forward_error, instance_solution, oracle_solution, run,  # noqa: E402
                      unpack_factor_block, workspace_views)


def _plan(b, mode, variant):
    plan = L.Plan(b.N, b.nx, b.nu, batch=b.batch, mode=mode)
    plan.set_variant(variant)
    assert plan.variant == variant
    return plan


def _oracle_blocks(p, x, u, lam):
    rho, rel = kkt.residual(p, x, u, lam)
    _, bvec, lay = kkt.assemble(p)
    ru = np.stack([rho[lay.u(k)] for k in range(p.N)])
    rx = np.stack([rho[lay.x(k)] for k in range(1, p.N + 1)])
    rl = np.stack([rho[lay.lam(k)] for k in range(p.N)])
    return ru, rx, rl, rel, np.abs(bvec).max()


CASES = [("small", 12, 4), ("small", 6, 2), ("tile", 12, 4), ("tile", 20, 5), ("generic", 12, 4),
         ("generic", 20, 5)]


@pytest.mark.parametrize("variant,nx,nu", CASES)
@pytest.mark.parametrize("mode", ["f64", "mixed_f32"])
def test_library_residual_is_the_oracle_residual_of_the_same_iterate(variant, nx, nu, mode):
    print(f"case: residual blocks {variant} nx={nx} nu={nu} {mode}", flush=True)
    b = synth.random_problem(700 + nx + nu, 9, nx, nu, batch=5)  # S and f nonzero
    res = run(b, mode, tol=1e30, max_it=1, plan=_plan(b, mode, variant))
    assert np.all(res["info"] == 0) and np.all(res["iters"] == 0)
    views = workspace_views(res)
    for i in range(b.batch):
        p = b.instance(i)
        ru, rx, rl, rel_o, nb = _oracle_blocks(p, *instance_solution(res, i))
        if mode == "mixed_f32":
            assert rel_o > 1e-9, rel_o  # the unrefined iterate: a residual well above rounding
        assert abs(res["rel"][i] - rel_o) <= 1e-12, (i, res["rel"][i], rel_o)
        st = views[i][1]
        # every variant stores the dynamics residual as the correction's f = -rho_lambda
        assert np.abs(st["flam"] + rl).max() <= 1e-12 * nb, i
        if variant == "generic":
            continue  # the generic kernel sweeps rho_u, rho_x on the fly and stores neither
        sgn = 1.0 if variant == "small" else -1.0  # tile: stored as the correction's r, q = -rho
        assert np.abs(sgn * st["rho_u"] - ru).max() <= 1e-12 * nb, i
        assert np.abs(sgn * st["rho_x"][1:] - rx).max() <= 1e-12 * nb, i


def _check_factors(res, insts, bound):
    views = workspace_views(res)
    worst = 0.0
    for i, p in enumerate(insts):
        LQ, LR, LS = riccati.reference_factors(p)
        blocks = views[i][0]
        for k in range(p.N + 1):
            Lr, dR, Ls, Lq, dQ = unpack_factor_block(blocks[k], p.nx, p.nu)
            errs = []
            if k >= 1:
                errs.append(np.abs(Lq - LQ[k]).max() / np.abs(LQ[k]).max())
                errs.append(np.abs(dQ * np.diag(LQ[k]) - 1).max())
            if k < p.N:
                errs.append(np.abs(Lr - LR[k]).max() / np.abs(LR[k]).max())
                errs.append(np.abs(Ls - LS[k]).max() / max(1.0, np.abs(LS[k]).max()))
                errs.append(np.abs(dR * np.diag(LR[k]) - 1).max())
            worst = max(worst, max(errs))
    print(f"  worst factor error {worst:.2e} (bound {bound:.0e})", flush=True)
    assert worst <= bound


@pytest.mark.parametrize("nx,nu", [(12, 4), (4, 2), (10, 6)])
@pytest.mark.parametrize("mode,bound", [("f64", 1e-12), ("mixed_f32", 1e-4)])
def test_small_kernel_factors_match_oracle(nx, nu, mode, bound):
    print(f"case: small factors nx={nx} nu={nu} {mode}", flush=True)
    b = synth.random_problem(810 + nx, 7, nx, nu, batch=5)
    res = run(b, mode, max_it=0 if mode == "f64" else 8, plan=_plan(b, mode, "small"))
    _check_factors(res, [b.instance(i) for i in range(b.batch)], bound)


def test_small_kernel_factors_workload2_instances():
    print("case: small factors, workload-2 generators, f64 and mixed", flush=True)
    b = synth.make_batch(2, batch=6, N=20)
    for mode, bound in (("f64", 1e-12), ("mixed_f32", 1e-4)):
        res = run(b, mode, max_it=0 if mode == "f64" else 8, plan=_plan(b, mode, "small"))
        _check_factors(res, [b.instance(i) for i in range(b.batch)], bound)


@pytest.mark.parametrize("nx,nu", [(21, 18), (40, 8)])
def test_tile_kernel_mixed_factors_match_oracle(nx, nu):
    print(f"case: tile factors mixed nx={nx} nu={nu}", flush=True)
    b = synth.make_batch(5, batch=3, N=8, nx=nx, nu=nu)
    res = run(b, "mixed_f32", max_it=8, plan=_plan(b, "mixed_f32", "tile"))
    _check_factors(res, [b.instance(i) for i in range(b.batch)], 1e-4)


@pytest.mark.parametrize("variant,nx,nu", [("small", 12, 4), ("tile", 20, 5), ("generic", 20, 5)])
@pytest.mark.parametrize("mode", ["f64", "mixed_f32"])
def test_solution_entrywise(variant, nx, nu, mode):
    print(f"case: entrywise {variant} nx={nx} nu={nu} {mode}", flush=True)
    b = synth.random_problem(900 + nx, 12, nx, nu, batch=4)
    res = run(b, mode, max_it=0 if mode == "f64" else 10, plan=_plan(b, mode, variant))
    assert np.all(res["info"] == 0)
    rtol, atol = (1e-9, 1e-11) if mode == "f64" else (1e-7, 1e-9)
    for i in range(b.batch):
        sol, ref = instance_solution(res, i), oracle_solution(b.instance(i))
        assert forward_error(sol, ref) <= 1e-9
        w = elementwise_ok(sol, ref, rtol, atol)
        assert w <= 1.0, (i, w)


@pytest.mark.parametrize("nx,nu", [(12, 4), (8, 4), (6, 2)])
@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 8)])
def test_nonsymmetric_Q_R_through_small_kernel(nx, nu, mode, max_it):
    """Only the symmetric parts of Q_k and R_k enter the KKT system: adding antisymmetric parts
    leaves the solution and the factors unchanged."""
    print(f"case: nonsymmetric Q, R small nx={nx} nu={nu} {mode}", flush=True)
    b = synth.random_problem(950 + nx, 10, nx, nu, batch=5)
    rng = np.random.default_rng(17)
    WQ = rng.standard_normal(b.Q.shape)
    WR = rng.standard_normal(b.R.shape)
    b.Q = b.Q + 0.4 * (WQ - np.swapaxes(WQ, -1, -2))
    b.R = b.R + 0.4 * (WR - np.swapaxes(WR, -1, -2))
    assert np.abs(b.Q - np.swapaxes(b.Q, -1, -2)).max() > 0.1
    res = run(b, mode, max_it=max_it, plan=_plan(b, mode, "small"))
    assert np.all(res["info"] == 0)
    assert res["rel"].max() <= 1e-10
    for i in range(b.batch):
        p = b.instance(i)
        sol = instance_solution(res, i)
        assert kkt.residual(p, *sol)[1] <= 1e-10
        assert forward_error(sol, kkt.solve_dense(p)) <= 1e-9
    _check_factors(res, [b.instance(i) for i in range(b.batch)], 1e-12 if mode == "f64" else 1e-4)


def test_adjoint_workload_full_size_checkpointed_mixed_gradients():
    """Workload 5 as reported (1024 x N = 100, nx = 32, nu = 8, mixed float32, checkpoints every
    10 stages) through the autograd function; sampled instances' gradients of the loss
    1/2 sum ||x_k||^2 + ||u_k||^2 against the oracle's adjoint gradient."""
    from paper_2512_09058_amd.autograd import lq_solve
    b = synth.make_batch(5)
    assert b.batch == 1024 and b.N == 100
    print("case: workload 5 full size, mixed, ckpt 10, gradients", flush=True)
    names = ("A", "B", "Q", "R", "q", "r", "x0")
    t = {k: torch.tensor(np.ascontiguousarray(getattr(b, k)), dtype=torch.float64, device="cuda",
                         requires_grad=True) for k in names}
    x, u, _ = lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"], mode="mixed_f32",
                       ckpt_stride=10)
    (0.5 * (x.pow(2).sum() + u.pow(2).sum())).backward()
    torch.cuda.synchronize()
    for i in (0, 511, 1023):
        p = b.instance(i)
        xo, uo, _ = riccati.solve(p)
        _, gx, gu = adjoint.quad_loss(xo, uo)
        ref, _, _ = adjoint.adjoint_grad_banded(p, gx, gu)
        for k in names:
            g = t[k].grad[i].cpu().numpy()
            err = np.abs(g - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300)
            assert err <= 1e-7, (i, k, err)


def test_autograd_raises_on_failed_instances():
    """A non-finite input, a stage that is not positive definite and refinement stopped above tol
    each raise through the autograd function; check=False returns without reading the status."""
    from paper_2512_09058_amd.autograd import SolveError, last_status, lq_solve
    print("case: autograd failure statuses", flush=True)

    def tensors(b):
        return {k: torch.tensor(np.ascontiguousarray(getattr(b, k)), dtype=torch.float64, device="cuda",
                                requires_grad=True) for k in ("A", "B", "Q", "R", "q", "r", "x0")}

    b = synth.make_batch(2, batch=3, N=8)
    b.A[1, 2, 0, 0] = np.nan
    t = tensors(b)
    with pytest.raises(SolveError, match="instance 1: info=-1"):
        lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"])
    lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"], check=False)
    torch.cuda.synchronize()
    assert last_status["forward"][0].cpu().tolist() == [0, -1, 0]

    b = synth.make_batch(2, batch=3, N=8)
    b.R[2, 3] = -1e4 * np.eye(4)  # far below -B^T P B: the first pivot of stage 3 is negative
    t = tensors(b)
    with pytest.raises(SolveError, match="instance 2: info=4"):
        lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"])

    b = synth.make_batch(2, batch=3, N=8)
    t = tensors(b)
    with pytest.raises(SolveError, match="info=-2"):
        lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"], mode="mixed_f32", tol=1e-30,
                 max_it=1)


@pytest.mark.parametrize("variant,nx,nu", [("small", 12, 4), ("tile", 12, 4), ("generic", 12, 4), ("tile", 20, 5)])
@pytest.mark.parametrize("mode", ["f64", "mixed_f32"])
def test_first_failing_pivot_classifies_the_stage(variant, nx, nu, mode):
    """A stage matrix that is not positive definite reports k+1 in every variant, also when the
    unit pivot substituted for the failing one makes later pivots of the same stage overflow
    (R_3 = -1e4 I: the first pivot of stage 3 is finite and negative)."""
    print(f"case: indefinite stage 3 {variant} nx={nx} nu={nu} {mode}", flush=True)
    b = synth.make_batch(2, batch=3, N=8, nx=nx, nu=nu)
    b.R[1, 3] = -1e4 * np.eye(nu)
    res = run(b, mode, max_it=0 if mode == "f64" else 3, plan=_plan(b, mode, variant))
    assert res["info"].tolist() == [0, 4, 0], res["info"]
