"""Uniform batches with nx + nu <= 16 whose shape has no size-specialised kernel of its own run
padded to the smallest compiled shape that covers it (extra states and inputs with identity cost
and no coupling).  The padded problem's solution restricted to the original unknowns is the
original solution, so the bars are those of every other variant: the oracle's dense KKT solve,
the oracle's residual, agreement with the tile variant to rounding, the factor blocks in the shared
layout against the tile variant's, and gradients through the adjoint."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from paper_2512_09058_amd import update as U  # noqa: E402
from paper_2512_09058_amd.autograd import lq_solve  # noqa: E402
from gpu_util import forward_error, instance_solution, oracle_solution, run  # noqa: E402
from oracle import kkt  # noqa: E402

# (nx, nu) without a compiled shape of their own, and the shape each is padded to
SHAPES = [(11, 4), (12, 3), (5, 3), (3, 1), (9, 6), (2, 13), (14, 1), (7, 7)]


def _plan(b, mode, variant=None):
    plan = L.Plan(b.N, b.nx, b.nu, batch=b.batch, mode=mode)
    if variant:
        plan.set_variant(variant)
    return plan


@pytest.mark.parametrize("nx,nu", SHAPES)
@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 6)])
def test_padded_matches_oracle_and_tile(nx, nu, mode, max_it):
    print(f"case: small_padded nx={nx} nu={nu} {mode}", flush=True)
    b = synth.random_problem(300 + 16 * nx + nu, 13, nx, nu, batch=6)
    res = run(b, mode, max_it=max_it, plan=_plan(b, mode))
    assert res["plan"].variant == "small_padded"
    assert np.all(res["info"] == 0) and res["rel"].max() <= 1e-10, (res["info"], res["rel"])
    tile = run(b, mode, max_it=max_it, plan=_plan(b, mode, "tile"))
    for i in range(b.batch):
        sol = instance_solution(res, i)
        p = b.instance(i)
        _, rel_o = kkt.residual(p, *sol)
        assert rel_o <= 1e-10, (i, rel_o)
        assert forward_error(sol, oracle_solution(p)) <= 1e-9, i
        assert forward_error(sol, instance_solution(tile, i)) <= (1e-11 if mode == "f64" else 1e-9), i


@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 6)])
def test_padded_without_S_and_f_headline_generator(mode, max_it):
    """The batch-4096 generator (S = 0, f = 0 passed as NULL) at nx = 11, nu = 4."""
    print(f"case: small_padded headline generator {mode}", flush=True)
    b = synth.make_batch(2, batch=64, N=20, nx=11, nu=4)
    res = run(b, mode, max_it=max_it, plan=_plan(b, mode))
    assert res["plan"].variant == "small_padded"
    assert np.all(res["info"] == 0) and res["rel"].max() <= 1e-10
    for i in (0, 17, 63):
        sol = instance_solution(res, i)
        assert forward_error(sol, oracle_solution(b.instance(i))) <= 1e-9, i


@pytest.mark.parametrize("mode", ["f64", "mixed_f32"])
def test_padded_factor_blocks_in_shared_layout(mode):
    """lq_factor leaves the factor blocks in the layout every variant writes: equal to the tile
    variant's to rounding (stage 0 has no L^Q part, stage N no L^R, L^S part)."""
    print(f"case: small_padded factor blocks {mode}", flush=True)
    nx, nu, N = 11, 4, 9
    b = synth.random_problem(5, N, nx, nu, batch=3)
    pad = run(b, mode, max_it=0, plan=_plan(b, mode))
    tile = run(b, mode, max_it=0, plan=_plan(b, mode, "tile"))
    dt = np.float64 if mode == "f64" else np.float32
    fs = nu * (nu + 1) // 2 + nu + nx * nu + nx * (nx + 1) // 2 + nx
    olq = nu * (nu + 1) // 2 + nu + nx * nu
    n = b.batch * (N + 1) * fs
    A = pad["ws"].cpu().numpy().view(dt)[:n].reshape(b.batch, N + 1, fs).astype(np.float64)
    B = tile["ws"].cpu().numpy().view(dt)[:n].reshape(b.batch, N + 1, fs).astype(np.float64)
    for M in (A, B):  # stage 0 has no L^Q part, stage N only L^Q_N
        M[:, 0, olq:] = 0.0
        M[:, N, :olq] = 0.0
    tol = 1e-12 if mode == "f64" else 1e-5
    assert np.abs(A - B).max() <= tol * np.abs(B).max()


@pytest.mark.parametrize("mode", ["f64", "mixed_f32"])
def test_padded_gradients_match_tile(mode):
    print(f"case: small_padded gradients {mode}", flush=True)
    b = synth.make_batch(2, batch=3, N=12, nx=11, nu=4)
    grads = []
    for variant in (None, "tile"):
        t = {k: torch.tensor(getattr(b, k), dtype=torch.float64, device="cuda", requires_grad=True)
             for k in ("A", "B", "Q", "R", "q", "r", "x0")}
        x, u, _ = lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"], mode=mode, variant=variant)
        (0.5 * (x.pow(2).sum() + u.pow(2).sum())).backward()
        grads.append({k: v.grad.clone() for k, v in t.items()})
    for k in grads[0]:
        g0, g1 = grads[0][k].cpu().numpy(), grads[1][k].cpu().numpy()
        assert np.abs(g0 - g1).max() <= 1e-9 * max(1.0, np.abs(g1).max()), k


def test_padded_plan_refuses_updates():
    b = synth.random_problem(9, 6, 11, 4, batch=2)
    res = run(b, "f64", plan=_plan(b, "f64"))
    plan = res["plan"]
    assert plan.variant == "small_padded"
    info = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="small_padded"):
        U.factor_update(plan, res["data"], None, res["ws"], info)
