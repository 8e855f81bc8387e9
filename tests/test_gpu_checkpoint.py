"""Factor checkpointing: only every s-th cost-to-go factor is kept; lq_solve and
lq_solve_backward recompute each segment from its stored right end.  The recomputation repeats
the factor sweep's arithmetic, so the recomputed blocks are bit-identical to the stored ones:
generic plans give bit-identical solutions with and without checkpoints; tile plans (whose
checkpointed solve runs with another wavefront count, hence another summation order) are checked
block by block for the factors and to 1e-11 for the solutions, plus the oracle bars."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from paper_2512_09058_amd.autograd import lq_solve  # noqa: E402
from gpu_util import forward_error, instance_solution, oracle_solution, run  # noqa: E402
from oracle import kkt  # noqa: E402


def _solve(b, mode, ckpt, max_it):
    # the checkpointed solve recomputes segments with the generic factor code, so the reference
    # without checkpoints uses the generic kernels too
    plan = L.Plan(b.N, b.nx, b.nu, batch=b.batch, mode=mode, ckpt_stride=ckpt)
    plan.set_variant("generic")
    return run(b, mode, max_it=max_it, plan=plan)


@pytest.mark.parametrize("N,stride", [(35, 10), (40, 10), (7, 10), (9, 1), (12, 5)])
@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 6)])
def test_checkpointed_solve_is_bit_identical(N, stride, mode, max_it):
    print(f"case: checkpoint N={N} s={stride} {mode}", flush=True)
    b = synth.make_batch(5, batch=3, N=N)
    full = _solve(b, mode, 0, max_it)
    ck = _solve(b, mode, stride, max_it)
    assert full["plan"].variant == "generic" and ck["plan"].variant == "generic"
    assert np.all(ck["info"] == 0) and ck["rel"].max() <= 1e-10
    for k in ("x", "u", "lam"):
        assert torch.equal(full[k], ck[k]), k
    assert np.array_equal(full["iters"], ck["iters"])
    if 1 < stride < N:
        assert ck["plan"].workspace_bytes < full["plan"].workspace_bytes
    for i in range(b.batch):
        assert forward_error(instance_solution(ck, i), oracle_solution(b.instance(i))) <= 1e-9


@pytest.mark.parametrize("mode", ["f64", "mixed_f32"])
def test_checkpointed_adjoint_is_bit_identical(mode):
    print(f"case: checkpointed adjoint {mode}", flush=True)
    b = synth.make_batch(5, batch=2, N=23)
    grads = []
    for ckpt in (0, 10):
        t = {k: (None if getattr(b, k) is None else
                 torch.tensor(getattr(b, k), dtype=torch.float64, device="cuda", requires_grad=True))
             for k in ("A", "B", "Q", "R", "q", "r", "x0")}
        x, u, _ = lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"], mode=mode, ckpt_stride=ckpt,
                           variant="generic")
        (0.5 * (x.pow(2).sum() + u.pow(2).sum())).backward()
        grads.append({k: v.grad.clone() for k, v in t.items()})
    for k in grads[0]:
        assert torch.equal(grads[0][k], grads[1][k]), k


def _tile_plan(b, mode, ckpt):
    plan = L.Plan(b.N, b.nx, b.nu, batch=b.batch, mode=mode, ckpt_stride=ckpt)
    assert plan.variant == "tile"
    return plan


@pytest.mark.parametrize("N,stride", [(35, 10), (7, 10), (9, 1), (12, 5), (100, 10)])
@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 6)])
def test_tile_checkpointed_solve(N, stride, mode, max_it):
    """Tile plan with checkpoints (segments recomputed inside the solve kernel) against the oracle
    and against the same plan without checkpoints."""
    print(f"case: tile checkpoint N={N} s={stride} {mode}", flush=True)
    b = synth.make_batch(5, batch=3, N=N)
    full = run(b, mode, max_it=max_it, plan=_tile_plan(b, mode, 0))
    ck = run(b, mode, max_it=max_it, plan=_tile_plan(b, mode, stride))
    assert np.all(ck["info"] == 0) and ck["rel"].max() <= 1e-10, (ck["info"], ck["rel"])
    if 1 < stride < N:
        assert ck["plan"].workspace_bytes < full["plan"].workspace_bytes
    for i in range(b.batch):
        sol = instance_solution(ck, i)
        assert kkt.residual(b.instance(i), *sol)[1] <= 1e-10, i
        assert forward_error(sol, oracle_solution(b.instance(i))) <= 1e-9, i
        assert forward_error(sol, instance_solution(full, i)) <= 1e-11, i


def _blocks(ws, fbytes, fs, first, count):
    v = ws.cpu().numpy().view(np.float64 if fbytes == 8 else np.float32)
    return v[first * fs:(first + count) * fs].reshape(count, fs)


def _waves(t):
    # wavefronts of the tile factor sweep for t tile columns (3, 5 or 10)
    return 3 if t <= 3 else 5 if t <= 5 else 10


@pytest.mark.parametrize("nx,nu,mode", [(32, 8, "f64"), (40, 20, "f64"), (12, 50, "f64"), (32, 8, "mixed_f32"),
                                        (40, 20, "mixed_f32"), (12, 50, "mixed_f32"), (100, 20, "f64"),
                                        (100, 20, "mixed_bf16"), (40, 20, "mixed_bf16")])
def test_tile_recomputed_blocks_are_bit_identical(nx, nu, mode):
    """One instance, N = 23, s = 5: the checkpoint slots written by the factor kernel are the
    blocks of the full sweep (where both use one wavefront count), and the segment the solve
    kernel recomputed last ([20, 23) after a primal solve without refinement) equals the full
    sweep's blocks and its own checkpoint slot 20, bit for bit."""
    print(f"case: tile recomputed blocks nx={nx} nu={nu} {mode}", flush=True)
    N, s = 23, 5
    # wide states: the large-state generator (stable dynamics; I + 0.3 G would grow like 4^k at nx = 100)
    p = synth.make_instance(4, 0, N=N, nx=nx, nu=nu) if nx > 64 else synth.random_problem(800 + nx + nu, N, nx, nu)
    fbytes = 8 if mode == "f64" else 4
    fs = nu * (nu + 1) // 2 + nu + nx * nu + nx * (nx + 1) // 2 + nx
    full = run([p], mode, max_it=0, plan=L.Plan([N], [nx], [nu], mode=mode))
    plan = L.Plan([N], [nx], [nu], mode=mode, ckpt_stride=s)
    assert plan.variant == "tile"
    ck = run([p], mode, max_it=0, plan=plan)
    # (a sanity bound on the unrefined residual: bf16 products leave it of order one at nx = 100,
    # which the refinement of a real solve removes; this test is about the blocks)
    assert ck["info"][0] == 0 and ck["rel"][0] <= {"f64": 1e-10, "mixed_f32": 1e-3, "mixed_bf16": 10.0}[mode]
    F = _blocks(full["ws"], fbytes, fs, 0, N + 1)
    nslots = N // s + 2                     # stages 0, 5, 10, 15, 20 and N
    slots = _blocks(ck["ws"], fbytes, fs, 0, nslots)
    seg = _blocks(ck["ws"], fbytes, fs, nslots, N - 20)
    assert np.array_equal(seg[0], slots[4])
    # the checkpointed plan's factor sweep runs with the wavefront count of the padded sizes
    nxp = 32 if nx <= 32 else 64 if nx <= 64 else 128
    nup = 16 if nu <= 16 else 32 if nu <= 32 else 64
    same_waves = (_waves((nx + 15) // 16 + (nu + 15) // 16) == _waves(nxp // 16 + nup // 16)
                  or full["plan"].variant != "tile")
    olq = nu * (nu + 1) // 2 + nu + nx * nu  # stage 0 leaves its L^Q part unwritten
    if same_waves:
        assert np.array_equal(slots[0][:olq], F[0][:olq])
        for j, k in enumerate([5, 10, 15, 20]):
            assert np.array_equal(slots[j + 1], F[k]), k
        assert np.array_equal(slots[-1][olq:], F[N][olq:])
        assert np.array_equal(seg, F[20:N])
    else:
        np.testing.assert_allclose(seg, F[20:N], rtol=0, atol=1e-12 * np.abs(F).max())


@pytest.mark.parametrize("mode", ["f64", "mixed_f32"])
def test_tile_checkpointed_adjoint(mode):
    """Gradients through the checkpointed tile path against the uncheckpointed tile path and the
    oracle's dense adjoint."""
    from oracle import adjoint
    print(f"case: tile checkpointed adjoint {mode}", flush=True)
    b = synth.make_batch(5, batch=2, N=23)
    grads = []
    for ckpt in (0, 10):
        t = {k: torch.tensor(getattr(b, k), dtype=torch.float64, device="cuda", requires_grad=True)
             for k in ("A", "B", "Q", "R", "q", "r", "x0")}
        x, u, _ = lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"], mode=mode, ckpt_stride=ckpt,
                           variant="tile")
        (0.5 * (x.pow(2).sum() + u.pow(2).sum())).backward()
        grads.append({k: v.grad.clone() for k, v in t.items()})
    for i in range(b.batch):
        p = b.instance(i)
        xo, uo, _ = kkt.solve_dense(p)
        _, gx, gu = adjoint.quad_loss(xo, uo)
        ref, _, _ = adjoint.adjoint_grad(p, gx, gu)
        for k in grads[0]:
            g0, g1 = grads[0][k][i].cpu().numpy(), grads[1][k][i].cpu().numpy()
            scale = max(1.0, np.abs(ref[k]).max())
            assert np.abs(g1 - g0).max() <= 1e-10 * scale, (i, k)
            assert np.abs(g1 - ref[k]).max() <= 1e-8 * scale, (i, k)


def test_nonfinite_right_hand_side_reports_info():
    """A NaN only in the right-hand side (q) leaves the factors finite: the solve's residual must
    come out NaN and the instance flagged, in every variant, with and without checkpoints."""
    print("case: NaN in q, every variant", flush=True)
    cases = [("small", synth.make_batch(2, batch=3, N=10), 0),
             ("tile", synth.make_batch(5, batch=3, N=12), 0),
             ("tile", synth.make_batch(5, batch=3, N=12), 5),
             ("generic", synth.make_batch(5, batch=3, N=12), 0),
             ("generic", synth.make_batch(5, batch=3, N=12), 5)]
    for variant, b, ckpt in cases:
        b.q = b.q.copy()
        b.q[1, 3, 0] = np.nan
        for mode, mi in (("f64", 0), ("mixed_f32", 4)):
            plan = L.Plan(b.N, b.nx, b.nu, batch=b.batch, mode=mode, ckpt_stride=ckpt)
            plan.set_variant(variant)
            res = run(b, mode, max_it=mi, plan=plan)
            assert res["info"][1] == -1, (variant, ckpt, mode, res["info"])
            assert np.isnan(res["rel"][1]), (variant, ckpt, mode, res["rel"])
            assert res["info"][0] == 0 and res["info"][2] == 0, (variant, ckpt, mode, res["info"])


@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 8)])
def test_tile_checkpointed_ragged_batch(mode, max_it):
    """A ragged checkpointed batch spanning both padded state sizes of the checkpointed tile solve
    (nx 10..60, nu 3..40, N 6..31, stride 7; persistent grid): library residual, oracle residual and
    forward error for every instance."""
    import numpy as np_
    rng = np_.random.default_rng(77)
    insts = [synth.random_problem(900 + i, int(rng.integers(6, 32)), int(rng.integers(10, 61)),
                                  int(rng.integers(3, 41))) for i in range(10)]
    print(f"case: tile checkpointed ragged {mode}", flush=True)
    plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode=mode, ckpt_stride=7)
    assert plan.variant == "tile"
    res = run(insts, mode, max_it=max_it, plan=plan)
    assert np.all(res["info"] == 0) and res["rel"].max() <= 1e-10, (res["info"], res["rel"])
    for i, p in enumerate(insts):
        sol = instance_solution(res, i)
        assert kkt.residual(p, *sol)[1] <= 1e-10, i
        assert forward_error(sol, oracle_solution(p)) <= 1e-9, i


@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 8), ("mixed_bf16", 12)])
def test_tile_checkpointed_wide_state_and_bf16(mode, max_it):
    """Checkpointed tile plans at padded nx 128 (nx = 100, nu = 20: nine tile columns) in every
    mode, bf16 products included: against the oracle, the oracle's residual and the same plan
    without checkpoints (whose factor sweep uses the same wavefront count, so the factor blocks
    agree bit for bit and the solutions to rounding)."""
    print(f"case: tile checkpoint nx=100 nu=20 {mode}", flush=True)
    b = synth.make_batch(4, batch=2, N=12, nx=100, nu=20)
    full = run(b, mode, max_it=max_it, plan=_tile_plan(b, mode, 0))
    ck = run(b, mode, max_it=max_it, plan=_tile_plan(b, mode, 5))
    assert ck["plan"].variant == "tile"
    assert np.all(ck["info"] == 0) and ck["rel"].max() <= 1e-10, (ck["info"], ck["rel"])
    assert ck["plan"].workspace_bytes < full["plan"].workspace_bytes
    bar = 1e-11 if mode == "f64" else 1e-9
    for i in range(b.batch):
        sol = instance_solution(ck, i)
        assert kkt.residual(b.instance(i), *sol)[1] <= 1e-10, i
        assert forward_error(sol, oracle_solution(b.instance(i))) <= 1e-9, i
        assert forward_error(sol, instance_solution(full, i)) <= bar, i


@pytest.mark.parametrize("mode", ["f64", "mixed_bf16"])
def test_tile_checkpointed_adjoint_wide_state(mode):
    """Gradients through the checkpointed tile path at padded nx 128 (nx = 100, nu = 20), float64
    and bf16 products: against the same plan without checkpoints and the oracle's dense adjoint."""
    from oracle import adjoint
    print(f"case: tile checkpointed adjoint nx=100 {mode}", flush=True)
    b = synth.make_batch(4, batch=2, N=12, nx=100, nu=20)
    grads = []
    for ckpt in (0, 5):
        t = {k: torch.tensor(getattr(b, k), dtype=torch.float64, device="cuda", requires_grad=True)
             for k in ("A", "B", "Q", "R", "q", "r", "x0")}
        x, u, _ = lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"], mode=mode, ckpt_stride=ckpt,
                           variant="tile", max_it=12)
        (0.5 * (x.pow(2).sum() + u.pow(2).sum())).backward()
        grads.append({k: v.grad.clone() for k, v in t.items()})
    for i in range(b.batch):
        p = b.instance(i)
        xo, uo, _ = kkt.solve_dense(p)
        _, gx, gu = adjoint.quad_loss(xo, uo)
        ref, _, _ = adjoint.adjoint_grad(p, gx, gu)
        for k in grads[0]:
            g0, g1 = grads[0][k][i].cpu().numpy(), grads[1][k][i].cpu().numpy()
            scale = max(1.0, np.abs(ref[k]).max())
            assert np.abs(g1 - g0).max() <= 1e-9 * scale, (i, k)
            assert np.abs(g1 - ref[k]).max() <= 1e-7 * scale, (i, k)
