"""Factor checkpointing: only every s-th cost-to-go factor is kept; lq_solve and
lq_solve_backward recompute each segment from its stored right end.  The recomputation repeats
the factor sweep's arithmetic, so results are bit-identical to storing every stage."""
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
