"""The allocation-free entry point (lq_factor_solve_noalloc) against lq_factor + lq_solve on a
plan: the same size-specialised kernels, so the outputs must be bit-identical; two calls in a row,
the second with a smaller batch (the shared scratch array keeps the first call's contents), in
float64 and mixed precision; plus its refusal of a batch above the scratch limit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_09058_amd as L  # noqa: E402
from gpu_util import run  # noqa: E402


def _noalloc(b, mode, max_it):
    data = L.pack(b)
    plan_like = L.Plan(b.N, b.nx, b.nu, batch=b.batch, mode=mode)  # only for the output sizes
    x, u, lam = plan_like.empty_outputs()
    rel = torch.full((b.batch,), -1.0, dtype=torch.float64, device="cuda")
    its = torch.full((b.batch,), -1, dtype=torch.int32, device="cuda")
    info = torch.full((b.batch,), 7, dtype=torch.int32, device="cuda")
    L.api.factor_solve_noalloc(b.batch, b.N, b.nx, b.nu, data, x, u, lam, rel, its, info, mode=mode, tol=1e-10,
                               max_it=max_it)
    torch.cuda.synchronize()
    return {"x": x.cpu().numpy(), "u": u.cpu().numpy(), "lam": lam.cpu().numpy(), "rel": rel.cpu().numpy(),
            "iters": its.cpu().numpy(), "info": info.cpu().numpy()}


@pytest.mark.parametrize("mode,max_it", [("f64", 0), ("mixed_f32", 10)])
def test_noalloc_matches_plan_path_twice(mode, max_it):
    for batch, N, seed in ((600, 50, 0), (37, 20, 1)):
        print(f"case: noalloc {mode} batch={batch} N={N}", flush=True)
        b = synth.make_batch(2, batch=batch, N=N, start=seed * 1000)
        ref = run(b, mode, max_it=max_it)
        assert ref["plan"].variant == "small"
        got = _noalloc(b, mode, max_it)
        for k in ("x", "u", "lam"):
            assert np.array_equal(got[k], ref[k].cpu().numpy()), k
        assert np.array_equal(got["rel"], ref["rel"])
        assert np.array_equal(got["iters"], ref["iters"])
        assert np.array_equal(got["info"], ref["info"])
        assert np.all(got["info"] == 0) and got["rel"].max() <= 1e-10


def test_noalloc_refuses_batches_above_the_limit():
    from paper_2512_09058_amd import _lib
    big = 20000  # config-2 sizes: about 86 kB of scratch per instance in float64
    data = {k: torch.zeros(1, dtype=torch.float64, device="cuda") for k in ("A", "B", "Q", "R", "q", "r", "x0")}
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="status -2"):
        L.api.factor_solve_noalloc(big, 50, 12, 4, data, out, out, out, None, None, info)
    assert "scratch" in _lib.load().lq_last_error().decode()
    with pytest.raises(RuntimeError, match="status -2"):
        L.api.factor_solve_noalloc(4, 10, 5, 3, data, out, out, out, None, None, info)  # no small kernel
