"""Adjoint (lq_solve_backward / torch.autograd.Function) against the oracle's adjoint gradient,
which is itself pinned to central finite differences in the CPU suite.

Bar: per input array, ||g_gpu - g_oracle||_inf <= 1e-8 ||g_oracle||_inf in float64 mode and
<= 1e-7 in mixed mode (both solves refined to rel_res <= 1e-10; the gradient error is the
solution error times the conditioning of K, ~1e5 here)."""
import numpy as np
import pytest

import synth
from oracle import adjoint, kkt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2512_09058_amd.autograd import lq_solve  # noqa: E402

NAMES = ["A", "B", "Q", "R", "S", "q", "r", "f", "x0"]


def _tensors(b, requires_grad=True):
    out = {}
    for k in NAMES:
        a = getattr(b, k)
        if a is None:
            out[k] = None
            continue
        out[k] = torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda", requires_grad=requires_grad)
    return out


def _gpu_grads(b, mode):
    t = _tensors(b)
    x, u, lam = lq_solve(t["A"], t["B"], t["Q"], t["R"], t["q"], t["r"], t["x0"], S=t["S"], f=t["f"], mode=mode)
    loss = 0.5 * (x.pow(2).sum() + u.pow(2).sum())
    loss.backward()
    return {k: (None if v is None else v.grad.cpu().numpy()) for k, v in t.items()}, (x, u, lam)


def _oracle_grads(p):
    x, u, _ = kkt.solve_dense(p)
    _, gx, gu = adjoint.quad_loss(x, u)
    g, _, _ = adjoint.adjoint_grad(p, gx, gu)
    return g


def _compare(b, gpu, tol):
    for i in range(b.batch):
        go = _oracle_grads(b.instance(i))
        for k in NAMES:
            if gpu[k] is None:
                continue
            ref = go[k]
            err = np.abs(gpu[k][i] - ref).max()
            assert err <= tol * max(np.abs(ref).max(), 1e-300), (i, k, err, np.abs(ref).max())


@pytest.mark.parametrize("mode,tol", [("f64", 1e-8), ("mixed_f32", 1e-7)])
def test_adjoint_random_with_S_and_f(mode, tol):
    print(f"case: adjoint random N=6 nx=5 nu=3 {mode}", flush=True)
    b = synth.random_problem(404, 6, 5, 3, batch=3)
    g, _ = _gpu_grads(b, mode)
    _compare(b, g, tol)


@pytest.mark.parametrize("mode,tol", [("f64", 1e-8), ("mixed_f32", 1e-7)])
def test_adjoint_config2_shape_small_factors(mode, tol):
    """nx=12, nu=4: the factors come from the size-specialised kernel, the adjoint sweeps from the
    generic one (same factor layout)."""
    print(f"case: adjoint config-2 shape {mode}", flush=True)
    b = synth.make_batch(2, batch=5, N=15)
    g, _ = _gpu_grads(b, mode)
    _compare(b, g, tol)


@pytest.mark.parametrize("mode,tol", [("f64", 1e-8), ("mixed_f32", 1e-7)])
def test_adjoint_config5_generators_reduced_horizon(mode, tol):
    print(f"case: adjoint config-5 generators N=20 {mode}", flush=True)
    b = synth.make_batch(5, batch=3, N=20)
    g, _ = _gpu_grads(b, mode)
    _compare(b, g, tol)


def test_gradcheck_tiny():
    """Finite differences of the HIP forward path itself against its hand-written backward."""
    print("case: gradcheck tiny", flush=True)
    b = synth.random_problem(7, 3, 2, 1, batch=2)
    t = _tensors(b)

    def fn(A, B, Q, R, S, q, r, f, x0):
        x, u, _ = lq_solve(A, B, Q, R, q, r, x0, S=S, f=f, mode="f64")
        return x, u

    args = tuple(t[k] for k in NAMES)
    assert torch.autograd.gradcheck(fn, args, eps=1e-6, atol=1e-8, rtol=1e-6)
