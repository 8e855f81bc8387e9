"""torch.autograd.Function over the C ABI: forward = lq_factor + lq_solve, backward =
lq_solve_backward (the adjoint KKT solve with the stored factors, then the per-stage gradient
outer products).  Uniform batches with shaped tensors:

    A [B, N, nx, nx]   B [B, N, nx, nu]   Q [B, N+1, nx, nx]   R [B, N, nu, nu]
    S [B, N, nu, nx] or None   q [B, N+1, nx]   r [B, N, nu]   f [B, N, nx] or None   x0 [B, nx]

returns x [B, N, nx] (x_1..x_N), u [B, N, nu] (u_0..u_{N-1}) and lam [B, N, nx].  x and u are
differentiable; lam is returned as a constant.

With check=True (the default) the forward pass and the backward pass each synchronise once and raise
SolveError when an instance reports a non-zero status (a stage matrix that is not positive
definite, a non-finite value, refinement stopped above tol) or a relative KKT residual above tol;
check=False leaves the statuses unread (no synchronisation), for callers that inspect them
through `last_status`.
"""
from __future__ import annotations

from typing import Dict, Optional, Tuple

import torch

from . import api

_PLANS: Dict[Tuple, api.Plan] = {}


class SolveError(RuntimeError):
    """An instance of the batch did not solve: `info` and `rel_res` hold the per-instance values."""

    def __init__(self, what, info, rel_res, tol):
        self.info, self.rel_res, self.tol = info, rel_res, tol
        bad = [int(i) for i in ((info != 0) | ~(rel_res <= tol)).nonzero().flatten()[:8]]
        detail = ", ".join(f"instance {i}: info={int(info[i])} rel_res={float(rel_res[i]):.3e}" for i in bad)
        super().__init__(f"{what}: {detail} (tol {tol:.1e})")


# statuses of the most recent forward and backward call (device tensors; read them after a sync)
last_status: Dict[str, Tuple[torch.Tensor, torch.Tensor]] = {}


def _raise_on_failure(what, info, rel, tol):
    info_h, rel_h = info.cpu(), rel.cpu()
    if bool(((info_h != 0) | ~(rel_h <= tol)).any()):
        raise SolveError(what, info_h, rel_h, tol)


def _plan(batch, N, nx, nu, mode, ckpt, variant, device) -> api.Plan:
    key = (batch, N, nx, nu, mode, ckpt, variant, torch.device(device).index)
    p = _PLANS.get(key)
    if p is None:
        p = api.Plan(N, nx, nu, batch=batch, mode=mode, ckpt_stride=ckpt)
        if variant:
            p.set_variant(variant)
        _PLANS[key] = p
    return p


class LQSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, Q, R, S, q, r, f, x0, mode, tol, max_it, ckpt, variant, check):
        batch, N, nx, _ = A.shape
        nu = B.shape[-1]
        plan = _plan(batch, N, nx, nu, mode, ckpt, variant, A.device)
        data = {"A": A, "B": B, "Q": Q, "R": R, "q": q, "r": r, "x0": x0}
        if S is not None:
            data["S"] = S
        if f is not None:
            data["f"] = f
        data = {k: v.detach().contiguous().reshape(-1) for k, v in data.items()}
        ws = plan.workspace(A.device)
        info = torch.zeros(batch, dtype=torch.int32, device=A.device)
        rel = torch.empty(batch, dtype=torch.float64, device=A.device)
        x, u, lam = plan.empty_outputs(A.device)
        api.factor(plan, data, ws, info)
        api.solve(plan, data, ws, x, u, lam, rel, None, info, tol=tol, max_it=max_it)
        last_status["forward"] = (info, rel)
        if check:
            _raise_on_failure("lq_solve", info, rel, tol)
        ctx.save_for_backward(x, u, lam)
        ctx.plan, ctx.data, ctx.ws, ctx.info = plan, data, ws, info
        ctx.has_S, ctx.has_f = S is not None, f is not None
        ctx.tol, ctx.max_it, ctx.check = tol, max_it, check
        ctx.shapes = (batch, N, nx, nu)
        lam_s = lam.view(batch, N, nx)
        ctx.mark_non_differentiable(lam_s)
        return x.view(batch, N, nx), u.view(batch, N, nu), lam_s

    @staticmethod
    def backward(ctx, gx, gu, glam):
        x, u, lam = ctx.saved_tensors
        batch, N, nx, nu = ctx.shapes
        dev = x.device
        gx = torch.zeros_like(x) if gx is None else gx.contiguous().reshape(-1)
        gu = torch.zeros_like(u) if gu is None else gu.contiguous().reshape(-1)
        plan = ctx.plan
        g = {k: torch.empty(plan.totals[k], dtype=torch.float64, device=dev) for k in ("A", "B", "Q", "R", "q", "r", "x0")}
        if ctx.has_S:
            g["S"] = torch.empty(plan.totals["S"], dtype=torch.float64, device=dev)
        if ctx.has_f:
            g["f"] = torch.empty(plan.totals["f"], dtype=torch.float64, device=dev)
        info = ctx.info.clone()
        rel = torch.empty(batch, dtype=torch.float64, device=dev)
        api.solve_backward(plan, ctx.data, ctx.ws, x, u, lam, gx, gu, g, rel, None, info, tol=ctx.tol,
                           max_it=ctx.max_it)
        last_status["backward"] = (info, rel)
        if ctx.check:
            _raise_on_failure("lq_solve_backward", info, rel, ctx.tol)
        sh = {"A": (batch, N, nx, nx), "B": (batch, N, nx, nu), "Q": (batch, N + 1, nx, nx), "R": (batch, N, nu, nu),
              "S": (batch, N, nu, nx), "q": (batch, N + 1, nx), "r": (batch, N, nu), "f": (batch, N, nx),
              "x0": (batch, nx)}
        out = {k: v.view(sh[k]) for k, v in g.items()}
        return (out["A"], out["B"], out["Q"], out["R"], out.get("S"), out["q"], out["r"], out.get("f"), out["x0"],
                None, None, None, None, None, None)


def lq_solve(A, B, Q, R, q, r, x0, S=None, f=None, mode: str = "f64", tol: float = 1e-10,
             max_it: Optional[int] = None, ckpt_stride: int = 0, variant: Optional[str] = None,
             check: bool = True):
    """Differentiable batched LQ KKT solve (see module docstring for shapes).  ckpt_stride > 0
    keeps only every ckpt_stride-th cost-to-go factor between forward and backward and recomputes
    the rest segment by segment.  variant selects the factor kernel ("small", "small_padded", "tile", "generic";
    default: the plan's choice).  check: raise SolveError on a failed instance (module docstring)."""
    if max_it is None:
        max_it = 0 if mode == "f64" else 10
    return LQSolveFn.apply(A, B, Q, R, S, q, r, f, x0, mode, tol, max_it, int(ckpt_stride), variant, bool(check))
