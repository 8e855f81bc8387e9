"""Helpers for GPU tests: run the HIP path through the binding and compare with the oracle."""
import numpy as np
import torch

import paper_2512_09058_amd as L
from oracle import kkt, riccati


def run(problems, mode="f64", tol=1e-10, max_it=0, check=True, plan=None):
    """Factor + solve a batch (LQProblem batch or list of instances); returns dict of results."""
    insts = problems if isinstance(problems, list) else [problems.instance(i) for i in range(problems.batch)]
    if plan is None:
        plan = L.Plan([p.N for p in insts], [p.nx for p in insts], [p.nu for p in insts], mode=mode)
    data = L.pack(problems)
    ws = plan.workspace()
    info = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    x, u, lam = plan.empty_outputs()
    rel = torch.full((plan.batch,), -1.0, dtype=torch.float64, device="cuda")
    its = torch.full((plan.batch,), -1, dtype=torch.int32, device="cuda")
    L.factor(plan, data, ws, info)
    L.solve(plan, data, ws, x, u, lam, rel, its, info, tol=tol, max_it=max_it, check_res=check)
    torch.cuda.synchronize()
    return {"plan": plan, "data": data, "ws": ws, "info": info.cpu().numpy(), "x": x, "u": u, "lam": lam,
            "rel": rel.cpu().numpy(), "iters": its.cpu().numpy(), "insts": insts}


def instance_solution(res, i):
    plan = res["plan"]
    return (L.unpack(plan, "x", res["x"], i), L.unpack(plan, "u", res["u"], i), L.unpack(plan, "lam", res["lam"], i))


def forward_error(sol, ref):
    num = max(np.abs(a - b).max() for a, b in zip(sol, ref))
    den = max(np.abs(b).max() for b in ref)
    return num / den


def oracle_solution(p):
    return riccati.solve(p) if p.N * (2 * p.nx + p.nu) > 3000 else kkt.solve_dense(p)


# ---------------------------------------------------------------------------------------------
# Workspace layout (as documented with the descriptor in the library's internal header): the
# factor region first (per instance (N+1) stage blocks of FS elements of the factor type), then,
# each 256-byte aligned, the float64 sweep vectors (N nu + (N+1) nx per instance) and the float64
# refinement state (rbar2 [N nu] | p2 [(N+1) nx] | flam [N nx] | rho_u [N nu] | rho_x [(N+1) nx]).

def _a256(v):
    return (v + 255) & ~255


def stage_elems(nx, nu):
    return nu * (nu + 1) // 2 + nu + nx * nu + nx * (nx + 1) // 2 + nx


def workspace_views(res):
    """Per-instance views of the factor blocks and of the refinement state (host numpy)."""
    plan = res["plan"]
    raw = res["ws"].cpu().numpy()
    fdt = np.float64 if plan.mode == "f64" else np.float32
    fb = np.dtype(fdt).itemsize
    N, nx, nu = plan.N.astype(np.int64), plan.nx.astype(np.int64), plan.nu.astype(np.int64)
    fs = np.array([stage_elems(a, b) for a, b in zip(nx, nu)], np.int64)
    aF = int(np.sum((N + 1) * fs))
    aV = int(np.sum(N * nu + (N + 1) * nx))
    offV = _a256(aF * fb)
    offV2 = _a256(offV + aV * 8)
    F = raw[:aF * fb].view(fdt)
    v2n = 2 * N * nu + 2 * (N + 1) * nx + N * nx
    V2 = raw[offV2:offV2 + int(v2n.sum()) * 8].view(np.float64)
    out = []
    oF, o2 = 0, 0
    for i in range(plan.batch):
        n, x, u = int(N[i]), int(nx[i]), int(nu[i])
        blocks = F[oF:oF + (n + 1) * int(fs[i])].reshape(n + 1, int(fs[i])).astype(np.float64)
        v = V2[o2:o2 + int(v2n[i])]
        st = {"rbar2": v[:n * u].reshape(n, u),
              "flam": v[n * u + (n + 1) * x:n * u + (n + 1) * x + n * x].reshape(n, x),
              "rho_u": v[n * u + (n + 1) * x + n * x:2 * n * u + (n + 1) * x + n * x].reshape(n, u),
              "rho_x": v[2 * n * u + (n + 1) * x + n * x:].reshape(n + 1, x)}
        out.append((blocks, st))
        oF += (n + 1) * int(fs[i])
        o2 += int(v2n[i])
    return out


def unpack_factor_block(blk, nx, nu):
    """(L^R, 1/diag L^R, L^S, L^Q, 1/diag L^Q) of one stage block."""
    def tri(v, n):
        M = np.zeros((n, n))
        M[np.tril_indices(n)] = v
        return M
    o = 0
    Lr = tri(blk[o:o + nu * (nu + 1) // 2], nu); o += nu * (nu + 1) // 2
    dR = blk[o:o + nu]; o += nu
    Ls = blk[o:o + nx * nu].reshape(nx, nu); o += nx * nu
    Lq = tri(blk[o:o + nx * (nx + 1) // 2], nx); o += nx * (nx + 1) // 2
    dQ = blk[o:o + nx]
    return Lr, dR, Ls, Lq, dQ


def elementwise_ok(sol, ref, rtol, atol_rel):
    """|a_i - b_i| <= rtol |b_i| + atol_rel ||b||_inf for every entry of x, u and lam; returns the
    worst ratio of the error to that bound (<= 1 passes)."""
    scale = max(np.abs(b).max() for b in ref)
    worst = 0.0
    for a, b in zip(sol, ref):
        bound = rtol * np.abs(b) + atol_rel * scale
        worst = max(worst, float((np.abs(a - b) / bound).max()))
    return worst
