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
