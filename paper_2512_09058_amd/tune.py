"""Autotuner of the general-size kernels' launch shape (workgroup size, persistent grid,
workgroups per CU) for a plan's shape signature.

tune(plan, data) times every candidate on the caller's data (factor + solve, best of a few
runs), applies the fastest to the plan and records it in a JSON cache keyed by device name and
plan signature; apply_cached(plan) reuses a recorded choice.  The cache path is the argument,
else $LQKKT_TUNE_CACHE; without either nothing is read or written.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

import torch

from . import api

CANDIDATES = [{"threads": t, "persistent": p, "blocks_per_cu": b}
              for t in (64, 128, 256) for p, b in ((0, 0), (1, 0), (1, 1), (1, 2))]


def _key(plan: api.Plan) -> str:
    return f"{torch.cuda.get_device_name()}|{plan.signature()}"


def _cache_path(path: Optional[str]) -> Optional[str]:
    return path or os.environ.get("LQKKT_TUNE_CACHE")


def apply_cached(plan: api.Plan, path: Optional[str] = None) -> Optional[Dict]:
    p = _cache_path(path)
    if not p or not os.path.exists(p):
        return None
    cfg = json.load(open(p)).get(_key(plan))
    if cfg:
        plan.set_launch(**cfg["launch"])
    return cfg


def tune(plan: api.Plan, data: Dict[str, torch.Tensor], tol: float = 1e-10, max_it: int = 0, reps: int = 3,
         path: Optional[str] = None, candidates=CANDIDATES) -> Dict:
    ws = plan.workspace()
    info = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    rel = torch.zeros(plan.batch, dtype=torch.float64, device="cuda")
    x, u, lam = plan.empty_outputs()
    results = []
    for c in candidates:
        plan.set_launch(**c)
        best = float("inf")
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            api.factor(plan, data, ws, info)
            api.solve(plan, data, ws, x, u, lam, rel, None, info, tol=tol, max_it=max_it)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        results.append((best, c))
    results.sort(key=lambda r: r[0])
    choice = {"launch": results[0][1], "ms": results[0][0] * 1e3,
              "tried": [{"ms": r[0] * 1e3, **r[1]} for r in results]}
    plan.set_launch(**choice["launch"])
    p = _cache_path(path)
    if p:
        db = json.load(open(p)) if os.path.exists(p) else {}
        db[_key(plan)] = choice
        tmp = p + ".tmp"
        json.dump(db, open(tmp, "w"), indent=1)
        os.replace(tmp, p)
    return choice
