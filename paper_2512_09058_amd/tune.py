"""Autotuner of a plan's kernel variant and launch shape for its shape signature.

Candidates are every factor-kernel variant that can take the plan (size-specialised, matrix-core
tile, generic) and, per variant, the launch shapes it honours (workgroup size for the generic
kernels; one workgroup per instance or a persistent grid with 1, 2 or as many workgroups per CU
as fit).  tune(plan, data) times every candidate on the caller's data (factor + solve, best of a
few runs), applies the fastest to the plan and records it in a JSON cache keyed by device name
and plan signature; apply_cached(plan) reuses a recorded choice.  The cache path is the
argument, else $LQKKT_TUNE_CACHE; without either nothing is read or written.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

import torch

from . import api

PERSISTENCE = ((0, 0), (1, 0), (1, 1), (1, 2))
CANDIDATES = [{"threads": t, "persistent": p, "blocks_per_cu": b} for t in (64, 128, 256, 512) for p, b in PERSISTENCE]


def candidates(plan: api.Plan):
    """(variant, launch) pairs the plan can run; the plan's current variant is kept."""
    out = []
    current = plan.variant
    for v in ("small", "small_padded", "tile", "generic"):
        try:
            plan.set_variant(v)
        except RuntimeError:
            continue
        if v in ("small", "small_padded"):
            out.append({"variant": v, "launch": plan.get_launch()})
        elif v == "tile":
            out += [{"variant": v, "launch": {"threads": 128, "persistent": p, "blocks_per_cu": b}}
                    for p, b in PERSISTENCE]
        else:
            out += [{"variant": v, "launch": c} for c in CANDIDATES]
    plan.set_variant(current)
    return out


def _apply(plan: api.Plan, cand: Dict):
    plan.set_variant(cand["variant"])
    plan.set_launch(**cand["launch"])


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
        _apply(plan, cfg)
    return cfg


def tune(plan: api.Plan, data: Dict[str, torch.Tensor], tol: float = 1e-10, max_it: int = 0, reps: int = 3,
         path: Optional[str] = None, cands=None, prune: float = 3.0) -> Dict:
    """Times the candidates (best of reps runs after a first one); a candidate whose first run
    already takes more than prune times the best time so far is not run again."""
    ws = plan.workspace()
    info = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    rel = torch.zeros(plan.batch, dtype=torch.float64, device="cuda")
    x, u, lam = plan.empty_outputs()
    results = []
    overall = float("inf")
    for c in (cands if cands is not None else candidates(plan)):
        _apply(plan, c)
        best = float("inf")
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            api.factor(plan, data, ws, info)
            api.solve(plan, data, ws, x, u, lam, rel, None, info, tol=tol, max_it=max_it)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
            if r == 0 and best > prune * overall:
                break
        overall = min(overall, best)
        results.append((best, c))
    results.sort(key=lambda r: r[0])
    choice = {"variant": results[0][1]["variant"], "launch": results[0][1]["launch"], "ms": results[0][0] * 1e3,
              "tried": [{"ms": r[0] * 1e3, **r[1]} for r in results]}
    _apply(plan, choice)
    p = _cache_path(path)
    if p:
        db = json.load(open(p)) if os.path.exists(p) else {}
        db[_key(plan)] = choice
        tmp = p + ".tmp"
        json.dump(db, open(tmp, "w"), indent=1)
        os.replace(tmp, p)
    return choice
