"""Python binding of the box-constrained QP solver (include/lqqp.h): argument marshalling only; the
Newton systems, the line search, the iterate and outer updates run in the library's HIP kernels and
the Newton systems are solved by its factorisation and solve."""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check
from .api import Plan, _data, _ptr, _stream


class LqQpConstraints(C.Structure):
    _fields_ = [("m", C.c_int32), ("C", C.c_void_p), ("D", C.c_void_p), ("bl", C.c_void_p), ("bu", C.c_void_p)]


class LqQpOpts(C.Structure):
    _fields_ = [("sigma0", C.c_double), ("gamma", C.c_double), ("eps", C.c_double), ("theta", C.c_double),
                ("sigma_up", C.c_double), ("sigma_max", C.c_double), ("inner_tol", C.c_double),
                ("max_outer", C.c_int32), ("max_inner", C.c_int32), ("warm", C.c_int32), ("intervals", C.c_int32)]


DEFAULTS = dict(sigma0=1e2, gamma=1e7, eps=1e-9, theta=0.25, sigma_up=10.0, sigma_max=1e9, inner_tol=1e-11,
                max_outer=100, max_inner=50, warm=0, intervals=0)


def pack_constraints(Cs: Sequence[np.ndarray], Ds: Sequence[np.ndarray], bls: Sequence[np.ndarray],
                     bus: Sequence[np.ndarray], device="cuda") -> Dict[str, torch.Tensor]:
    """Per-instance rows (C [N+1, m, nx], D [N, m, nu], bl, bu [N+1, m], the same m everywhere), in the
    plan's instance order, concatenated into the device layout of lqqp.h."""
    m = {int(np.shape(c)[-2]) for c in Cs}
    if len(m) != 1:
        raise ValueError("every instance needs the same number of rows per stage")
    flat = lambda xs: torch.from_numpy(np.concatenate(  # noqa: E731
        [np.ascontiguousarray(x, dtype=np.float64).reshape(-1) for x in xs])).to(device)
    return {"m": m.pop(), "C": flat(Cs), "D": flat(Ds), "bl": flat(bls), "bu": flat(bus)}


def workspace(plan: Plan, m: int, intervals: int = 0, device="cuda") -> torch.Tensor:
    n = int(_lib.load().lq_qp_workspace_bytes(plan.handle, int(m), int(intervals)))
    if n == 0:
        raise ValueError("invalid plan or m")
    return torch.empty(n, dtype=torch.uint8, device=device)


def solve(plan: Plan, data: Dict[str, torch.Tensor], cons: Dict[str, torch.Tensor], ws: torch.Tensor,
          qws: torch.Tensor, x, u, lam, y, status, iters, opts: Optional[dict] = None, stream=None):
    """lq_qp_solve.  x, u, lam in the plan's output layout; y, status, iters as in lqqp.h; with
    opts["warm"] = 1 the given u and y are the start."""
    o = dict(DEFAULTS)
    o.update(opts or {})
    oo = LqQpOpts(float(o["sigma0"]), float(o["gamma"]), float(o["eps"]), float(o["theta"]), float(o["sigma_up"]),
                  float(o["sigma_max"]), float(o["inner_tol"]), int(o["max_outer"]), int(o["max_inner"]),
                  int(o["warm"]), int(o["intervals"]))
    cc = LqQpConstraints(int(cons["m"]), _ptr(cons["C"]), _ptr(cons["D"]), _ptr(cons["bl"]), _ptr(cons["bu"]))
    dd = _data(data)
    check(_lib.load().lq_qp_solve(plan.handle, C.byref(dd), C.byref(cc), C.byref(oo), _ptr(ws), _ptr(qws), _ptr(x),
                                  _ptr(u), _ptr(lam), _ptr(y), _ptr(status), _ptr(iters), _stream(stream)),
          "lq_qp_solve")
