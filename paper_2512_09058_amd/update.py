"""Python binding of the factorisation updates (include/lqupdate.h): argument marshalling only; the
modification of the stage Hessians, the hyperbolic Householder update of the stored factors and
the right-hand-side sweep run in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check
from .api import Plan, _data, _ptr, _stream

LQ_UPDATE_MAX_ROWS = 64
LQ_INFO_UPDATE_RANK = -3


class LqUpdate(C.Structure):
    _fields_ = [("m", C.c_int32), ("C", C.c_void_p), ("D", C.c_void_p), ("dsig", C.c_void_p)]


def pack_rows(C_rows: Sequence[np.ndarray], D_rows: Sequence[np.ndarray], dsig: Sequence[np.ndarray],
              device="cuda") -> Dict[str, torch.Tensor]:
    """Per-instance rows (C [N+1, m, nx], D [N, m, nu], dsig [N+1, m], the same m everywhere) in the
    plan's instance order, concatenated into the device layout of lqupdate.h (a uniform batch may pass
    arrays with a leading batch axis)."""
    m = {int(np.shape(c)[-2]) for c in C_rows}
    if len(m) != 1:
        raise ValueError("every instance needs the same number of rows per stage")
    flat = lambda xs: torch.from_numpy(np.concatenate(  # noqa: E731
        [np.ascontiguousarray(x, dtype=np.float64).reshape(-1) for x in xs])).to(device)
    return {"m": m.pop(), "C": flat(C_rows), "D": flat(D_rows), "dsig": flat(dsig)}


def _upd(rows: Optional[Dict[str, torch.Tensor]]) -> LqUpdate:
    if rows is None:
        return LqUpdate(0, None, None, None)
    return LqUpdate(int(rows["m"]), _ptr(rows["C"]), _ptr(rows["D"]), _ptr(rows["dsig"]))


def max_columns(plan: Plan) -> int:
    """Nonzero rows per instance (over all its stages) that one update takes for this plan."""
    return int(_lib.load().lq_update_max_columns(plan.handle))


def workspace(plan: Plan, device="cuda") -> torch.Tensor:
    """The update workspace lq_factor_update needs with update rows."""
    n = int(_lib.load().lq_update_workspace_bytes(plan.handle))
    if n == 0:
        raise ValueError("this plan's stages do not fit the update kernels")
    return torch.empty(n, dtype=torch.uint8, device=device)


def update_data(plan: Plan, rows: Dict[str, torch.Tensor], data: Dict[str, torch.Tensor], stream=None):
    """Applies the rows' penalty changes to data["Q"], data["R"], data["S"] in place."""
    u = _upd(rows)
    check(_lib.load().lq_update_data(plan.handle, C.byref(u), _ptr(data["Q"]), _ptr(data["R"]), _ptr(data["S"]),
                                     _stream(stream)), "lq_update_data")


def factor_update(plan: Plan, data: Dict[str, torch.Tensor], rows: Optional[Dict[str, torch.Tensor]],
                  ws: torch.Tensor, info: torch.Tensor, uws: Optional[torch.Tensor] = None, stream=None):
    """Updates the factors in ws to those of `data` (already modified) and recomputes the
    right-hand-side sweep; rows=None only recomputes the sweep (new q, r, f).  uws: the update
    workspace (`workspace(plan)`), required with rows."""
    dd = _data(data)
    u = _upd(rows)
    check(_lib.load().lq_factor_update(plan.handle, C.byref(dd), C.byref(u), _ptr(ws), _ptr(uws), _ptr(info),
                                       _stream(stream)), "lq_factor_update")
