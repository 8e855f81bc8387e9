"""Python binding of the parallel-in-time solve (include/lqpit.h): argument marshalling only; the
interval recursions, the Schur complement, its cyclic reduction and the sweeps run in the library's
HIP kernels.  Uniform batches in the packed layout of `api.pack`."""
from __future__ import annotations

import ctypes as C
from typing import Dict

import torch

from . import _lib
from ._lib import check
from .api import _data, _ptr, _stream


class PitPlan:
    """Sizes of a uniform batch split into P intervals, and its workspace size."""

    def __init__(self, batch: int, N: int, nx: int, nu: int, P: int):
        self.batch, self.N, self.nx, self.nu, self.P = int(batch), int(N), int(nx), int(nu), int(P)
        self.workspace_bytes = int(_lib.load().lq_pit_workspace_bytes(self.batch, self.N, self.nx, self.nu, self.P))
        if self.workspace_bytes == 0:
            raise ValueError(f"invalid sizes batch={batch} N={N} nx={nx} nu={nu} P={P}")

    def dims(self):
        return (self.batch, self.N, self.nx, self.nu, self.P)

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def empty_outputs(self, device="cuda"):
        b, N, nx, nu = self.batch, self.N, self.nx, self.nu
        return (torch.empty(b * N * nx, dtype=torch.float64, device=device),
                torch.empty(b * N * nu, dtype=torch.float64, device=device),
                torch.empty(b * N * nx, dtype=torch.float64, device=device))


def factor(plan: PitPlan, data: Dict[str, torch.Tensor], ws: torch.Tensor, info: torch.Tensor, stream=None):
    dd = _data(data)
    check(_lib.load().lq_pit_factor(*plan.dims(), C.byref(dd), _ptr(ws), _ptr(info), _stream(stream)),
          "lq_pit_factor")


def solve(plan: PitPlan, data: Dict[str, torch.Tensor], ws: torch.Tensor, x, u, lam, rel_res=None, info=None,
          stream=None):
    dd = _data(data)
    check(_lib.load().lq_pit_solve(*plan.dims(), C.byref(dd), _ptr(ws), _ptr(x), _ptr(u), _ptr(lam),
                                   _ptr(rel_res), _ptr(info), _stream(stream)), "lq_pit_solve")
