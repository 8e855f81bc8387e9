"""Python binding of the batched block-tridiagonal solvers (include/lqblocktri.h): argument
marshalling only; CR, PCR and PCG run in the library's HIP kernels.

Arrays are CUDA float64 tensors: M [batch, Nb, n, n], K [batch, Nb-1, n, n], b [batch, Nb, n].
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import check

METHODS = {"cr": 0, "pcr": 1, "pcg": 2}
PRECOND = {"jacobi": 0, "stair": 1}


def _p(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if t.dtype not in (torch.float64, torch.int32, torch.uint8):
        raise ValueError(f"unexpected dtype {t.dtype}")
    return t.data_ptr()


def _s(stream):
    return (torch.cuda.current_stream() if stream is None else stream).cuda_stream


def _dims(M):
    if M.dim() != 4 or M.shape[2] != M.shape[3]:
        raise ValueError("M must be [batch, Nb, n, n]")
    return int(M.shape[0]), int(M.shape[1]), int(M.shape[2])


def workspace(batch, Nb, n, method, device="cuda"):
    nbytes = int(_lib.load().lq_bt_workspace_bytes(batch, Nb, n, METHODS[method]))
    return torch.empty(max(nbytes, 8), dtype=torch.uint8, device=device)


def cr_factor(M, K, ws=None, info=None, stream=None):
    """Cyclic-reduction factorisation; returns (ws, info) -- ws holds the factors."""
    batch, Nb, n = _dims(M)
    ws = workspace(batch, Nb, n, "cr", M.device) if ws is None else ws
    info = torch.empty(batch, dtype=torch.int32, device=M.device) if info is None else info
    check(_lib.load().lq_bt_cr_factor(batch, Nb, n, _p(M), _p(K) if Nb > 1 else None, _p(ws), _p(info), _s(stream)),
          "lq_bt_cr_factor")
    return ws, info


def cr_solve(batch, Nb, n, ws, b, x=None, stream=None):
    x = torch.empty_like(b) if x is None else x
    check(_lib.load().lq_bt_cr_solve(batch, Nb, n, _p(ws), _p(b), _p(x), _s(stream)), "lq_bt_cr_solve")
    return x


def cr_views(ws, batch, Nb, n):
    """(L, U, Y) factor blocks of a CR workspace as [batch, Nb, n, n] views."""
    blocks = batch * Nb * n * n
    w = ws[: 4 * blocks * 8].view(torch.float64)
    return tuple(w[i * blocks:(i + 1) * blocks].view(batch, Nb, n, n) for i in (0, 2, 3))


def pcr_solve(M, K, b, x=None, ws=None, info=None, stream=None):
    batch, Nb, n = _dims(M)
    ws = workspace(batch, Nb, n, "pcr", M.device) if ws is None else ws
    info = torch.empty(batch, dtype=torch.int32, device=M.device) if info is None else info
    x = torch.empty_like(b) if x is None else x
    check(_lib.load().lq_bt_pcr_solve(batch, Nb, n, _p(M), _p(K) if Nb > 1 else None, _p(b), _p(x), _p(ws),
                                      _p(info), _s(stream)), "lq_bt_pcr_solve")
    return x, info


def pcg(M, K, b, precond="stair", tol=1e-12, max_it=1000, x=None, ws=None, iters=None, rel_res=None, info=None,
        stream=None):
    batch, Nb, n = _dims(M)
    dev = M.device
    ws = workspace(batch, Nb, n, "pcg", dev) if ws is None else ws
    x = torch.empty_like(b) if x is None else x
    iters = torch.empty(batch, dtype=torch.int32, device=dev) if iters is None else iters
    rel_res = torch.empty(batch, dtype=torch.float64, device=dev) if rel_res is None else rel_res
    info = torch.empty(batch, dtype=torch.int32, device=dev) if info is None else info
    check(_lib.load().lq_bt_pcg(batch, Nb, n, _p(M), _p(K) if Nb > 1 else None, _p(b), _p(x), PRECOND[precond],
                                float(tol), int(max_it), _p(ws), _p(iters), _p(rel_res), _p(info), _s(stream)),
          "lq_bt_pcg")
    return x, iters, rel_res, info
