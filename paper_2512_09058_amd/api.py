"""Python binding of liblqkkt: marshals torch CUDA tensors and streams into the C ABI.

Every numerical step runs in the library's HIP kernels; this module only packs arguments.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence, Union

import numpy as np
import torch

from . import _lib
from ._lib import ARRAYS, LqData, LqLaunch, LqSolveOpts, MODES, check

INPUTS = ["A", "B", "Q", "R", "S", "q", "r", "f", "x0"]


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("lqkkt expects device tensors")
    if t.dtype != torch.float64 and t.dtype != torch.int32 and t.dtype != torch.uint8:
        raise ValueError(f"unexpected dtype {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("lqkkt expects contiguous tensors")
    return t.data_ptr()


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Plan:
    """Sizes, precision and kernel variant of a batch; owns the device descriptor table."""

    def __init__(self, N: Union[int, Sequence[int]], nx: Union[int, Sequence[int]],
                 nu: Union[int, Sequence[int]], batch: Optional[int] = None, mode: str = "f64",
                 ckpt_stride: int = 0):
        lib = _lib.load()
        if np.isscalar(N):
            if batch is None:
                raise ValueError("batch is required with scalar sizes")
            Ns = np.full(batch, N, np.int32)
            nxs = np.full(batch, nx, np.int32)
            nus = np.full(batch, nu, np.int32)
        else:
            Ns, nxs, nus = (np.ascontiguousarray(a, dtype=np.int32) for a in (N, nx, nu))
        self.batch = int(len(Ns))
        self.N, self.nx, self.nu = Ns, nxs, nus
        self.mode = mode
        self.ckpt_stride = int(ckpt_stride)
        self._h = C.c_void_p()
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))  # noqa: E731
        check(lib.lq_plan_create(self.batch, ip(Ns), ip(nxs), ip(nus), MODES[mode], int(ckpt_stride),
                                 C.byref(self._h)), "lq_plan_create")
        self._describe()

    def _describe(self):
        lib = _lib.load()
        self.workspace_bytes = int(lib.lq_plan_workspace_bytes(self._h))
        self.variant = lib.lq_plan_variant(self._h).decode()
        self.offsets: Dict[str, np.ndarray] = {}
        self.totals: Dict[str, int] = {}
        for i, name in enumerate(ARRAYS):
            offs = np.zeros(self.batch, np.int64)
            self.totals[name] = int(lib.lq_plan_offsets(self._h, i, offs.ctypes.data_as(C.POINTER(C.c_int64))))
            self.offsets[name] = offs

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().lq_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def subset(self, idx, mode: str = "f64", ckpt_stride: int = 0) -> "Plan":
        """lq_plan_create_subset: a plan over instances idx of this batch that reads and writes this
        plan's packed arrays (data and x, u, lam); its status arrays have len(idx) entries."""
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1))
        sub = Plan.__new__(Plan)
        sub._h = C.c_void_p()
        check(_lib.load().lq_plan_create_subset(self._h, int(idx.size), idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                                MODES[mode], int(ckpt_stride), C.byref(sub._h)),
              "lq_plan_create_subset")
        sub.batch = int(idx.size)
        sub.N, sub.nx, sub.nu = self.N[idx], self.nx[idx], self.nu[idx]
        sub.mode = mode
        sub.ckpt_stride = int(ckpt_stride)
        sub.parent_index = idx
        sub._describe()
        return sub

    def set_variant(self, name: str):
        """Select the factor kernel variant ("small", "small_padded", "tile" or "generic"; see
        lq_plan_set_variant)."""
        lib = _lib.load()
        check(lib.lq_plan_set_variant(self._h, name.encode()), "lq_plan_set_variant")
        self.variant = lib.lq_plan_variant(self._h).decode()

    @property
    def launch_groups(self) -> int:
        """Kernel-shape groups launched per call (see lq_plan_launch_groups)."""
        return int(_lib.load().lq_plan_launch_groups(self._h))

    def set_launch(self, threads: int = 128, persistent: int = 0, blocks_per_cu: int = 0):
        """Launch shape of the general-size kernels (see lq_plan_set_launch)."""
        c = LqLaunch(int(threads), int(persistent), int(blocks_per_cu), 0)
        check(_lib.load().lq_plan_set_launch(self._h, C.byref(c)), "lq_plan_set_launch")

    def get_launch(self) -> dict:
        c = LqLaunch()
        check(_lib.load().lq_plan_get_launch(self._h, C.byref(c)), "lq_plan_get_launch")
        return {"threads": c.threads, "persistent": c.persistent, "blocks_per_cu": c.blocks_per_cu}

    def signature(self) -> str:
        """Shape signature used as the autotuner's cache key."""
        import hashlib
        h = hashlib.sha1()
        for a in (self.N, self.nx, self.nu):
            h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
        return f"{self.mode}:{self.ckpt_stride}:{self.batch}:{h.hexdigest()[:16]}"

    def workspace(self, device=None) -> torch.Tensor:
        # torch's caching allocator returns 256-byte aligned blocks
        return torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=device or "cuda")

    def empty_outputs(self, device=None):
        dev = device or "cuda"
        return tuple(torch.empty(self.totals[k], dtype=torch.float64, device=dev) for k in ("x", "u", "lam"))


def _data(d: Dict[str, torch.Tensor]) -> LqData:
    return LqData(*[_ptr(d.get(k)) for k in INPUTS])


def factor(plan: Plan, data: Dict[str, torch.Tensor], ws: torch.Tensor, info: torch.Tensor, stream=None):
    lib = _lib.load()
    dd = _data(data)
    check(lib.lq_factor(plan.handle, C.byref(dd), _ptr(ws), _ptr(info), _stream(stream)), "lq_factor")


def solve(plan: Plan, data: Dict[str, torch.Tensor], ws: torch.Tensor, x, u, lam, rel_res=None, iters=None,
          info=None, tol: float = 1e-10, max_it: int = 0, check_res: bool = True, stream=None):
    lib = _lib.load()
    dd = _data(data)
    o = LqSolveOpts(float(tol), int(max_it), int(bool(check_res)))
    check(lib.lq_solve(plan.handle, C.byref(dd), _ptr(ws), C.byref(o), _ptr(x), _ptr(u), _ptr(lam),
                       _ptr(rel_res), _ptr(iters), _ptr(info), _stream(stream)), "lq_solve")


def solve_with_fallback(plan: Plan, data: Dict[str, torch.Tensor], ws: torch.Tensor, x, u, lam, rel_res, iters,
                        info, tol: float = 1e-10, max_it: int = 10, fallback_max_it: int = 2, stream=None) -> np.ndarray:
    """Factor + solve with the plan's precision, then factor and solve again in float64 every instance
    whose info is not 0 (a stage matrix that lost positive definiteness with float32 products, a
    refinement that stopped above tol, a non-finite residual).  The float64 subset plan reads the
    same data and writes x, u, lam in place; its info, rel_res and iters replace those of the
    instances it solved.  Returns the indices of those instances.  (Orchestration only: every step
    runs in the library's kernels; the one host synchronisation reads info.)"""
    factor(plan, data, ws, info, stream=stream)
    solve(plan, data, ws, x, u, lam, rel_res, iters, info, tol=tol, max_it=max_it, check_res=True, stream=stream)
    if isinstance(stream, torch.cuda.Stream):
        torch.cuda.current_stream().wait_stream(stream)
    bad = torch.nonzero(info != 0).reshape(-1).cpu().numpy().astype(np.int32)
    if bad.size == 0 or plan.mode == "f64":
        return bad[:0]
    sub = plan.subset(bad, "f64")
    ws2 = sub.workspace(device=info.device)
    dev = info.device
    info2 = torch.zeros(sub.batch, dtype=torch.int32, device=dev)
    rel2 = torch.zeros(sub.batch, dtype=torch.float64, device=dev)
    it2 = torch.zeros(sub.batch, dtype=torch.int32, device=dev)
    factor(sub, data, ws2, info2, stream=stream)
    solve(sub, data, ws2, x, u, lam, rel2, it2, info2, tol=tol, max_it=fallback_max_it, check_res=True, stream=stream)
    ib = torch.from_numpy(bad.astype(np.int64)).to(dev)
    info.index_copy_(0, ib, info2)
    if rel_res is not None:
        rel_res.index_copy_(0, ib, rel2)
    if iters is not None:
        iters.index_copy_(0, ib, it2)
    torch.cuda.synchronize(dev)  # the subset plan's workspace and tables are released on return
    return bad


def solve_backward(plan: Plan, data: Dict[str, torch.Tensor], ws: torch.Tensor, x, u, lam, gx, gu,
                   grads: Dict[str, torch.Tensor], rel_res=None, iters=None, info=None, tol: float = 1e-10,
                   max_it: int = 0, check_res: bool = True, stream=None):
    lib = _lib.load()
    dd = _data(data)
    o = LqSolveOpts(float(tol), int(max_it), int(bool(check_res)))
    g = [grads.get(k) for k in ("A", "B", "Q", "R", "S", "q", "r", "f", "x0")]
    check(lib.lq_solve_backward(plan.handle, C.byref(dd), _ptr(ws), C.byref(o), _ptr(x), _ptr(u), _ptr(lam),
                                _ptr(gx), _ptr(gu), *[_ptr(t) for t in g], _ptr(rel_res), _ptr(iters),
                                _ptr(info), _stream(stream)), "lq_solve_backward")


def factor_solve_noalloc(batch: int, N: int, nx: int, nu: int, data: Dict[str, torch.Tensor], x, u, lam,
                         rel_res=None, iters=None, info=None, mode: str = "f64", tol: float = 1e-10,
                         max_it: int = 0, check_res: bool = True, stream=None):
    """lq_factor_solve_noalloc: factor + solve of a uniform batch with the library's own device
    scratch array as workspace (no plan, no allocation; see the header for the size limit)."""
    lib = _lib.load()
    dd = _data(data)
    o = LqSolveOpts(float(tol), int(max_it), int(bool(check_res)))
    check(lib.lq_factor_solve_noalloc(int(batch), int(N), int(nx), int(nu), MODES[mode], C.byref(dd), C.byref(o),
                                      _ptr(x), _ptr(u), _ptr(lam), _ptr(rel_res), _ptr(iters), _ptr(info),
                                      _stream(stream)), "lq_factor_solve_noalloc")


# ---------------------------------------------------------------------------------------------
# Packing of problems into the boundary layout (instance blocks back to back, row-major).

def pack(problems, device="cuda", with_S=None, with_f=None) -> Dict[str, torch.Tensor]:
    """Pack an LQProblem batch (uniform) or a list of instances into device float64 arrays."""
    if hasattr(problems, "batched") and problems.batched:
        p = problems
        out = {}
        for k in INPUTS:
            a = getattr(p, k)
            if a is None:
                continue
            out[k] = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to(device)
        return out
    insts = problems if isinstance(problems, (list, tuple)) else [problems]
    out = {}
    for k in INPUTS:
        vals = [getattr(p, k) for p in insts]
        if all(v is None for v in vals):
            continue
        flat = []
        for p, v in zip(insts, vals):
            if v is None:
                shape = {"S": (p.N, p.nu, p.nx), "f": (p.N, p.nx)}[k]
                v = np.zeros(shape)
            flat.append(np.ascontiguousarray(v, dtype=np.float64).reshape(-1))
        out[k] = torch.from_numpy(np.concatenate(flat)).to(device)
    return out


def unpack(plan: Plan, name: str, flat: torch.Tensor, i: int) -> np.ndarray:
    """Instance i's block of output or input array `name` as (stages, dim) numpy array."""
    N, nx, nu = int(plan.N[i]), int(plan.nx[i]), int(plan.nu[i])
    shapes = {"x": (N, nx), "u": (N, nu), "lam": (N, nx), "A": (N, nx, nx), "B": (N, nx, nu),
              "Q": (N + 1, nx, nx), "R": (N, nu, nu), "S": (N, nu, nx), "q": (N + 1, nx), "r": (N, nu),
              "f": (N, nx), "x0": (nx,)}
    shp = shapes[name]
    n = int(np.prod(shp))
    o = int(plan.offsets[name][i])
    return flat[o:o + n].detach().cpu().numpy().reshape(shp)


def capture(plan: Plan, data: Dict[str, torch.Tensor], ws: torch.Tensor, x, u, lam, rel_res=None, iters=None,
            info=None, tol: float = 1e-10, max_it: int = 0, check_res: bool = True, warmup: int = 1):
    """Capture lq_factor + lq_solve on a side stream into a HIP graph (torch.cuda.CUDAGraph);
    replay() re-runs the whole sequence on the captured buffers.  The calls only enqueue kernels
    (work counters are reset by a kernel, not a memset), so nothing else lands in the graph.

    The graph's kernels read the plan's device tables and the given buffers by address, so the
    returned graph holds references to all of them (`g.lq_keepalive`): the plan and the buffers
    live at least as long as the graph."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(warmup):
            factor(plan, data, ws, info, stream=s)
            solve(plan, data, ws, x, u, lam, rel_res, iters, info, tol=tol, max_it=max_it, check_res=check_res,
                  stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        st = torch.cuda.current_stream()
        factor(plan, data, ws, info, stream=st)
        solve(plan, data, ws, x, u, lam, rel_res, iters, info, tol=tol, max_it=max_it, check_res=check_res,
              stream=st)
    g.lq_keepalive = (plan, data, ws, x, u, lam, rel_res, iters, info)
    return g
