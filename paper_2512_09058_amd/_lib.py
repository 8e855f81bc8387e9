"""ctypes declarations of the C ABI in include/lqkkt.h (loaded from the in-tree liblqkkt.so)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblqkkt.so")

LQ_OK, LQ_EINVAL, LQ_EUNSUPPORTED, LQ_EHIP, LQ_ENOMEM = 0, -1, -2, -3, -4
LQ_INFO_NONFINITE, LQ_INFO_NOT_CONVERGED = -1, -2
MODES = {"f64": 0, "mixed_f32": 1, "mixed_bf16": 2}
ARRAYS = ["A", "B", "Q", "R", "S", "q", "r", "f", "x0", "x", "u", "lam"]


class LqData(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("A", "B", "Q", "R", "S", "q", "r", "f", "x0")]


class LqLaunch(C.Structure):
    _fields_ = [("threads", C.c_int32), ("persistent", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("reserved", C.c_int32)]


class LqSolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_it", C.c_int32), ("check", C.c_int32)]


EXPORTS = {
    "lq_version": (C.c_int, []),
    "lq_last_error": (C.c_char_p, []),
    "lq_plan_create": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), C.c_int, C.c_int32, C.POINTER(C.c_void_p)]),
    "lq_plan_destroy": (None, [C.c_void_p]),
    "lq_plan_create_subset": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int, C.c_int32,
                                        C.POINTER(C.c_void_p)]),
    "lq_plan_workspace_bytes": (C.c_size_t, [C.c_void_p]),
    "lq_plan_offsets": (C.c_int64, [C.c_void_p, C.c_int, C.POINTER(C.c_int64)]),
    "lq_plan_variant": (C.c_char_p, [C.c_void_p]),
    "lq_plan_set_variant": (C.c_int, [C.c_void_p, C.c_char_p]),
    "lq_plan_launch_groups": (C.c_int, [C.c_void_p]),
    "lq_plan_set_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lq_plan_get_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lq_factor": (C.c_int, [C.c_void_p, C.POINTER(LqData), C.c_void_p, C.c_void_p, C.c_void_p]),
    "lq_solve": (C.c_int, [C.c_void_p, C.POINTER(LqData), C.c_void_p, C.POINTER(LqSolveOpts)]
                 + [C.c_void_p] * 6 + [C.c_void_p]),
    "lq_solve_backward": (C.c_int, [C.c_void_p, C.POINTER(LqData), C.c_void_p, C.POINTER(LqSolveOpts)]
                          + [C.c_void_p] * 17 + [C.c_void_p]),
    "lq_factor_solve_noalloc": (C.c_int, [C.c_int32] * 4 + [C.c_int, C.POINTER(LqData), C.POINTER(LqSolveOpts)]
                                + [C.c_void_p] * 6 + [C.c_void_p]),
    # block-tridiagonal solvers (include/lqblocktri.h)
    "lq_bt_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32, C.c_int]),
    "lq_bt_cr_factor": (C.c_int, [C.c_int32] * 3 + [C.c_void_p] * 4 + [C.c_void_p]),
    "lq_bt_cr_solve": (C.c_int, [C.c_int32] * 3 + [C.c_void_p] * 3 + [C.c_void_p]),
    "lq_bt_pcr_solve": (C.c_int, [C.c_int32] * 3 + [C.c_void_p] * 6 + [C.c_void_p]),
    "lq_bt_pcg": (C.c_int, [C.c_int32] * 3 + [C.c_void_p] * 4 + [C.c_int32, C.c_double, C.c_int32]
                  + [C.c_void_p] * 4 + [C.c_void_p]),
    # factorisation updates (include/lqupdate.h)
    "lq_update_data": (C.c_int, [C.c_void_p, C.c_void_p] + [C.c_void_p] * 3 + [C.c_void_p]),
    "lq_update_max_columns": (C.c_int32, [C.c_void_p]),
    "lq_update_workspace_bytes": (C.c_size_t, [C.c_void_p]),
    "lq_factor_update": (C.c_int, [C.c_void_p, C.POINTER(LqData)] + [C.c_void_p] * 5),
    # box-constrained QPs (include/lqqp.h)
    "lq_qp_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int32, C.c_int32]),
    "lq_qp_solve": (C.c_int, [C.c_void_p, C.POINTER(LqData)] + [C.c_void_p] * 10 + [C.c_void_p]),
    # parallel-in-time solve (include/lqpit.h)
    "lq_pit_workspace_bytes": (C.c_size_t, [C.c_int32] * 5),
    "lq_pit_factor": (C.c_int, [C.c_int32] * 5 + [C.POINTER(LqData), C.c_void_p, C.c_void_p, C.c_void_p]),
    "lq_pit_solve": (C.c_int, [C.c_int32] * 5 + [C.POINTER(LqData)] + [C.c_void_p] * 6 + [C.c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load liblqkkt.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2512_09058_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int, what: str):
    if rc != LQ_OK:
        msg = load().lq_last_error().decode()
        raise RuntimeError(f"{what} failed with status {rc}: {msg}")
