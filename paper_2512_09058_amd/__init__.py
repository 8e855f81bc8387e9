"""Batched factorised-Riccati LQ KKT solver on AMD MI355X (gfx950).

The compute path is the HIP library liblqkkt.so (C ABI in include/lqkkt.h); this package is
its thin Python binding.  Import fails loudly at call time if the library was not built.
"""
from .api import Plan, factor, pack, solve, solve_backward, unpack  # noqa: F401
