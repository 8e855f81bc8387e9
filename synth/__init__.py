"""Seeded synthetic LQ optimal-control problems.

This module only draws input data (dynamics, costs, initial states) from
seeded random-number streams.  It contains none of the solver's arithmetic
and is shared by the CPU oracle, the tests and the benchmark.
"""
from .problems import (  # noqa: F401
    LQProblem,
    SEED_ROOT,
    config_sizes,
    make_batch,
    make_batch_parallel,
    make_instance,
    make_ragged,
    random_problem,
    stack,
)
from .blocktri import random_blocktri  # noqa: F401
from .update import random_update_rows  # noqa: F401
from .massspring import mass_spring  # noqa: F401
