"""Seeded synthetic LP generators with planted primal-dual optima.

This module produces inputs only. It holds none of the solver's arithmetic:
no scaling, no PDHG step, no learner, no KKT evaluation. Both the oracle's
tests and the GPU path's tests and benchmarks draw their problems from here,
so the two sides see bit-identical inputs for a given seed.

The LP form is the general one the solver accepts (the paper's standard form,
Section 2, eq. (1), widened to two-sided variable bounds and mixed
equality / greater-or-equal rows):

    min  c^T x + obj_offset
    s.t. A_i x  = b_i   (row_sense[i] == 0)
         A_i x >= b_i   (row_sense[i] == 1)
         l <= x <= u    (entries of l may be -inf, of u +inf)
"""

from .generators import (  # noqa: F401
    LP,
    PlantedLP,
    config_lp,
    config_names,
    random_lp,
    plant_optimum,
    tiny_lp,
    block_angular_lp,
    batch_lps,
    serving_requests,
    study_lps,
)
