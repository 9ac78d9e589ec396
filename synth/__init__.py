"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package holds only random-number generation and the workload recipes
(shapes, value distributions, which stencil a batched grid gets).  It holds
none of the stencil arithmetic: no sweep, no folding, no rounding of folded
weights.  Both the oracle (test infrastructure) and the product's tests and
benchmark draw their inputs from here, so the two sides see identical bits.
"""

from .splitmix import splitmix64, uniform_f64, uniform_f32, u64_stream  # noqa: F401
from .workloads import (  # noqa: F401
    SEED,
    STREAM_GRID,
    STREAM_WEIGHTS,
    STREAM_BATCH_SIDES,
    STREAM_BATCH_KIND,
    STREAM_BATCH_WEIGHTS,
    Workload,
    WORKLOADS,
    grid_f32,
    grid_f64,
    random_positive_weights,
    heat1d_weights,
    star2d_weights,
    star3d_weights,
    to_f32_exact,
    batched_recipe,
    star_mask,
    STAR,
    BOX,
    APOP,
    LIFE,
    apop_payoff,
    life_cells,
)
