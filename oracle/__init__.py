"""CPU oracle for the stencil sweep and temporal computation folding.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the library's product path never does,
and this package imports nothing from the library.  It computes, slowly and
plainly, what the paper defines; see ``oracle.core`` for each function's
citation and ``oracle/stencil_oracle.c`` for the sweep itself.
"""

from .core import (  # noqa: F401
    available,
    num_threads,
    sweep,
    sweep_f32,
    sweep_window,
    sweep_spectral,
    fold_weights,
    fold_weights_f32,
    bf16_rne,
    bf16_split,
    schedule,
    folded_reference_f32,
    band_mask,
    dirichlet_folded,
    floor_sweep,
    life,
    errors,
    exact_sum,
    collect_counts,
)
