"""MI355X (gfx950) implementation of the two-sided sketched numerical-rank
estimator of Meier & Nakatsukasa (arXiv 2105.07388, Algorithm 1).

The estimator runs entirely in the HIP library ``librankest.so`` (C ABI in
include/rankest.h); this package only marshals arguments.  Importing it does not
load the library; the first call does, and raises ``RankEstError`` if the
library has not been built.
"""
from ._binding import (  # noqa: F401
    FLAG_NOT_CONVERGED,
    FLAG_PREC_FALLBACK,
    FLAG_USED_BF16,
    FLAG_USED_FP16,
    FLAG_COLUMNS_DROPPED,
    FLAG_PREC_BELOW_FLOOR,
    FLAG_SVD_RELAUNCHED,
    FLAG_ZERO,
    Handle,
    close_all_handles,
    RankEstError,
    default_handle,
    gap_rank,
    gauss_fill,
    lib,
    make_blocks,
    mlp_adam,
    mlp_forward,
    mlp_loss_grad,
    philox,
    project,
    r1_from_k,
    rangefinder,
    rangefinder_stage_ms,
    rank_adaptive,
    rank_count,
    rank_estimate,
    rank_estimate_batched,
    rank_estimate_qr,
    rank_gap,
    singular_values,
    singular_values_noalloc,
    sketch_x,
    sketch_y,
    srht_select,
    srht_signs,
    thin_qr,
)
