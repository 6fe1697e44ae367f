"""MI355X-native Momentum Iterative Hessian Sketch (M-IHS) for tall ridge regression.

The solver lives in libmihs.so (hand-written HIP for gfx950, C ABI in
include/mihs.h); this package is its thin Python binding.  torch tensors supply
device memory and the current HIP stream.

    import paper_1912_03514_amd as mihs
    SA = mihs.mihs_sketch(A, "srht", m, seed)              # Lemma 3 sketches
    alpha, beta = mihs.momentum(sd, m)                      # Corollary 4
    x, info = mihs.mihs_solve(A, b, lam, SA, alpha, beta)  # Algorithm 1
"""
from ._binding import (  # noqa: F401
    EXPORTED, INFO_BYTES, LIB_PATH, BatchedSolver, MihsError, SolveWorkspace, handle,
    batched_schedule, info_to_dict, sketch_workspace_bytes,
    load_library, mihs_estimate_sd, mihs_sketch, mihs_sketch_two_stage, mihs_solve,
    mihs_solve_backward, mihs_solve_batched, mihs_solve_dual, mihs_solve_multi, mihs_solve_pd,
    mihs_solve_pd_dual, mihs_transpose, MIHSRidge, momentum, momentum_thm1, lambda_from_log,
    release_all, mihs_solve_noalloc, NOALLOC_SCRATCH_BYTES, tuning_cache_save,
    tuning_cache_load, row_weights, set_row_weights, calibrate_rows, row_split,
)
