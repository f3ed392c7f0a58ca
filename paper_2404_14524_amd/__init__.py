"""MI355X (gfx950) implementation of the hot path of Nys-IP-PMM (randomized
Nystrom preconditioned IP-PMM, arXiv 2404.14524) for separable convex QPs.

The compute lives in libnysipm.so (HIP kernels behind the C ABI declared in
include/nysipm.h); ``nysipm`` is its ctypes binding and ``autograd`` wraps
the solver and its adjoint in a torch.autograd.Function.
"""

from .nysipm import (NysError, Precond, ipm_adjoint, ipm_solve, load_library, nys_last_timing, nys_sketch_product,
                     nys_profile_enable, nys_profile_read, nys_stream_read,
                     nys_newton_solve, nys_normal_apply, nys_pcg_solve, nys_pcg_solve_noalloc, nys_precond_apply,
                     nys_sketch, nys_sketch_tiles, nys_sketch_tiles_bytes, nys_test_matrix, nys_transpose, PChol, nys_pchol_build, nys_pchol_apply,
                     ipm_solve_box, VAR_NONNEG, VAR_FREE, VAR_BOX, nys_deff_estimate,
                     nys_sketch_size_rule, nys_precond_rebuild_due, ELL_RULES, TRACE_FIELDS)

__all__ = ["NysError", "Precond", "ipm_adjoint", "ipm_solve", "load_library", "nys_last_timing",
           "nys_newton_solve", "nys_normal_apply", "nys_pcg_solve", "nys_pcg_solve_noalloc", "nys_precond_apply",
           "nys_sketch", "nys_sketch_product", "nys_sketch_tiles", "nys_sketch_tiles_bytes", "nys_test_matrix", "nys_profile_enable",
           "nys_profile_read", "nys_stream_read", "nys_transpose", "PChol", "nys_pchol_build",
           "nys_pchol_apply", "ipm_solve_box", "VAR_NONNEG", "VAR_FREE", "VAR_BOX", "nys_deff_estimate",
           "nys_sketch_size_rule", "nys_precond_rebuild_due", "ELL_RULES", "TRACE_FIELDS"]
