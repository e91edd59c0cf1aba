"""MI355X-native Parallel Coordinate Descent Newton (PCDN) for L1-regularised
logistic regression and L1-regularised L2-loss SVM.

The method (Bian, Li, Liu, Yang, arXiv:1306.4080) runs in the HIP library
``libpcdn.so`` built for gfx950 from ``csrc/``; its C ABI is ``include/pcdn.h``
and ``binding`` marshals Python arguments into it.  Nothing here computes the
method in Python and there is no CPU fallback.
"""
import os

from .binding import (LOSSES, PCDN_LOSS_L2SVM, PCDN_LOSS_LOGISTIC, PcdnError, Server, Solver,  # noqa: F401
                      load_library, pcdn_create, pcdn_destroy, pcdn_evaluate, pcdn_get_cache,
                      pcdn_get_w, pcdn_iterate, pcdn_last_error, pcdn_load_csc, pcdn_load_csc_bias, pcdn_permutation, pcdn_profile,
                      pcdn_autotune, pcdn_profile_read, pcdn_reset, pcdn_solve, pcdn_solve_batch,
                      pcdn_solve_path, pcdn_solve_path_lanes, pcdn_solve_static, pcdn_step, solve_batch, pcdn_iterate_batch, iterate_batch)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpcdn.so")


def ensure_built() -> str:
    """Build libpcdn.so when it is missing or was built from other sources
    (its stamp holds the SHA-256 of the sources, headers and compile
    command)."""
    from . import build
    if build.is_stale():
        build.build()
    return LIB_PATH
