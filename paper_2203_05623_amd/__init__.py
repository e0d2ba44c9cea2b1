"""MI355X-native batched Sternheimer solver (hot path of full-frequency GW, arXiv 2203.05623).

The computation lives in the HIP library ``libsth.so`` (C-ABI in include/sth.h);
``paper_2203_05623_amd._lib`` is its thin ctypes binding with the same names.
"""
from . import _lib
from ._lib import (SOLVE_BREAKDOWN, SOLVE_CONVERGED, SOLVE_MAXIT, SOLVE_NAN, STH_E_AGAIN,
                   STH_E_DEVICE, STH_E_INTERNAL, STH_E_INVALID, STH_E_NOMEM, STH_E_NOT_FOUND,
                   STH_E_NOT_READY, STH_FP64, STH_MIXED, STH_MIXED_BF16, SthError, sth_apply_h, sth_apply_h_noalloc, sth_chi0_block,
                   sth_create, sth_destroy, sth_fetch_drho, sth_fetch_dpsi, sth_fetch_stats,
                   sth_lanczos, sth_last_error, sth_pdep, sth_poll, sth_profile,
                   sth_profile_read, sth_release_system, sth_release_ticket, sth_set_system,
                   sth_submit_solves, sth_system_info_get, sth_valence, sth_wait)

__all__ = ["SOLVE_BREAKDOWN", "SOLVE_CONVERGED", "SOLVE_MAXIT", "SOLVE_NAN", "STH_E_AGAIN",
           "STH_E_DEVICE", "STH_E_INTERNAL", "STH_E_INVALID", "STH_E_NOMEM", "STH_E_NOT_FOUND",
           "STH_E_NOT_READY", "STH_FP64", "STH_MIXED", "STH_MIXED_BF16", "SthError", "sth_apply_h", "sth_apply_h_noalloc",
           "sth_chi0_block", "sth_create", "sth_destroy", "sth_fetch_drho", "sth_fetch_dpsi",
           "sth_fetch_stats", "sth_lanczos", "sth_last_error", "sth_pdep", "sth_poll",
           "sth_profile", "sth_profile_read", "sth_release_system", "sth_release_ticket",
           "sth_set_system", "sth_submit_solves", "sth_system_info_get", "sth_valence",
           "sth_wait", "_lib"]
