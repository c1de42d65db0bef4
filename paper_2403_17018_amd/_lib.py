"""ctypes declarations of libhenry's C ABI (include/henry.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhenry.so")

HENRY_OK, HENRY_EINVAL, HENRY_EDEVICE, HENRY_ENOMEM, HENRY_EUNSUPPORTED = 0, -1, -2, -3, -4
EXPORTS = ("henry_problem_default", "henry_solver_opts_default", "henry_ctx_create", "henry_ctx_destroy",
           "henry_last_error", "henry_sample_fields", "henry_solve_batch", "henry_adjoint_batch",
           "mlmc_estimate", "mlmc_optimal_samples", "henry_autotune", "henry_profile", "henry_profile_read",
           "mlmc_estimate_series", "mlmc_plan", "mlmc_estimate_noalloc", "henry_assemble", "henry_jacobian_apply",
           "henry_gs_pass", "henry_coarse_solve", "henry_vc_solve", "henry_vc_solve_batch", "henry_vc_assemble")
PROF_CLASSES = ("assemble", "gs", "spmv", "restrict", "prolong", "band_factor", "band_solve", "dense_factor",
                "dense_solve", "host_sync")


class henry_problem(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("Lx", "Ly", "T", "rho0", "rho1", "mu", "g", "Dm", "phi_mean", "phi_amp",
                                           "phi_min", "phi_max", "K_mean", "logK_amp", "corr_len", "q_in",
                                           "q_in_amp")] + [
        ("n_kl_phi", C.c_int), ("n_kl_logK", C.c_int), ("right_c_dirichlet", C.c_int), ("c_left", C.c_double),
        ("field_model", C.c_int), ("kappa_kc", C.c_double), ("recharge_omega", C.c_double),
        ("qoi_xmin", C.c_double)]


class henry_grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nsteps", C.c_int)]


class henry_solver_opts(C.Structure):
    _fields_ = [("mg_precision", C.c_int), ("coarse_nx", C.c_int), ("coarse_ny", C.c_int), ("nu_pre", C.c_int),
                ("nu_post", C.c_int), ("newton_tol", C.c_double), ("newton_dc_max", C.c_double),
                ("newton_maxit", C.c_int), ("krylov_rtol", C.c_double), ("krylov_maxit", C.c_int),
                ("c_range_tol", C.c_double), ("use_graphs", C.c_int), ("red_blocks", C.c_int),
                ("krylov_rtol_adjoint", C.c_double), ("newton_extrapolate", C.c_int),
                ("newton_predict", C.c_double),
                ("newton_jac_reuse", C.c_double),
                ("mg_cycle", C.c_int),
                ("adjoint_guess", C.c_int),
                ("coarse_solver", C.c_int),
                ("step_graphs", C.c_int),
                ("ragged_threads", C.c_int),
                ("sample_block", C.c_int),
                ("fuse_prolong", C.c_int),
                ("krylov_breakdown", C.c_double)]


class henry_batch(C.Structure):
    _fields_ = [("grid", henry_grid), ("nsamples", C.c_int), ("theta", C.c_void_p), ("c_T", C.c_void_p),
                ("p_T", C.c_void_p), ("qoi", C.c_void_p), ("status", C.c_void_p), ("stats", C.c_void_p),
                ("series", C.c_void_p)]

NSERIES = 17   # HENRY_NSERIES: Q_S, Q_FW, Q_1..Q_15


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libhenry.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2403_17018_amd.build`")
    lib = C.CDLL(path)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    P = C.POINTER
    lib.henry_problem_default.argtypes = [P(henry_problem)]
    lib.henry_problem_default.restype = None
    lib.henry_solver_opts_default.argtypes = [P(henry_solver_opts)]
    lib.henry_solver_opts_default.restype = None
    lib.henry_ctx_create.argtypes = [P(vp), i, vp]
    lib.henry_ctx_create.restype = i
    lib.henry_ctx_destroy.argtypes = [vp]
    lib.henry_ctx_destroy.restype = None
    lib.henry_last_error.argtypes = [vp]
    lib.henry_last_error.restype = C.c_char_p
    lib.henry_sample_fields.argtypes = [vp, P(henry_problem), henry_grid, i, vp, vp, vp, vp]
    lib.henry_sample_fields.restype = i
    lib.henry_solve_batch.argtypes = [vp, P(henry_problem), P(henry_solver_opts), P(henry_batch), i]
    lib.henry_solve_batch.restype = i
    lib.henry_adjoint_batch.argtypes = [vp, P(henry_problem), P(henry_solver_opts), henry_grid, i, vp, i, vp, vp, vp]
    lib.henry_adjoint_batch.restype = i
    lib.mlmc_estimate.argtypes = [vp, i, P(i), P(henry_grid), P(vp), P(vp), P(vp), P(vp), d, P(d), P(d), P(d), P(d),
                                  vp, vp]
    lib.mlmc_estimate.restype = i
    lib.mlmc_estimate_noalloc.argtypes = lib.mlmc_estimate.argtypes
    lib.mlmc_estimate_noalloc.restype = i
    lib.mlmc_optimal_samples.argtypes = [i, P(d), P(d), d, P(C.c_longlong), P(d)]
    lib.mlmc_optimal_samples.restype = i
    lib.henry_autotune.argtypes = [vp, P(henry_problem), P(henry_solver_opts), henry_grid, i, vp, P(d)]
    lib.henry_autotune.restype = i
    lib.henry_profile.argtypes = [vp, i]
    lib.henry_profile.restype = i
    lib.henry_profile_read.argtypes = [vp, i, P(C.c_longlong), P(C.c_longlong), P(d)]
    lib.henry_profile_read.restype = i
    lib.mlmc_estimate_series.argtypes = [vp, i, P(i), P(henry_grid), i, P(vp), P(vp), vp, vp, vp, vp]
    lib.mlmc_estimate_series.restype = i
    lib.mlmc_plan.argtypes = [i, P(d), P(d), P(d), d, d, i, P(C.c_longlong), P(d), P(d)]
    lib.mlmc_plan.restype = i
    lib.henry_assemble.argtypes = [vp, P(henry_problem), henry_grid, i, vp, vp, vp, vp, i, vp, vp]
    lib.henry_assemble.restype = i
    lib.henry_jacobian_apply.argtypes = [vp, henry_grid, i, vp, vp, vp, i]
    lib.henry_jacobian_apply.restype = i
    lib.henry_gs_pass.argtypes = [vp, henry_grid, i, vp, vp, vp, i, i]
    lib.henry_gs_pass.restype = i
    lib.henry_coarse_solve.argtypes = [vp, i, i, henry_grid, i, vp, vp, vp, i]
    lib.henry_coarse_solve.restype = i
    lib.henry_vc_solve.argtypes = [vp, P(henry_problem), P(henry_solver_opts), henry_grid, i, vp, vp, vp, vp, vp, vp]
    lib.henry_vc_solve.restype = i
    lib.henry_vc_solve_batch.argtypes = [vp, P(henry_problem), P(henry_solver_opts), P(henry_batch), i]
    lib.henry_vc_solve_batch.restype = i
    lib.henry_vc_assemble.argtypes = [vp, P(henry_problem), henry_grid, i, vp, vp, vp, vp, i, vp, vp]
    lib.henry_vc_assemble.restype = i
    _lib = lib
    return lib
