"""ctypes mirror of include/ocp_admm.h (argument marshalling only).

The shared library is loaded from this package directory; there is no
fallback: if it is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

from .build import LIB_PATH

OCP_OK, OCP_E_ARG, OCP_E_SHAPE, OCP_E_HIP, OCP_E_NOMEM, OCP_E_ORDER, OCP_E_UNSUPPORTED, OCP_E_SCRATCH = range(8)
NOALLOC_SCRATCH_BYTES = 64 << 20
MODEL_QP, MODEL_LTI, MODEL_BICYCLE = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
ROW_HARD, ROW_L2, ROW_L1 = 0, 1, 2
SOLVED, MAX_ITER, NON_FINITE, FACTOR_BREAKDOWN, INFEASIBLE = 0, 1, 2, 3, 4
ADJ_OK, ADJ_RESIDUAL, ADJ_NON_FINITE, ADJ_BREAKDOWN = 0, 1, 2, 3
ADJ_LAST_QP, ADJ_SQP_GN, ADJ_SQP_EXACT = 0, 1, 2
LINSOLVE_DIRECT, LINSOLVE_PCG = 0, 1

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class ocp_dims(C.Structure):
    _fields_ = [("batch", C.c_int32), ("nx", C.c_int32), ("nu", C.c_int32), ("ng", C.c_int32),
                ("model", C.c_int32), ("precision", C.c_int32), ("time_invariant", C.c_int32)]


class ocp_settings(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "sigma", "rho0", "rho_f_scale", "rho_min", "rho_max", "k_ratio", "alpha", "eps_abs", "eps_rel",
        "eps_c", "armijo_eta", "eps_active", "adj_sigma", "adj_rho", "adj_tol", "eps_pinf")] + [(k, C.c_int32) for k in (
            "max_admm", "k_rho", "k_check", "adapt_rho", "warm_start", "max_sqp", "fixed_sqp", "refine_sweeps",
            "adj_mode")]


class ocp_lti(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("A", "Bm", "Qd", "Rd", "Qfd", "G", "lo", "hi", "x0")]


class ocp_qp(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("D", "E", "q", "Am", "Ap", "b", "G", "lo", "hi", "x_init", "soft")] + [
        ("gamma2", C.c_double), ("gamma1", C.c_double)]


class ocp_bicycle(C.Structure):
    _fields_ = [("ref", C.c_void_p), ("normal", C.c_void_p), ("x0", C.c_void_p)] + [
        (k, C.c_double) for k in ("dt", "wheelbase", "a_bound", "steer_bound", "lat_bound", "gamma1")] + [
        ("Qd", C.c_double * 4), ("Rd", C.c_double * 2), ("Qfd", C.c_double * 4), ("integrator", C.c_int32),
        ("Wd", C.c_double * 2), ("u_init", C.c_void_p)]


class ocp_solution(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in (
        "x", "xi", "z_g", "y_f", "y_g", "status", "admm_iters", "sqp_iters", "n_factor",
        "r_prim", "r_dual", "rho", "sqp_kkt")]


class ocp_qp_grads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("d_q", "d_Ddiag", "d_x_init", "d_lo", "d_hi", "eta_x", "active",
                                          "d_gamma2", "eta_f", "eta_g", "adj_resid", "adj_status", "eta_xi",
                                          "d_gamma1")]


# (name, restype, argtypes) for every symbol declared in include/ocp_admm.h
K_FACTOR, K_ITER, K_CHECK, K_ADJOINT, K_SQP, K_OTHER, K_SOLVE, K_COUNT = range(8)
K_NAMES = ("factor", "iter", "check", "adjoint", "sqp", "other", "solve")


class ocp_kernel_times(C.Structure):
    _fields_ = [("ms", C.c_double * K_COUNT), ("launches", C.c_int64 * K_COUNT)]


SIGNATURES = [
    ("ocp_default_settings", None, [C.POINTER(ocp_settings)]),
    ("ocp_status_string", C.c_char_p, [C.c_int]),
    ("ocp_supported", C.c_int32, [C.c_int32, C.c_int32, C.c_int32]),
    ("ocp_workspace_bytes", C.c_int, [C.POINTER(ocp_dims), _ip, C.POINTER(C.c_size_t)]),
    ("ocp_create", C.c_int, [C.POINTER(ocp_dims), _ip, C.POINTER(C.c_void_p)]),
    ("ocp_destroy", C.c_int, [C.c_void_p]),
    ("ocp_set_lti", C.c_int, [C.c_void_p, C.POINTER(ocp_lti), C.c_void_p]),
    ("ocp_set_qp", C.c_int, [C.c_void_p, C.POINTER(ocp_qp), C.c_void_p]),
    ("ocp_set_bicycle", C.c_int, [C.c_void_p, C.POINTER(ocp_bicycle), C.c_void_p]),
    ("ocp_solve", C.c_int, [C.c_void_p, C.POINTER(ocp_settings), C.POINTER(ocp_solution), C.c_void_p]),
    ("ocp_get_solution", C.c_int, [C.c_void_p, C.POINTER(ocp_solution), C.c_void_p]),
    ("ocp_adjoint", C.c_int, [C.c_void_p, C.POINTER(ocp_settings), C.c_void_p, C.c_void_p, C.POINTER(ocp_qp_grads),
                              C.c_void_p]),
    ("ocp_profile", C.c_int, [C.c_void_p, C.c_int32]),
    ("ocp_graph_capture", C.c_int, [C.c_void_p, C.POINTER(ocp_settings), C.POINTER(ocp_solution), C.c_void_p,
                                    C.c_void_p,
                                    C.POINTER(ocp_qp_grads), C.c_void_p]),
    ("ocp_graph_launch", C.c_int, [C.c_void_p, C.c_void_p]),
    ("ocp_set_segmented", C.c_int, [C.c_void_p, C.c_int32]),
    ("ocp_set_multiwave", C.c_int, [C.c_void_p, C.c_int32]),
    ("ocp_set_linsolve", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double]),
    ("ocp_set_segmented_after", C.c_int, [C.c_void_p, C.c_int32]),
    ("ocp_set_tail_workgroup", C.c_int, [C.c_void_p, C.c_int32]),
    ("ocp_set_iterate", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ocp_autotune", C.c_int, [C.c_void_p, C.POINTER(ocp_settings), C.c_int32, C.c_void_p, C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("ocp_profile_read", C.c_int, [C.c_void_p, C.POINTER(ocp_kernel_times)]),
    ("ocp_set_scaling", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ocp_set_scaling_box", C.c_int, [C.c_void_p, C.c_double]),
    ("ocp_solve_noalloc", C.c_int, [C.POINTER(ocp_dims), _ip, C.c_void_p, C.POINTER(ocp_settings),
                                    C.POINTER(ocp_solution), C.c_void_p]),
]

_LIB = None


class OCPError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().ocp_status_string(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where}: {msg} (status {code})")


def lib() -> C.CDLL:
    """Load libocp_admm.so from the package directory (raises if it is not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_24039_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def check(code: int, where: str):
    if code != OCP_OK:
        raise OCPError(code, where)


def default_settings(**overrides) -> ocp_settings:
    s = ocp_settings()
    lib().ocp_default_settings(C.byref(s))
    for k, v in overrides.items():
        if not hasattr(s, k):
            raise AttributeError(f"unknown setting {k}")
        setattr(s, k, v)
    return s
