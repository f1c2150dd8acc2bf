"""ctypes declarations of the C ABI in include/paradiag.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libparadiag.so")

PD_OK = 0
PD_NOT_CONVERGED = 1
PD_ERR_INVALID = -1
PD_ERR_UNSUPPORTED = -2
PD_ERR_WORKSPACE = -3
PD_ERR_HIP = -4
PD_ERR_NONFINITE = -5
PD_ERR_BREAKDOWN = -6
PD_STATIC_SCRATCH_BYTES = 128 << 20

STATUS_NAMES = {0: "PD_OK", 1: "PD_NOT_CONVERGED", -1: "PD_ERR_INVALID", -2: "PD_ERR_UNSUPPORTED",
                -3: "PD_ERR_WORKSPACE", -4: "PD_ERR_HIP", -5: "PD_ERR_NONFINITE",
                -6: "PD_ERR_BREAKDOWN"}

SCHEMES = {"be": 0, "tr": 1, "lf": 2, "hyb": 3, "hyb2": 4}
PRECS = {"fp64": 0, "fp32": 1, "fp32_bf16gemm": 2, "fp32_bf16x1": 3, "fp32_fp16gemm": 4}
MODES = {"fgmres": 0, "stationary": 1, "direct": 2, "parareal": 3, "nonlinear": 4}
STAGES = ["fft_fwd", "xform_fwd", "line_solve", "xform_inv", "fft_inv", "matvec", "dot", "update",
          "other", "fine", "reaction"]


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("batch", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("reserved", ctypes.c_int32), ("T", ctypes.c_double),
                ("nu", ctypes.c_double), ("ax", ctypes.c_double), ("ay", ctypes.c_double),
                ("alpha", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("use_x0", ctypes.c_int32), ("rtol", ctypes.c_double)]


class Cubic(ctypes.Structure):
    _fields_ = [("k1", ctypes.c_double), ("k2", ctypes.c_double), ("k3", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("iters_per_rhs", ctypes.POINTER(ctypes.c_int32)),
                ("resid_per_rhs", ctypes.POINTER(ctypes.c_double)),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int32),
                ("history_len", ctypes.c_int32)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); every symbol include/paradiag.h declares
SIGNATURES = {
    "paradiag_setup": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(_P)]),
    "paradiag_oc_setup": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_double, ctypes.POINTER(_P)]),
    "paradiag_oc_build_rhs": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "paradiag_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(SolveOpts), ctypes.POINTER(ctypes.c_size_t)]),
    "paradiag_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "paradiag_build_rhs": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "paradiag_rhs_transpose": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "paradiag_matvec": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P]),
    "paradiag_apply_precond": (ctypes.c_int, [_P, _P, _P, _P]),
    "paradiag_apply_precond_static": (ctypes.c_int, [_P, _P, _P, _P]),
    "paradiag_solve": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P]),
    "paradiag_adjoint_solve": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P]),
    "paradiag_parareal": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.POINTER(SolveOpts),
                                         ctypes.POINTER(SolveInfo), _P]),
    "paradiag_nonlinear_solve": (ctypes.c_int, [_P, ctypes.POINTER(Cubic), _P, ctypes.c_int32, _P,
                                                ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P]),
    "paradiag_get_xbasis": (ctypes.c_int, [_P, ctypes.c_int32, _D, _D]),
    "paradiag_get_symbols": (ctypes.c_int, [_P, _D, _D]),
    "paradiag_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "paradiag_get_stage_times": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64), _D, _D,
                                                ctypes.c_int32]),
    "paradiag_destroy": (None, [_P]),
    "paradiag_last_error": (ctypes.c_char_p, []),
    "paradiag_version": (ctypes.c_char_p, []),
}

_lib = None


class ParaDiagError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libparadiag.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} not found: build the HIP library first (python -m paper_2005_09158_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str, allow_not_converged: bool = False) -> int:
    if status == PD_OK or (allow_not_converged and status == PD_NOT_CONVERGED):
        return status
    msg = load().paradiag_last_error().decode(errors="replace")
    raise ParaDiagError(status, where, msg)
