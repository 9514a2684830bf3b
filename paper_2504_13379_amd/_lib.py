"""ctypes declarations for libnfr.so (the C ABI declared in include/nfr.h).

Loading fails loudly when the library has not been built; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("NFR_LIBRARY") or os.path.join(HERE, "libnfr.so")

NFR_OK = 0
NFR_ERR_INVALID_ARG = -1
NFR_ERR_NONFINITE = -2
NFR_ERR_NO_DEVICE = -3
NFR_ERR_UNSUPPORTED_ARCH = -4
NFR_ERR_HIP = -5
NFR_ERR_WORKSPACE = -6
NFR_ERR_INTERNAL = -7

GAUSS_MH = 0
EXP_MH = 1

NFR_APPLY_NOALLOC_MAX_BYTES = 64 << 20   # fixed scratch of nfr_apply_noalloc (include/nfr.h)

PROJ_PLANES = 0
PROJ_ORIGIN = 1
PROJ_ORTHOGONAL = 2

FORM_AUTO = -1
FORM_ONTHEFLY_FP32 = 0
FORM_W_FP32 = 1
FORM_W_BF16X3 = 2
FORM_W_FP16X3 = 3
FORM_ONTHEFLY_BF16X3 = 4
FORM_ONTHEFLY_FP16X3 = 5
FORM_ONTHEFLY_FP32_MFMA = 6


class NfrKernel(ctypes.Structure):
    _fields_ = [("kind", c_int), ("A_e", c_double), ("s_e", c_double), ("A_i", c_double), ("s_i", c_double)]


class NfrFiring(ctypes.Structure):
    _fields_ = [("beta", c_double), ("theta", c_double), ("theta_dev", c_void_p)]


class NfrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (%d): %s" % (status_name(status), status, message))
        self.status = status


_lib = None


def _declare(lib):
    P = c_void_p
    sig = {
        "nfr_version": (c_int, [POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
        "nfr_status_string": (c_char_p, [c_int]),
        "nfr_last_error": (c_char_p, []),
        "nfr_context_create": (c_int, [c_int, P, POINTER(P)]),
        "nfr_context_destroy": (c_int, [P]),
        "nfr_context_arch": (c_char_p, [P]),
        "nfr_context_set_timing": (c_int, [P, c_int]),
        "nfr_context_timing": (c_int, [P, POINTER(c_int64), POINTER(c_double)]),
        "nfr_context_last_graph": (c_int, [P, POINTER(c_int64), POINTER(c_int64)]),
        "nfr_probe": (c_int, [P, c_int, c_int64, P, c_size_t, POINTER(c_double)]),
        "nfr_problem_bytes": (c_size_t, [c_int64]),
        "nfr_problem_create": (c_int, [P, c_int64, P, P, P, c_size_t, POINTER(P)]),
        "nfr_problem_create_periodic": (c_int, [P, c_int64, P, P, c_double, P, c_size_t, POINTER(P)]),
        "nfr_problem_period": (c_double, [P]),
        "nfr_tune_workspace_size": (c_size_t, [c_int64, c_int]),
        "nfr_tune": (c_int, [P, c_char_p, c_int64, c_int, P, c_size_t]),
        "nfr_tune_load": (c_int, [c_char_p]),
        "nfr_tune_target": (c_int64, [c_int64, c_int]),
        "nfr_tune_clear": (c_int, []),
        "nfr_quad_workspace_size": (c_size_t, [c_int64, c_int64, c_int]),
        "nfr_quad_weights": (c_int, [P, c_int64, P, P, c_int64, P, c_int, c_int, P, P, P, P, c_size_t]),
        "nfr_problem_destroy": (c_int, [P]),
        "nfr_problem_n": (c_int64, [P]),
        "nfr_problem_npad": (c_int64, [P]),
        "nfr_far_blocks_workspace_size": (c_size_t, [P]),
        "nfr_far_blocks": (c_int, [P, POINTER(NfrKernel), P, c_size_t, POINTER(c_int64), POINTER(c_int64)]),
        "nfr_w_bytes": (c_size_t, [c_int64, c_int]),
        "nfr_w_build": (c_int, [P, POINTER(NfrKernel), c_int, P, c_size_t]),
        "nfr_apply_workspace_size": (c_size_t, [P, c_int, c_int]),
        "nfr_apply": (c_int, [P, POINTER(NfrKernel), POINTER(NfrFiring), c_int, P, P, c_int, P, P, c_size_t]),
        "nfr_apply_noalloc": (c_int, [P, POINTER(NfrKernel), POINTER(NfrFiring), c_int, P, P, c_int, P]),
        "nfr_integrate_workspace_size": (c_size_t, [P, c_int, c_int]),
        "nfr_integrate": (c_int, [P, POINTER(NfrKernel), POINTER(NfrFiring), c_int, P, c_double, c_int64, c_int, P,
                                  P, c_int64, c_int, P, c_size_t]),
    }
    optional = {
        "nfr_adjoint_workspace_size": (c_size_t, [P, c_int64, c_int64]),
        "nfr_adjoint": (c_int, [P, POINTER(NfrKernel), POINTER(NfrFiring), P, c_int64, c_int64, c_double, P, P,
                                POINTER(c_double), P, c_size_t]),
        "nfr_integrate_forced": (c_int, [P, POINTER(NfrKernel), POINTER(NfrFiring), c_int, P, c_double, c_int64, P,
                                         c_int, P, P, c_size_t]),
        "nfr_integrate_ab5_workspace_size": (c_size_t, [P, c_int, c_int]),
        "nfr_integrate_ab5": (c_int, [P, POINTER(NfrKernel), POINTER(NfrFiring), c_int, P, c_double, c_int64, c_int,
                                      P, P, c_size_t]),
        "nfr_integrate_syndep_workspace_size": (c_size_t, [P, c_int]),
        "nfr_integrate_syndep": (c_int, [P, POINTER(NfrKernel), POINTER(NfrFiring), c_int, P, P, c_double, c_double,
                                         c_double, c_int64, P, c_size_t]),
        "nfr_batch_workspace_size": (c_size_t, [P]),
        "nfr_batch_create": (c_int, [P, c_int, POINTER(P), POINTER(NfrKernel), POINTER(NfrFiring), POINTER(c_int),
                                     POINTER(P)]),
        "nfr_batch_destroy": (c_int, [P]),
        "nfr_batch_set_config": (c_int, [P, c_int64, c_int]),
        "nfr_batch_get_config": (c_int, [P, POINTER(c_int64), POINTER(c_int)]),
        "nfr_batch_tune": (c_int, [P, POINTER(P), P, c_size_t, POINTER(c_double)]),
        "nfr_batch_integrate": (c_int, [P, POINTER(P), c_double, c_int64, c_int, P, c_size_t]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype, fn.argtypes = res, args
    for name, (res, args) in optional.items():
        fn = getattr(lib, name, None)
        if fn is not None:
            fn.restype, fn.argtypes = res, args
    return lib


def lib():
    """The loaded library; raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libnfr.so is not built (expected at %s); run __graft_entry__.build()" % LIB_PATH)
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def status_name(status: int) -> str:
    try:
        return lib().nfr_status_string(status).decode()
    except ImportError:
        return "NFR_STATUS_%d" % status


def check(status: int) -> None:
    if status != NFR_OK:
        raise NfrError(status, lib().nfr_last_error().decode())
