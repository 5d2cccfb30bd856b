"""ctypes declarations of liblfa's C ABI (include/lfa.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblfa.so")

LFA_F32 = 0
LFA_F64 = 1

LFA_WANT_U = 1
LFA_WANT_V = 2
LFA_ASM_MFMA = 4
LFA_ASM_BF16X2 = 8
LFA_ASM_BF16X3 = 16
LFA_PHASE_NORMALIZE = 32

LFA_SPECTRAL_IDENTITY = 0
LFA_SPECTRAL_CLIP = 1
LFA_SPECTRAL_PINV = 2
LFA_SPECTRAL_TRUNCATE = 3
LFA_CRYSTAL_FORWARD = 0
LFA_CRYSTAL_ADJOINT = 1

LFA_TUNE_LAYERS = 1
LFA_TUNE_PERSISTENT = 2

LFA_OK = 0
LFA_ERR_INVALID_ARG = -1
LFA_ERR_UNSUPPORTED = -2
LFA_ERR_WORKSPACE = -3
LFA_ERR_HIP = -4
LFA_ERR_NO_DEVICE = -5
LFA_ERR_NOT_PREPARED = -6

LFA_WARN_NOT_CONVERGED = 1
LFA_WARN_NONFINITE = 2
LFA_WARN_TEAM_TIMEOUT = 4

LFA_INFO_NONCONVERGED = 0
LFA_INFO_MAX_SWEEPS = 1
LFA_INFO_SUM_SWEEPS = 2
LFA_INFO_NONFINITE = 3
LFA_INFO_HIST = 4
LFA_INFO_HIST_BINS = 41
LFA_INFO_WORDS = 45


class LfaLayer(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in ("c_out", "c_in", "kh", "kw", "n", "m")]


P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
I32 = ctypes.c_int32
I32P = ctypes.POINTER(ctypes.c_int32)
SZ = ctypes.c_size_t

# name -> (restype, argtypes)
SIGNATURES = {
    "lfa_plan_create": (I32, [ctypes.POINTER(P), ctypes.POINTER(LfaLayer), I32, I32, ctypes.c_uint32]),
    "lfa_plan_destroy": (I32, [P]),
    "lfa_plan_prepare": (I32, [P, I32]),
    "lfa_plan_set_max_sweeps": (I32, [P, I32]),
    "lfa_plan_record_phases": (I32, [P, P]),
    "lfa_info_status": (I32, [I32P, I32]),
    "lfa_plan_workspace_bytes": (I32, [P, ctypes.POINTER(SZ)]),
    "lfa_plan_num_layers": (I32, [P, I32P]),
    "lfa_plan_layer": (I32, [P, I32, ctypes.POINTER(LfaLayer)]),
    "lfa_symbols": (I32, [P, PP, PP, P]),
    "lfa_svd": (I32, [P, PP, PP, PP, PP, P, P, SZ, P]),
    "lfa_svd_persistent": (I32, [P, PP, PP, PP, PP, P, P, SZ, P]),
    "lfa_svd_noalloc": (I32, [P, PP, PP, PP, PP, P, P]),
    "lfa_svd_persistent_busy": (I32, [P, PP, PP, PP, PP, P, P, SZ, P, I32, P]),
    "lfa_plan_persistent_grid": (I32, [P, I32P]),
    "lfa_svd_symbols": (I32, [P, PP, PP, PP, PP, P, P, SZ, P]),
    "lfa_topk": (I32, [P, PP, I32, P, P, P]),
    "lfa_adjoint": (I32, [P, PP, PP, P, P, I32, PP, P]),
    "lfa_sigma_grad": (I32, [P, PP, P, P, I32, PP, P, SZ, P]),
    "lfa_sigma_grad_persistent": (I32, [P, PP, P, P, I32, PP, P, SZ, P]),
    "lfa_graph_create": (I32, [P, PP, PP, I32, P, P, P, PP, P, P, SZ, P, ctypes.POINTER(P)]),
    "lfa_graph_create_uv": (I32, [P, PP, PP, PP, PP, I32, P, P, P, PP, P, P, SZ, P, ctypes.POINTER(P)]),
    "lfa_graph_create_onesided": (I32, [P, PP, PP, PP, I32, P, P, P, PP, P, P, SZ, P, ctypes.POINTER(P)]),
    "lfa_adjoint_onesided": (I32, [P, PP, PP, PP, P, P, I32, PP, P, SZ, P]),
    "lfa_graph_launch": (I32, [P, P]),
    "lfa_graph_destroy": (I32, [P]),
    "lfa_autotune": (I32, [P, PP, PP, PP, PP, ctypes.c_char_p, ctypes.c_uint32, P]),
    "lfa_plan_tuning": (I32, [P, I32, I32P, I32P, I32P, I32P]),
    "lfa_plan_cost_model": (I32, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]),
    "lfa_plan_launch_shape": (I32, [P, I32, I32P, I32P, I32P, I32P]),
    "lfa_apply_workspace_bytes": (I32, [P, I32, I32, ctypes.POINTER(SZ)]),
    "lfa_apply": (I32, [P, I32, P, P, P, I32, ctypes.c_double, P, P, I32, P, SZ, P]),
    "lfa_lift": (I32, [P, I32, P, P, P, I32, P, P, P]),
    "lfa_crystal_layer": (I32, [ctypes.POINTER(LfaLayer), I32, ctypes.POINTER(LfaLayer)]),
    "lfa_crystal_weights": (I32, [ctypes.POINTER(LfaLayer), I32, I32, P, P, I32, P]),
    "lfa_plan_queue_info": (I32, [P, I32, I32P, I32P]),
    "lfa_plan_preconditioned": (I32, [P, I32, I32P]),
    "lfa_status_string": (ctypes.c_char_p, [I32]),
    "lfa_last_hip_error": (I32, []),
    "lfa_version": (I32, []),
}

_lib = None


def load():
    """Load liblfa.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"liblfa.so not found at {LIB_PATH}: build it with "
            "`python -m paper_2506_05617_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LfaError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.lfa_status_string(status).decode()
        hip = lib.lfa_last_hip_error() if status == LFA_ERR_HIP else 0
        super().__init__(f"{where}: {msg} (status {status}" + (f", hipError {hip})" if hip else ")"))
        self.status = status


def check(status: int, where: str) -> int:
    if status < 0:
        raise LfaError(status, where)
    return status


def ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(p) if p else None for p in ptrs])
    return ctypes.cast(arr, PP), arr
