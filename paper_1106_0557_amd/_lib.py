"""ctypes binding of ``libpspfft.so`` (the C ABI in ``include/pspfft.h``).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  torch is imported first so that the library binds to the HIP runtime
torch already loaded (both use the soname libamdhip64.so.7): device pointers and
streams are then shared.  A missing library raises at load time; there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded before libpspfft.so)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpspfft.so")

PSPFFT_OK = 0
STATUS_NAMES = {
    0: "PSPFFT_OK",
    1: "PSPFFT_ERR_INVALID_ARGUMENT",
    2: "PSPFFT_ERR_UNSUPPORTED_SIZE",
    3: "PSPFFT_ERR_OUT_OF_MEMORY",
    4: "PSPFFT_ERR_DEVICE",
    5: "PSPFFT_ERR_NOT_IMPLEMENTED",
}
PSPFFT_FP32 = 0
PSPFFT_FP64 = 1
PASS_X_FWD, PASS_Y_FWD, PASS_Z_CONV, PASS_Y_INV, PASS_X_INV = range(5)
PASS_NAMES = ("x_fwd", "y_fwd", "z_conv", "y_inv", "x_inv")

# Every symbol the header declares, for the load check.
EXPORTS = (
    "pspfft_plan_create", "pspfft_plan_create_ex", "pspfft_plan_fused", "pspfft_plan_spectrum_kz_fastest",
    "pspfft_workspace_ztile",
    "pspfft_destroy", "pspfft_solve",
    "pspfft_workspace_create", "pspfft_workspace_wrap", "pspfft_workspace_destroy",
    "pspfft_solve_ws", "pspfft_solve_batched", "pspfft_pass_batched",
    "pspfft_plan_bytes", "pspfft_plan_resident_bytes", "pspfft_workspace_bytes", "pspfft_pass_bytes",
    "pspfft_plan_info", "pspfft_plan_green", "pspfft_status_string",
    "pspfft_set_verbosity", "pspfft_get_verbosity", "pspfft_set_log_callback",
    "pspfft_solve_noalloc",
)
NOALLOC_MAX_BYTES = 128 << 20  # PSPFFT_NOALLOC_MAX_BYTES

# pspfft_verbosity (Sec. 3.2, VerbosityOption)
CONSOLE_ERROR, CONSOLE_WARNING, CONSOLE_INFO_1, CONSOLE_INFO_2 = range(4)
PLAN_VERBOSITY_SHIFT = 4
LOG_FN = ctypes.CFUNCTYPE(None, ctypes.c_int, ctypes.c_char_p, ctypes.c_void_p)


class PspfftError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)} ({_status_string(status)})")


_lib = None


def _status_string(status: int) -> str:
    try:
        return load().pspfft_status_string(status).decode()
    except Exception:  # pragma: no cover - only when the library itself is broken
        return "?"


def load():
    """Load ``libpspfft.so``; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1106_0557_amd.build` "
            "(the solver has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    vpp = ctypes.POINTER(ctypes.c_void_p)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "pspfft_plan_create": ([ip, ip, ip, dp, ip, vpp], ip),
        "pspfft_plan_create_ex": ([ip, ip, ip, dp, ip, ctypes.c_uint, vpp], ip),
        "pspfft_plan_fused": ([vp], ip),
        "pspfft_plan_spectrum_kz_fastest": ([vp], ip),
        "pspfft_workspace_ztile": ([vp], ip),
        "pspfft_destroy": ([vp], ip),
        "pspfft_solve": ([vp, vp, vp, vp], ip),
        "pspfft_solve_noalloc": ([vp, vp, vp, vp], ip),
        "pspfft_workspace_create": ([vp, vpp], ip),
        "pspfft_workspace_wrap": ([vp, vp, sz, vpp], ip),
        "pspfft_workspace_destroy": ([vp], ip),
        "pspfft_solve_ws": ([vp, vp, vp, vp, vp], ip),
        "pspfft_solve_batched": ([ip, vpp, vpp, vpp, vpp, vp], ip),
        "pspfft_pass_batched": ([ip, ip, vpp, vpp, vpp, vpp, vp], ip),
        "pspfft_plan_bytes": ([vp], sz),
        "pspfft_workspace_bytes": ([ip, ip, ip, ip], sz),
        "pspfft_plan_resident_bytes": ([ip, ip, ip, ip], sz),
        "pspfft_pass_bytes": ([vp, ip], sz),
        "pspfft_plan_info": ([vp, ctypes.POINTER(ctypes.c_int), dp, ctypes.POINTER(ctypes.c_int)], ip),
        "pspfft_plan_green": ([vp, vp, vp], ip),
        "pspfft_status_string": ([ip], ctypes.c_char_p),
        "pspfft_set_verbosity": ([ip], ip),
        "pspfft_get_verbosity": ([], ip),
        "pspfft_set_log_callback": ([LOG_FN, vp], ip),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status: int, what: str) -> None:
    if status != PSPFFT_OK:
        raise PspfftError(status, what)


def ptr_array(values):
    values = list(values)
    return (ctypes.c_void_p * max(1, len(values)))(*values)
