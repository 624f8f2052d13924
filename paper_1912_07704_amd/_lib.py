"""Loads ``libdd_mi355x.so`` and declares the C ABI of ``include/dd.h``."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libdd_mi355x.so")

# Every symbol include/dd.h declares, with its ctypes signature.
P = ctypes.c_void_p
I32, I64, F64, SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "dd_plan_create": (ctypes.c_int, [P, I32, F64, I64, P, I32, ctypes.c_int, P]),
    "dd_plan_destroy": (None, [P]),
    "dd_plan_info": (ctypes.c_int, [P, P, P, P]),
    "dd_plan_range": (ctypes.c_int, [P, I32, P, P, P, P, P]),
    "dd_plan_nranges": (ctypes.c_int, [P, P]),
    "dd_plan_dms": (ctypes.c_int, [P, P]),
    "dd_plan_shifts": (ctypes.c_int, [P, P]),
    "dd_plan_create_ex": (ctypes.c_int, [P, I32, F64, I64, P, I32, ctypes.c_int, P, P]),
    "dd_plan_strategy": (ctypes.c_int, [P, P, P, P, P, P]),
    "dd_workspace_bytes": (ctypes.c_int, [P, P]),
    "dd_plan_prepare": (ctypes.c_int, [P]),
    "dd_forward": (ctypes.c_int, [P, P, P, P, I64, P, SZ, P]),
    "dd_forward_bin": (ctypes.c_int, [P, P, P, P, SZ, P]),
    "dd_forward_sum": (ctypes.c_int, [P, P, I64, P, SZ, P]),
    "dd_forward_noalloc": (ctypes.c_int, [P, P, P, P, I64, P]),
    "dd_adjoint": (ctypes.c_int, [P, P, P, P, P, P, P, SZ, P]),
    "dd_boxcar_loss": (ctypes.c_int, [P, P, I32, P, I32, P, P, SZ, P]),
    "dd_boxcar_backward": (ctypes.c_int, [P, P, I32, P, I32, P, P, P, SZ, P]),
    "dd_batch_create": (ctypes.c_int, [P, I32, P]),
    "dd_batch_destroy": (None, [P]),
    "dd_batch_info": (ctypes.c_int, [P, P, P, P, P]),
    "dd_batch_beam": (ctypes.c_int, [P, I32, P, P]),
    "dd_batch_groups": (ctypes.c_int, [P, P]),
    "dd_batch_group": (ctypes.c_int, [P, I32, P, P, P, P]),
    "dd_batch_prepare": (ctypes.c_int, [P]),
    "dd_batch_forward": (ctypes.c_int, [P, P, P, I64, P, SZ, P]),
    "dd_batch_forward_weighted": (ctypes.c_int, [P, P, P, P, I64, P, SZ, P]),
    "dd_batch_boxcar_workspace": (ctypes.c_int, [P, P]),
    "dd_batch_boxcar_loss": (ctypes.c_int, [P, P, P, I32, P, P, SZ, P]),
    "dd_batch_boxcar_backward": (ctypes.c_int, [P, P, P, I32, P, P, P, SZ, P]),
    "dd_stream_create": (ctypes.c_int, [P, I32, P]),
    "dd_stream_destroy": (None, [P]),
    "dd_stream_info": (ctypes.c_int, [P, P, P]),
    "dd_stream_reset": (ctypes.c_int, [P]),
    "dd_stream_push": (ctypes.c_int, [P, P, I64, P, P, P, I64, P, SZ, P, P]),
    "dd_corner_turn": (ctypes.c_int, [ctypes.c_int, P, I64, I32, P, I64, P]),
    "dd_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "dd_last_error": (ctypes.c_char_p, []),
}

_lib = None


class DDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise ImportError(f"{library_path} is missing: build it with "
                              "`python -m paper_1912_07704_amd.build` (there is no fallback)")
        L = ctypes.CDLL(library_path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, what: str) -> None:
    if status != 0:
        L = lib()
        detail = (L.dd_last_error() or b"").decode()
        text = (L.dd_status_str(status) or b"").decode()
        raise DDError(status, f"{what}: {text}: {detail}")
