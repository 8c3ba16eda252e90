"""ctypes view of librd.so: the C ABI declared in include/rd.h, same names.

Argument marshalling only -- every step of the reduction runs in the HIP
kernels of librd.so.  Importing this module loads the library and raises if
it has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime librd.so links against)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librd.so")
TUNED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.txt")

# enums of include/rd.h
RD_I32, RD_U32, RD_F32, RD_F64, RD_F16, RD_BF16, RD_I64, RD_U64 = range(8)
RD_SUM, RD_PROD, RD_MIN, RD_MAX, RD_AND, RD_OR, RD_XOR = range(7)
RD_OK, RD_ERR_INVALID_ARG, RD_ERR_UNSUPPORTED, RD_ERR_HIP, RD_ERR_NOMEM, RD_ERR_CAPTURE, RD_ERR_WORKSPACE = (
    0, -1, -2, -3, -4, -5, -6)
(RD_KIND_PLAIN, RD_KIND_COMPENSATED, RD_KIND_SEGMENTED, RD_KIND_ROWWISE, RD_KIND_ROWWISE_BWD, RD_KIND_SCAN,
 RD_KIND_SEGMENTED_SCAN) = range(7)
RD_WAIT_GRID, RD_WAIT_SCAN = 1, 2

STATUS_NAMES = {0: "RD_OK", -1: "RD_ERR_INVALID_ARG", -2: "RD_ERR_UNSUPPORTED", -3: "RD_ERR_HIP",
                -4: "RD_ERR_NOMEM", -5: "RD_ERR_CAPTURE", -6: "RD_ERR_WORKSPACE"}

# Every function include/rd.h declares: name -> (restype, argtypes)
_i64, _vp, _ci, _sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t


class RdConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("unroll", ctypes.c_int),
                ("blocks_per_cu", ctypes.c_int), ("nontemporal", ctypes.c_int),
                ("layout", ctypes.c_int)]


SIGNATURES = {
    "rd_init": (_ci, []),
    "rd_workspace_create": (_ci, [ctypes.POINTER(_vp), _ci]),
    "rd_workspace_destroy": (_ci, [_vp]),
    "rd_workspace_reset": (_ci, [_vp, _vp]),
    "rd_workspace_status": (_ci, [_vp, ctypes.POINTER(ctypes.c_uint)]),
    "rd_debug_force_wait_timeout": (_ci, [_ci]),
    "rd_dtype_size": (_sz, [_ci]),
    "rd_out_dtype": (_ci, [_ci, _ci, ctypes.POINTER(_ci)]),
    "rd_reduce": (_ci, [_vp, _i64, _ci, _ci, _vp, _vp, _vp]),
    "rd_reduce_noalloc": (_ci, [_vp, _i64, _ci, _ci, _vp, _vp]),
    "rd_reduce_compensated": (_ci, [_vp, _i64, _ci, _vp, _vp, _vp]),
    "rd_segmented_reduce": (_ci, [_vp, _vp, _i64, _ci, _ci, _vp, _vp, _vp]),
    "rd_reduce_paper_design": (_ci, [_vp, _i64, _ci, _ci, _ci, _vp, _vp, _vp]),
    "rd_argreduce": (_ci, [_vp, _i64, _ci, _ci, _vp, _vp, _vp, _vp]),
    "rd_scan": (_ci, [_vp, _i64, _ci, _ci, _ci, _vp, _vp, _vp]),
    "rd_segmented_scan": (_ci, [_vp, _i64, _vp, _i64, _ci, _ci, _ci, _vp, _vp, _vp]),
    "rd_saved_bytes": (_sz, [_ci, _i64, _i64]),
    "rd_rowreduce_fwd": (_ci, [_vp, _i64, _i64, _ci, _ci, _vp, _vp, _vp]),
    "rd_rowreduce_bwd": (_ci, [_vp, _vp, _vp, _i64, _i64, _ci, _ci, _vp, _vp]),
    "rd_config_get": (_ci, [_ci, _ci, _ci, _i64, ctypes.POINTER(RdConfig)]),
    "rd_config_force": (_ci, [_ci, ctypes.POINTER(RdConfig)]),
    "rd_tune_load": (_ci, [ctypes.c_char_p]),
    "rd_last_error": (ctypes.c_char_p, []),
}

_lib = None


class RdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded librd.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(or python -m paper_1710_07358_amd.build)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
        # The measured launch table for gfx950, when present, replaces the
        # built-in defaults (RD_TUNE_TABLE=<path> picks another, =none keeps them).
        table = os.environ.get("RD_TUNE_TABLE", TUNED_TABLE)
        if table != "none" and os.path.exists(table):
            check(handle.rd_tune_load(table.encode()))
    return _lib


def check(status: int) -> None:
    if status != RD_OK:
        raise RdError(status, lib().rd_last_error().decode(errors="replace"))
