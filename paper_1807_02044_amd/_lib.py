"""ctypes binding of the C ABI in include/fbs.h (argument marshalling only).

Every function here forwards to the entry point of the same name in
``libfbs.so``.  Device buffers may be given as torch tensors (their
``data_ptr()`` is passed) or as raw integer device addresses; the stream
defaults to torch's current stream on the current device so the kernels are
ordered with torch's own work.  There is no fallback: if ``libfbs.so`` is
missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfbs.so")

FBS_OK = 0
FBS_E_INVALID = -1
FBS_E_UNSUPPORTED = -2
FBS_E_HIP = -3
FBS_E_WORKSPACE = -4

FBS_COST_TAD = 0
FBS_COST_NCC = 1

FBS_MAX_RADIUS = 16
FBS_MAX_NCC_RADIUS = 3
FBS_MAX_DISP = 1024

FBS_F_FORCE_VALU = 0x1

# Entry points declared in include/fbs.h (checked by the ABI tests).
EXPORTS = (
    "fbs_validate", "fbs_workspace_bytes", "fbs_cost", "fbs_aggregate", "fbs_wta_subpixel",
    "fbs_run", "fbs_run_variant", "fbs_status_str", "fbs_last_error", "fbs_version",
)


class FbsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class FbsParams(ctypes.Structure):
    """Mirror of ``fbs_params``."""

    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("channels", ctypes.c_int32), ("row_stride", ctypes.c_int32),
        ("d_min", ctypes.c_int32), ("d_max", ctypes.c_int32),
        ("radius", ctypes.c_int32),
        ("sigma_s", ctypes.c_float), ("sigma_r", ctypes.c_float),
        ("cost_cap", ctypes.c_float),
        ("cost_type", ctypes.c_int32), ("ncc_radius", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


def make_params(width: int, height: int, channels: int, d_min: int, d_max: int, radius: int,
                sigma_s: float, sigma_r: float, cost_cap: float = 40.0,
                cost_type: int = FBS_COST_TAD, ncc_radius: int = 1, flags: int = 0,
                row_stride: Optional[int] = None) -> FbsParams:
    return FbsParams(width, height, channels,
                     width * channels if row_stride is None else row_stride,
                     d_min, d_max, radius, float(sigma_s), float(sigma_r), float(cost_cap),
                     cost_type, ncc_radius, flags)


_lib = None


def lib() -> ctypes.CDLL:
    """Load libfbs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FbsError(FBS_E_HIP, f"{LIB_PATH} is missing: build it with "
                                      "paper_1807_02044_amd.build.build()")
        h = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(FbsParams)
        vp = ctypes.c_void_p
        h.fbs_validate.argtypes = [P]
        h.fbs_workspace_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        h.fbs_cost.argtypes = [P, vp, vp, vp, vp, vp]
        h.fbs_aggregate.argtypes = [P, vp, vp, vp, vp]
        h.fbs_wta_subpixel.argtypes = [P, vp, vp, vp, vp]
        h.fbs_run.argtypes = [P, vp, vp, vp, vp, vp, vp, vp]
        h.fbs_run_variant.argtypes = [P]
        for f in (h.fbs_validate, h.fbs_workspace_bytes, h.fbs_cost, h.fbs_aggregate,
                  h.fbs_wta_subpixel, h.fbs_run, h.fbs_run_variant):
            f.restype = ctypes.c_int
        h.fbs_status_str.argtypes = [ctypes.c_int]
        h.fbs_status_str.restype = ctypes.c_char_p
        h.fbs_last_error.argtypes = []
        h.fbs_last_error.restype = ctypes.c_char_p
        h.fbs_version.argtypes = []
        h.fbs_version.restype = ctypes.c_char_p
        _lib = h
    return _lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise FbsError(FBS_E_INVALID, "buffers must be device tensors")
    if not t.is_contiguous():
        raise FbsError(FBS_E_INVALID, "buffers must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(rc: int):
    if rc != FBS_OK:
        raise FbsError(rc, lib().fbs_last_error().decode())


def fbs_validate(p: FbsParams) -> int:
    return lib().fbs_validate(ctypes.byref(p))


def fbs_workspace_bytes(p: FbsParams) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().fbs_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return int(n.value)


def fbs_cost(p, left, right, cost, workspace=None, stream=None):
    _check(lib().fbs_cost(ctypes.byref(p), _ptr(left), _ptr(right), _ptr(cost),
                          _ptr(workspace), _stream(stream)))


def fbs_aggregate(p, left, cost, agg, stream=None):
    _check(lib().fbs_aggregate(ctypes.byref(p), _ptr(left), _ptr(cost), _ptr(agg),
                               _stream(stream)))


def fbs_wta_subpixel(p, agg, disp, disp_sub, stream=None):
    _check(lib().fbs_wta_subpixel(ctypes.byref(p), _ptr(agg), _ptr(disp), _ptr(disp_sub),
                                  _stream(stream)))


def fbs_run(p, left, right, disp, disp_sub, agg_out=None, workspace=None, stream=None):
    _check(lib().fbs_run(ctypes.byref(p), _ptr(left), _ptr(right), _ptr(disp), _ptr(disp_sub),
                         _ptr(agg_out), _ptr(workspace), _stream(stream)))


def fbs_run_variant(p: FbsParams) -> int:
    v = lib().fbs_run_variant(ctypes.byref(p))
    if v < 0:
        _check(v)
    return v


def fbs_status_str(status: int) -> str:
    return lib().fbs_status_str(status).decode()


def fbs_last_error() -> str:
    return lib().fbs_last_error().decode()


def fbs_version() -> str:
    return lib().fbs_version().decode()
