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

FBS_NOALLOC_SCRATCH_BYTES = 32 << 20

FBS_PLAN_TUNE = 0x1
FBS_PLAN_PER_TILE = 0x2

# Entry points declared in include/fbs.h (checked by the ABI tests).
EXPORTS = (
    "fbs_validate", "fbs_workspace_bytes", "fbs_cost", "fbs_aggregate", "fbs_wta_subpixel",
    "fbs_run", "fbs_run_variant", "fbs_cost_lr", "fbs_lrc", "fbs_lr_workspace_bytes",
    "fbs_run_lr", "fbs_run_lr_noalloc", "fbs_wmf", "fbs_range_tile", "fbs_guided_ranges",
    "fbs_run_ranged", "fbs_plan_create", "fbs_plan_launch", "fbs_plan_pair_config",
    "fbs_plan_num_launches", "fbs_plan_destroy", "fbs_surrogate_num_params",
    "fbs_surrogate_create", "fbs_surrogate_destroy", "fbs_surrogate_set_params",
    "fbs_surrogate_get_params", "fbs_surrogate_features", "fbs_surrogate_cheap_run",
    "fbs_surrogate_forward",
    "fbs_surrogate_gradients", "fbs_surrogate_adam", "fbs_surrogate_run",
    "fbs_surrogate_run_tiled", "fbs_status_str",
    "fbs_last_error", "fbs_version",
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
        h.fbs_cost_lr.argtypes = [P, vp, vp, vp, vp, vp, vp]
        h.fbs_lrc.argtypes = [P, vp, vp, ctypes.c_int32, vp, vp, vp]
        h.fbs_lr_workspace_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        h.fbs_run_lr.argtypes = [P, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp]
        h.fbs_wmf.argtypes = [P, vp, vp, vp, vp]
        h.fbs_wmf.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int32)
        h.fbs_range_tile.argtypes = [P, ip, ip]
        h.fbs_guided_ranges.argtypes = [P, vp, vp, ctypes.c_int32, ctypes.c_int32, vp, vp]
        h.fbs_run_ranged.argtypes = [P, vp, vp, vp, vp, vp, vp]
        for f in (h.fbs_range_tile, h.fbs_guided_ranges, h.fbs_run_ranged):
            f.restype = ctypes.c_int
        h.fbs_run_lr_noalloc.argtypes = [P, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp]
        h.fbs_run_lr_noalloc.restype = ctypes.c_int
        for f in (h.fbs_validate, h.fbs_workspace_bytes, h.fbs_cost, h.fbs_aggregate,
                  h.fbs_wta_subpixel, h.fbs_run, h.fbs_run_variant, h.fbs_cost_lr, h.fbs_lrc,
                  h.fbs_lr_workspace_bytes, h.fbs_run_lr):
            f.restype = ctypes.c_int
        pp = ctypes.POINTER(ctypes.c_void_p)
        h.fbs_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, P,
                                      ctypes.c_char_p, ctypes.c_uint32]
        h.fbs_plan_create.restype = ctypes.c_int
        h.fbs_plan_launch.argtypes = [vp, pp, pp, pp, pp, vp]
        h.fbs_plan_launch.restype = ctypes.c_int
        h.fbs_plan_pair_config.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)]
        h.fbs_plan_pair_config.restype = ctypes.c_int
        h.fbs_plan_num_launches.argtypes = [vp]
        h.fbs_plan_num_launches.restype = ctypes.c_int32
        h.fbs_plan_destroy.argtypes = [vp]
        h.fbs_plan_destroy.restype = None
        fp = ctypes.POINTER(ctypes.c_float)
        h.fbs_surrogate_num_params.argtypes = []
        h.fbs_surrogate_num_params.restype = ctypes.c_int32
        h.fbs_surrogate_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_int32]
        h.fbs_surrogate_destroy.argtypes = [vp]
        h.fbs_surrogate_destroy.restype = None
        h.fbs_surrogate_set_params.argtypes = [vp, fp]
        h.fbs_surrogate_get_params.argtypes = [vp, fp]
        h.fbs_surrogate_features.argtypes = [vp, P, vp, vp, vp, vp]
        h.fbs_surrogate_cheap_run.argtypes = [vp, P, vp, vp, vp, vp, vp]
        h.fbs_surrogate_forward.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
        h.fbs_surrogate_gradients.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                                              vp, vp, vp, vp]
        h.fbs_surrogate_adam.argtypes = [vp, vp, ctypes.c_float, vp]
        h.fbs_surrogate_run.argtypes = [vp, P, P, vp, vp, vp, ctypes.c_float, ctypes.c_float,
                                        ctypes.POINTER(ctypes.c_int32), vp]
        h.fbs_surrogate_run_tiled.argtypes = [vp, P, P, vp, vp, vp, ctypes.c_float,
                                              ctypes.c_float, vp]
        for f in (h.fbs_surrogate_create, h.fbs_surrogate_set_params,
                  h.fbs_surrogate_get_params, h.fbs_surrogate_features,
                  h.fbs_surrogate_cheap_run,
                  h.fbs_surrogate_forward, h.fbs_surrogate_gradients, h.fbs_surrogate_adam,
                  h.fbs_surrogate_run, h.fbs_surrogate_run_tiled):
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


def fbs_cost_lr(p, left, right, cost_left, cost_right, workspace=None, stream=None):
    _check(lib().fbs_cost_lr(ctypes.byref(p), _ptr(left), _ptr(right), _ptr(cost_left),
                             _ptr(cost_right), _ptr(workspace), _stream(stream)))


def fbs_lrc(p, disp_left, disp_right, max_diff, valid, disp_sub, stream=None):
    _check(lib().fbs_lrc(ctypes.byref(p), _ptr(disp_left), _ptr(disp_right), int(max_diff),
                         _ptr(valid), _ptr(disp_sub), _stream(stream)))


def fbs_lr_workspace_bytes(p: FbsParams) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().fbs_lr_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return int(n.value)


def fbs_run_lr(p, left, right, max_diff, disp_left, disp_right, valid, disp_sub, workspace,
               stream=None):
    _check(lib().fbs_run_lr(ctypes.byref(p), _ptr(left), _ptr(right), int(max_diff),
                            _ptr(disp_left), _ptr(disp_right), _ptr(valid), _ptr(disp_sub),
                            _ptr(workspace), _stream(stream)))


def fbs_wmf(p, reference, disp_in, disp_out, stream=None):
    _check(lib().fbs_wmf(ctypes.byref(p), _ptr(reference), _ptr(disp_in), _ptr(disp_out),
                         _stream(stream)))


def fbs_range_tile(p):
    tw, th = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().fbs_range_tile(ctypes.byref(p), ctypes.byref(tw), ctypes.byref(th)))
    return int(tw.value), int(th.value)


def fbs_guided_ranges(p, disp_seed, valid, halo, margin, ranges, stream=None):
    _check(lib().fbs_guided_ranges(ctypes.byref(p), _ptr(disp_seed), _ptr(valid), int(halo),
                                   int(margin), _ptr(ranges), _stream(stream)))


def fbs_run_ranged(p, left, right, ranges, disp, disp_sub, stream=None):
    _check(lib().fbs_run_ranged(ctypes.byref(p), _ptr(left), _ptr(right), _ptr(ranges),
                                _ptr(disp), _ptr(disp_sub), _stream(stream)))


def fbs_run_lr_noalloc(p, left, right, max_diff, disp_left, disp_right, valid, disp_sub,
                       stream=None):
    _check(lib().fbs_run_lr_noalloc(ctypes.byref(p), _ptr(left), _ptr(right), int(max_diff),
                                    _ptr(disp_left), _ptr(disp_right), _ptr(valid),
                                    _ptr(disp_sub), _stream(stream)))


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


class FbsPlan:
    """Batched plan (fbs_plan_create / fbs_plan_launch / fbs_plan_destroy)."""

    def __init__(self, params, tune_cache: Optional[str] = None, tune: bool = False,
                 per_tile: bool = False):
        arr = (FbsParams * len(params))(*params)
        h = ctypes.c_void_p(None)
        path = tune_cache.encode() if tune_cache else None
        flags = (FBS_PLAN_TUNE if tune else 0) | (FBS_PLAN_PER_TILE if per_tile else 0)
        _check(lib().fbs_plan_create(ctypes.byref(h), len(params), arr, path, flags))
        self.handle = h
        self.n = len(params)

    def launch(self, lefts, rights, disps, subs, stream=None):
        n = self.n
        if not (len(lefts) == len(rights) == len(disps) == len(subs) == n):
            raise FbsError(FBS_E_INVALID, f"need {n} buffers of each kind")

        def arr(ts):
            return (ctypes.c_void_p * n)(*[_ptr(t) for t in ts])

        _check(lib().fbs_plan_launch(self.handle, arr(lefts), arr(rights), arr(disps), arr(subs),
                                     _stream(stream)))

    def pair_config(self, i: int):
        m, w, b = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().fbs_plan_pair_config(self.handle, i, ctypes.byref(m), ctypes.byref(w),
                                          ctypes.byref(b)))
        return int(m.value), int(w.value), int(b.value)

    def num_launches(self) -> int:
        return int(lib().fbs_plan_num_launches(self.handle))

    def close(self):
        if self.handle:
            lib().fbs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FbsSurrogate:
    """Learned surrogate object (fbs_surrogate_*).  Parameters are numpy
    float32 arrays in the packed order; buffers are device tensors."""

    def __init__(self, max_width: int, max_height: int, max_disp: int):
        h = ctypes.c_void_p(None)
        _check(lib().fbs_surrogate_create(ctypes.byref(h), max_width, max_height, max_disp))
        self.handle = h
        self.n_params = int(lib().fbs_surrogate_num_params())

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != self.n_params:
            raise FbsError(FBS_E_INVALID, f"need {self.n_params} parameters, got {a.size}")
        _check(lib().fbs_surrogate_set_params(
            self.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self):
        import numpy as np
        a = np.empty(self.n_params, dtype=np.float32)
        _check(lib().fbs_surrogate_get_params(
            self.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return a

    def features(self, cheap: FbsParams, left, agg, feat, stream=None):
        _check(lib().fbs_surrogate_features(self.handle, ctypes.byref(cheap), _ptr(left),
                                            _ptr(agg), _ptr(feat), _stream(stream)))

    def cheap_run(self, cheap: FbsParams, left, right, cheap_sub, feat, stream=None):
        _check(lib().fbs_surrogate_cheap_run(self.handle, ctypes.byref(cheap), _ptr(left),
                                             _ptr(right), _ptr(cheap_sub), _ptr(feat),
                                             _stream(stream)))

    def forward(self, width: int, height: int, feat, cheap_sub, pred, stream=None):
        _check(lib().fbs_surrogate_forward(self.handle, width, height, _ptr(feat),
                                           _ptr(cheap_sub), _ptr(pred), _stream(stream)))

    def gradients(self, width: int, height: int, feat, cheap_sub, label, pred, grads,
                  loss=None, stream=None):
        _check(lib().fbs_surrogate_gradients(self.handle, width, height, _ptr(feat),
                                             _ptr(cheap_sub), _ptr(label), _ptr(pred),
                                             _ptr(grads), _ptr(loss), _stream(stream)))

    def adam(self, grads, lr: float, stream=None):
        _check(lib().fbs_surrogate_adam(self.handle, _ptr(grads), float(lr), _stream(stream)))

    def run(self, cheap: FbsParams, full: FbsParams, left, right, disp_sub, gate_px: float,
            gate_frac: float, stream=None) -> bool:
        fb = ctypes.c_int32(0)
        _check(lib().fbs_surrogate_run(self.handle, ctypes.byref(cheap), ctypes.byref(full),
                                       _ptr(left), _ptr(right), _ptr(disp_sub), float(gate_px),
                                       float(gate_frac), ctypes.byref(fb), _stream(stream)))
        return bool(fb.value)

    def run_tiled(self, cheap: FbsParams, full: FbsParams, left, right, disp_sub,
                  gate_px: float, tile_frac: float, stream=None):
        _check(lib().fbs_surrogate_run_tiled(self.handle, ctypes.byref(cheap), ctypes.byref(full),
                                             _ptr(left), _ptr(right), _ptr(disp_sub),
                                             float(gate_px), float(tile_frac), _stream(stream)))

    def close(self):
        if self.handle:
            lib().fbs_surrogate_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
