"""FP64 CPU oracle for fast bilateral stereo (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library and its Python binding
never import it; the two share no code.  The arithmetic lives in
``fbs_oracle.c`` (plain C, double precision, OpenMP over rows); this module
only compiles it with gcc, loads it, and marshals numpy arrays.

Each function follows the paper (Fan et al., "Real-Time Subpixel Fast
Bilateral Stereo"):

* :func:`cost`          Section II-A: TAD, or NCC (Eqs. 1-3) as the cost 1 - c
* :func:`weights`       Section II-B, Eqs. (7)-(8)
* :func:`aggregate`     Section II-B, Eq. (6)
* :func:`wta_subpixel`  Section II-C (WTA) and Section II-D, Eq. (10)
* :func:`fbs`           the four steps in order, left image as reference
* :func:`fbs_pixels`    the same four steps at chosen pixels only
* :func:`cost_right`    Section II-A: the right cost volume, C_R(u,v,d) = C_L(u+d,v,d)
* :func:`fbs_right`     the four steps with the right image as reference
* :func:`fbs_right_pixels`  the same at chosen right-image pixels
* :func:`lrc`           Section II-D, Eq. (9): left-right consistency of two maps
* :func:`fbs_lrc`       both maps, Eq. (9), and Eq. (10) on the surviving left pixels
* :func:`wmf`           weighted median filter of a disparity map (Section II-D)
* :func:`guided_ranges` per-tile search ranges from reliable seeds (Section V)
* :func:`fbs_ranged`    WTA and Eq. (10) restricted to each tile's range
* :func:`wmf_cumulative`  window weights below / up to a candidate median
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fbs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_fbs.so")

TAD = 0
NCC = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("channels", ctypes.c_int32), ("row_stride", ctypes.c_int32),
        ("d_min", ctypes.c_int32), ("d_max", ctypes.c_int32),
        ("radius", ctypes.c_int32), ("ncc_radius", ctypes.c_int32),
        ("cost_type", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("gamma_d", ctypes.c_double), ("gamma_r", ctypes.c_double), ("tau", ctypes.c_double),
    ]


@dataclass(frozen=True)
class Problem:
    """Parameters of one left-reference FBS evaluation."""

    d_min: int
    d_max: int
    radius: int
    gamma_d: float
    gamma_r: float
    tau: float = 40.0
    cost_type: int = TAD
    ncc_radius: int = 1

    @property
    def n_disp(self) -> int:
        return self.d_max - self.d_min + 1

    @staticmethod
    def from_workload(wl, cost_type: int = TAD, ncc_radius: int = 1) -> "Problem":
        return Problem(wl.d_min, wl.d_max, wl.radius, wl.sigma_s, wl.sigma_r, wl.cost_cap,
                       cost_type, ncc_radius)


_lib_handle = None


def lib() -> ctypes.CDLL:
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=False)
        h = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        f64 = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.POINTER(ctypes.c_int32)
        h.orc_cost.argtypes = [P, u8, u8, f64]
        h.orc_weights.argtypes = [P, u8, f64]
        h.orc_aggregate.argtypes = [P, f64, f64, f64]
        h.orc_wta_subpixel.argtypes = [P, f64, i32, f64]
        h.orc_fbs.argtypes = [P, u8, u8, i32, f64, f64]
        h.orc_fbs_pixels.argtypes = [P, u8, u8, ctypes.c_int32, i32, i32, f64, i32, f64]
        h.orc_threads.argtypes = []
        u8p = ctypes.POINTER(ctypes.c_uint8)
        h.orc_cost_right.argtypes = [P, u8, u8, f64]
        h.orc_fbs_right.argtypes = [P, u8, u8, i32, f64, f64]
        h.orc_fbs_right_pixels.argtypes = [P, u8, u8, ctypes.c_int32, i32, i32, f64, i32, f64]
        h.orc_lrc.argtypes = [P, i32, i32, ctypes.c_int32, u8p]
        h.orc_fbs_lrc.argtypes = [P, u8, u8, ctypes.c_int32, i32, i32, u8p, f64]
        h.orc_wmf.argtypes = [P, u8, i32, i32]
        h.orc_guided_ranges.argtypes = [P, i32, u8p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, i32]
        h.orc_fbs_ranged.argtypes = [P, u8, u8, ctypes.c_int32, ctypes.c_int32, i32, i32, f64]
        h.orc_wmf_cumulative.argtypes = [P, u8, i32, i32, f64, f64, f64]
        for f in (h.orc_cost, h.orc_weights, h.orc_aggregate, h.orc_wta_subpixel, h.orc_fbs,
                  h.orc_fbs_pixels, h.orc_threads, h.orc_cost_right, h.orc_fbs_right,
                  h.orc_fbs_right_pixels, h.orc_lrc, h.orc_fbs_lrc, h.orc_wmf,
                  h.orc_wmf_cumulative, h.orc_guided_ranges, h.orc_fbs_ranged):
            f.restype = ctypes.c_int
        _lib_handle = h
    return _lib_handle


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(lib().orc_threads())


def _shape(img: np.ndarray) -> Tuple[int, int, int]:
    if img.ndim == 2:
        return img.shape[0], img.shape[1], 1
    if img.ndim == 3 and img.shape[2] in (1, 3):
        return img.shape[0], img.shape[1], img.shape[2]
    raise ValueError(f"image must be HxW or HxWx3 uint8, got {img.shape}")


def _params(pb: Problem, img: np.ndarray) -> _Params:
    if img.dtype != np.uint8:
        raise TypeError("images are uint8")
    H, W, C = _shape(img)
    gd = math.inf if pb.gamma_d == math.inf else float(pb.gamma_d)
    gr = math.inf if pb.gamma_r == math.inf else float(pb.gamma_r)
    return _Params(W, H, C, W * C, pb.d_min, pb.d_max, pb.radius, pb.ncc_radius,
                   pb.cost_type, 0, gd, gr, float(pb.tau))


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8).ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _f64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid parameters (rc={rc})")


def cost(pb: Problem, left: np.ndarray, right: np.ndarray) -> np.ndarray:
    """Matching-cost volume [D][H][W] (float64)."""
    H, W, _ = _shape(left)
    if left.shape != right.shape:
        raise ValueError("left/right shapes differ")
    out = np.empty((pb.n_disp, H, W), dtype=np.float64)
    L = np.ascontiguousarray(left)
    R = np.ascontiguousarray(right)
    _check(lib().orc_cost(ctypes.byref(_params(pb, L)), _u8(L), _u8(R), _f64(out)), "cost")
    return out


def weights(pb: Problem, left: np.ndarray) -> np.ndarray:
    """Support weights [H][W][(2r+1)^2] (float64), tap order dy outer, dx inner."""
    H, W, _ = _shape(left)
    T = (2 * pb.radius + 1) ** 2
    out = np.empty((H, W, T), dtype=np.float64)
    L = np.ascontiguousarray(left)
    _check(lib().orc_weights(ctypes.byref(_params(pb, L)), _u8(L), _f64(out)), "weights")
    return out


def aggregate(pb: Problem, left: np.ndarray, cost_vol: np.ndarray,
              w: Optional[np.ndarray] = None) -> np.ndarray:
    """Eq. (6) on a given cost volume; weights come from ``left`` unless given."""
    H, W, _ = _shape(left)
    cv = np.ascontiguousarray(cost_vol, dtype=np.float64)
    if cv.shape != (pb.n_disp, H, W):
        raise ValueError(f"cost volume shape {cv.shape} != {(pb.n_disp, H, W)}")
    if w is None:
        w = weights(pb, left)
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.empty_like(cv)
    L = np.ascontiguousarray(left)
    _check(lib().orc_aggregate(ctypes.byref(_params(pb, L)), _f64(cv), _f64(w), _f64(out)),
           "aggregate")
    return out


def wta_subpixel(pb: Problem, agg: np.ndarray, width: Optional[int] = None,
                 height: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """First-minimum WTA and Eq. (10) on a [D][H][W] volume."""
    a = np.ascontiguousarray(agg, dtype=np.float64)
    D, H, W = a.shape
    if D != pb.n_disp:
        raise ValueError("volume depth != d_max - d_min + 1")
    disp = np.empty((H, W), dtype=np.int32)
    sub = np.empty((H, W), dtype=np.float64)
    fake = np.zeros((H, W), dtype=np.uint8)      # only the image shape is read
    _check(lib().orc_wta_subpixel(ctypes.byref(_params(pb, fake)), _f64(a), _i32(disp),
                                  _f64(sub)), "wta_subpixel")
    return disp, sub


def fbs(pb: Problem, left: np.ndarray, right: np.ndarray, want_agg: bool = False):
    """Whole pipeline. Returns (disp int32 [H][W], disp_sub f64 [H][W][, agg])."""
    H, W, _ = _shape(left)
    if left.shape != right.shape:
        raise ValueError("left/right shapes differ")
    L = np.ascontiguousarray(left)
    R = np.ascontiguousarray(right)
    disp = np.empty((H, W), dtype=np.int32)
    sub = np.empty((H, W), dtype=np.float64)
    agg = np.empty((pb.n_disp, H, W), dtype=np.float64) if want_agg else None
    rc = lib().orc_fbs(ctypes.byref(_params(pb, L)), _u8(L), _u8(R), _i32(disp), _f64(sub),
                       _f64(agg) if agg is not None else None)
    _check(rc, "fbs")
    return (disp, sub, agg) if want_agg else (disp, sub)


def fbs_pixels(pb: Problem, left: np.ndarray, right: np.ndarray, xs, ys):
    """Pipeline at chosen pixels. Returns (agg [n][D], disp [n], disp_sub [n])."""
    L = np.ascontiguousarray(left)
    R = np.ascontiguousarray(right)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    n = int(xs.size)
    agg = np.empty((n, pb.n_disp), dtype=np.float64)
    disp = np.empty(n, dtype=np.int32)
    sub = np.empty(n, dtype=np.float64)
    rc = lib().orc_fbs_pixels(ctypes.byref(_params(pb, L)), _u8(L), _u8(R), n, _i32(xs),
                              _i32(ys), _f64(agg), _i32(disp), _f64(sub))
    _check(rc, "fbs_pixels")
    return agg, disp, sub


# ------------------------------------------------------------ right reference


def cost_right(pb: Problem, left: np.ndarray, right: np.ndarray) -> np.ndarray:
    """Right cost volume [D][H][W] (float64): C_R(u,v,d) = C_L(u+d,v,d)."""
    H, W, _ = _shape(left)
    if left.shape != right.shape:
        raise ValueError("left/right shapes differ")
    out = np.empty((pb.n_disp, H, W), dtype=np.float64)
    L = np.ascontiguousarray(left)
    R = np.ascontiguousarray(right)
    _check(lib().orc_cost_right(ctypes.byref(_params(pb, L)), _u8(L), _u8(R), _f64(out)),
           "cost_right")
    return out


def fbs_right(pb: Problem, left: np.ndarray, right: np.ndarray, want_agg: bool = False):
    """Right-reference pipeline. Returns (disp, disp_sub[, agg]) of the right view."""
    H, W, _ = _shape(left)
    if left.shape != right.shape:
        raise ValueError("left/right shapes differ")
    L = np.ascontiguousarray(left)
    R = np.ascontiguousarray(right)
    disp = np.empty((H, W), dtype=np.int32)
    sub = np.empty((H, W), dtype=np.float64)
    agg = np.empty((pb.n_disp, H, W), dtype=np.float64) if want_agg else None
    rc = lib().orc_fbs_right(ctypes.byref(_params(pb, L)), _u8(L), _u8(R), _i32(disp), _f64(sub),
                             _f64(agg) if agg is not None else None)
    _check(rc, "fbs_right")
    return (disp, sub, agg) if want_agg else (disp, sub)


def fbs_right_pixels(pb: Problem, left: np.ndarray, right: np.ndarray, xs, ys):
    """Right-reference pipeline at chosen right-image pixels: (agg [n][D], disp, disp_sub)."""
    L = np.ascontiguousarray(left)
    R = np.ascontiguousarray(right)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    n = int(xs.size)
    agg = np.empty((n, pb.n_disp), dtype=np.float64)
    disp = np.empty(n, dtype=np.int32)
    sub = np.empty(n, dtype=np.float64)
    rc = lib().orc_fbs_right_pixels(ctypes.byref(_params(pb, L)), _u8(L), _u8(R), n, _i32(xs),
                                    _i32(ys), _f64(agg), _i32(disp), _f64(sub))
    _check(rc, "fbs_right_pixels")
    return agg, disp, sub


def lrc(pb: Problem, disp_left: np.ndarray, disp_right: np.ndarray,
        max_diff: int = 0) -> np.ndarray:
    """Eq. (9) on two integer maps: uint8 [H][W], 1 where the left match survives."""
    dl = np.ascontiguousarray(disp_left, dtype=np.int32)
    dr = np.ascontiguousarray(disp_right, dtype=np.int32)
    if dl.shape != dr.shape or dl.ndim != 2:
        raise ValueError("maps must be [H][W] of one shape")
    valid = np.empty(dl.shape, dtype=np.uint8)
    fake = np.zeros(dl.shape, dtype=np.uint8)      # only the image shape is read
    _check(lib().orc_lrc(ctypes.byref(_params(pb, fake)), _i32(dl), _i32(dr), int(max_diff),
                         valid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), "lrc")
    return valid


def fbs_lrc(pb: Problem, left: np.ndarray, right: np.ndarray, max_diff: int = 0):
    """The paper's full path: (disp_left, disp_right, valid, disp_sub) with
    disp_sub = Eq. (10) on the left map where Eq. (9) holds and -1 elsewhere."""
    H, W, _ = _shape(left)
    L = np.ascontiguousarray(left)
    R = np.ascontiguousarray(right)
    dl = np.empty((H, W), dtype=np.int32)
    dr = np.empty((H, W), dtype=np.int32)
    valid = np.empty((H, W), dtype=np.uint8)
    sub = np.empty((H, W), dtype=np.float64)
    rc = lib().orc_fbs_lrc(ctypes.byref(_params(pb, L)), _u8(L), _u8(R), int(max_diff), _i32(dl),
                           _i32(dr), valid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                           _f64(sub))
    _check(rc, "fbs_lrc")
    return dl, dr, valid, sub


# ------------------------------------------------------ weighted median filter


def wmf(pb: Problem, image: np.ndarray, disp_in: np.ndarray) -> np.ndarray:
    """Weighted median of int disparities over each (2 radius + 1)^2 window,
    weights of Eqs. (7)-(8) from `image`; values outside [d_min, d_max] are
    holes; -1 where a window holds no valid value."""
    img = np.ascontiguousarray(image)
    H, W, _ = _shape(img)
    din = np.ascontiguousarray(disp_in, dtype=np.int32)
    if din.shape != (H, W):
        raise ValueError("map and image shapes differ")
    out = np.empty((H, W), dtype=np.int32)
    _check(lib().orc_wmf(ctypes.byref(_params(pb, img)), _u8(img), _i32(din), _i32(out)), "wmf")
    return out


def wmf_cumulative(pb: Problem, image: np.ndarray, disp_in: np.ndarray, m: np.ndarray):
    """(below, upto, total) window weights for candidate medians m [H][W]."""
    img = np.ascontiguousarray(image)
    H, W, _ = _shape(img)
    din = np.ascontiguousarray(disp_in, dtype=np.int32)
    mm = np.ascontiguousarray(m, dtype=np.int32)
    below = np.empty((H, W), dtype=np.float64)
    upto = np.empty((H, W), dtype=np.float64)
    total = np.empty((H, W), dtype=np.float64)
    _check(lib().orc_wmf_cumulative(ctypes.byref(_params(pb, img)), _u8(img), _i32(din), _i32(mm),
                                    _f64(below), _f64(upto), _f64(total)), "wmf_cumulative")
    return below, upto, total


# ------------------------------------------------- guided search range (Sec. V)


def guided_ranges(pb: Problem, disp: np.ndarray, valid: np.ndarray, tile_w: int, tile_h: int,
                  halo: int, margin: int) -> np.ndarray:
    """Per-tile (lo, hi) ranges [tiles_y][tiles_x][2] from reliable seeds."""
    d = np.ascontiguousarray(disp, dtype=np.int32)
    v = np.ascontiguousarray(valid, dtype=np.uint8)
    H, W = d.shape
    ty, tx = (H + tile_h - 1) // tile_h, (W + tile_w - 1) // tile_w
    out = np.empty((ty, tx, 2), dtype=np.int32)
    fake = np.zeros((H, W), dtype=np.uint8)
    _check(lib().orc_guided_ranges(ctypes.byref(_params(pb, fake)), _i32(d),
                                   v.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), tile_w,
                                   tile_h, halo, margin, _i32(out)), "guided_ranges")
    return out


def fbs_ranged(pb: Problem, left: np.ndarray, right: np.ndarray, tile_w: int, tile_h: int,
               ranges: np.ndarray):
    """(disp, disp_sub) with WTA and Eq. (10) over each tile's range only."""
    L = np.ascontiguousarray(left)
    R = np.ascontiguousarray(right)
    H, W, _ = _shape(L)
    rg = np.ascontiguousarray(ranges, dtype=np.int32)
    if rg.shape != ((H + tile_h - 1) // tile_h, (W + tile_w - 1) // tile_w, 2):
        raise ValueError("ranges must be [tiles_y][tiles_x][2]")
    disp = np.empty((H, W), dtype=np.int32)
    sub = np.empty((H, W), dtype=np.float64)
    _check(lib().orc_fbs_ranged(ctypes.byref(_params(pb, L)), _u8(L), _u8(R), tile_w, tile_h,
                                _i32(rg), _i32(disp), _f64(sub)), "fbs_ranged")
    return disp, sub
