"""Comparison rules between the HIP path and the FP64 oracle.

* aggregated costs: |A_gpu - A_oracle| <= 1e-4 * |A_oracle| + 1e-6
  (the absolute floor only matters where the oracle's cost is 0);
* integer disparity: equal, or the GPU's pick lies in the oracle's tie zone,
  A_o(d_gpu) - A_o(d_o) <= 1e-5 * max(|A_o(d_gpu)|, |A_o(d_o)|) + floor.
  The absolute floor is the range limit of the kernels' weights.  The
  matrix-core kernel holds each weight w <= 1 as fp16 hi + lo of w * 2^14,
  and fp16's smallest subnormal is 2^-24, so weights below 2^-38 are zero
  there and each weight carries an absolute error below 2^-38; Eq. 6 then
  moves by at most T * c_max * 2^-38 (T taps, costs <= c_max, weight sum >= 1
  from the centre tap), and two costs closer than twice that cannot be told
  apart.  For the float32 vector kernel the same bound with 2^-126 is smaller
  still.  floor = weight_floor(T, c_max) = 2 * T * c_max * 2^-38;
* subpixel disparity: where the integers agree, |ds_gpu - ds_oracle| <= 1e-3.
  Eq. 10 amplifies cost errors by about 2 eps / (a + b), with
  a = A(d*-1) - A(d*) and b = A(d*+1) - A(d*), so a pixel whose parabola is
  flat, (a + b) < 4e-3 * A(d*) + 2000 * floor, may miss; every such violator is counted and
  returned, and a violator outside that zone fails.

The absolute floor is accounted for separately: ``disp_tie_floor`` counts the
pixels whose integer disparity is accepted only because of the floor (outside
the purely relative 1e-5 tie zone), ``sub_flat_floor`` the subpixel misses
excused only by the floor's share of the flat zone.  Both must be zero for a
report to pass, so the floor is never what decides a pixel.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

AGG_RTOL = 1e-4
AGG_ATOL = 1e-6
TIE_RTOL = 1e-5
TIE_ATOL = 1e-30


def weight_floor(taps: int, c_max: float) -> float:
    """Absolute resolution of the aggregated cost (see the module docstring)."""
    return 2.0 * taps * c_max * 2.0 ** -38 + TIE_ATOL
SUB_ATOL = 1e-3
FLAT_ZONE = 4e-3


@dataclass
class Report:
    n: int = 0
    disp_equal: int = 0
    disp_tie: int = 0
    disp_tie_floor: int = 0
    disp_bad: int = 0
    sub_bad: int = 0
    sub_flat: int = 0
    sub_flat_floor: int = 0
    agg_bad: int = 0
    agg_max_rel: float = 0.0
    notes: List[str] = field(default_factory=list)

    @property
    def ok(self) -> bool:
        return (self.disp_bad == 0 and self.sub_bad == 0 and self.agg_bad == 0
                and self.disp_tie_floor == 0 and self.sub_flat_floor == 0)

    def __str__(self):
        return (f"n={self.n} disp_equal={self.disp_equal} tie={self.disp_tie} "
                f"tie_floor={self.disp_tie_floor} disp_bad={self.disp_bad} sub_bad={self.sub_bad} "
                f"sub_flat={self.sub_flat} sub_flat_floor={self.sub_flat_floor} "
                f"agg_bad={self.agg_bad} agg_max_rel={self.agg_max_rel:.3g} "
                + "; ".join(self.notes[:5]))


def compare_agg(agg_gpu: np.ndarray, agg_o: np.ndarray, rep: Report,
                floor: float = 0.0) -> Report:
    g = np.asarray(agg_gpu, dtype=np.float64)
    o = np.asarray(agg_o, dtype=np.float64)
    err = np.abs(g - o)
    bad = err > AGG_RTOL * np.abs(o) + max(AGG_ATOL, floor)
    rep.agg_bad += int(bad.sum())
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(np.abs(o) > 0, err / np.abs(o), err)
    rep.agg_max_rel = max(rep.agg_max_rel, float(np.nanmax(rel)) if rel.size else 0.0)
    if bad.any():
        i = np.argwhere(bad)[0]
        rep.notes.append(f"agg bad at {tuple(i)}: gpu={g[tuple(i)]!r} oracle={o[tuple(i)]!r}")
    return rep


def compare_maps(disp_gpu, sub_gpu, disp_o, sub_o, agg_o_pd: np.ndarray, d_min: int,
                 rep: Report = None, floor: float = TIE_ATOL) -> Report:
    """agg_o_pd: oracle aggregated costs as [D][n] for the n compared pixels."""
    rep = rep or Report()
    dg = np.asarray(disp_gpu).ravel().astype(np.int64)
    do = np.asarray(disp_o).ravel().astype(np.int64)
    sg = np.asarray(sub_gpu).ravel().astype(np.float64)
    so = np.asarray(sub_o).ravel().astype(np.float64)
    A = np.asarray(agg_o_pd, dtype=np.float64).reshape(agg_o_pd.shape[0], -1)
    n = dg.size
    rep.n += n
    D = A.shape[0]
    if np.any((dg < d_min) | (dg >= d_min + D)):
        rep.disp_bad += int(np.sum((dg < d_min) | (dg >= d_min + D)))
        rep.notes.append("gpu disparity out of range")
        return rep
    idx = np.arange(n)
    ag = A[dg - d_min, idx]
    ao = A[do - d_min, idx]
    eq = dg == do
    rel_gap = TIE_RTOL * np.maximum(np.abs(ag), np.abs(ao))
    tie = (~eq) & (ag - ao <= rel_gap + floor)
    tie_rel = (~eq) & (ag - ao <= rel_gap + TIE_ATOL)
    bad = (~eq) & (~tie)
    rep.disp_equal += int(eq.sum())
    rep.disp_tie += int(tie.sum())
    rep.disp_tie_floor += int((tie & ~tie_rel).sum())
    if (tie & ~tie_rel).any():
        i = int(np.argwhere(tie & ~tie_rel)[0][0])
        rep.notes.append(f"tie only by the floor at {i}: gpu={dg[i]} oracle={do[i]} "
                         f"A_o(gpu)={ag[i]!r} A_o(oracle)={ao[i]!r}")
    rep.disp_bad += int(bad.sum())
    if bad.any():
        i = int(np.argwhere(bad)[0][0])
        rep.notes.append(f"disp bad at {i}: gpu={dg[i]} oracle={do[i]} "
                         f"A_o(gpu)={ag[i]!r} A_o(oracle)={ao[i]!r}")
    # subpixel, where the integer disparities agree
    serr = np.abs(sg - so)
    viol = eq & (serr > SUB_ATOL)
    if viol.any():
        k = do - d_min
        km = np.clip(k - 1, 0, D - 1)
        kp = np.clip(k + 1, 0, D - 1)
        c0 = A[k, idx]
        a = A[km, idx] - c0
        b = A[kp, idx] - c0
        # with the absolute floor as cost error, 2 * eps / (a + b) > 1e-3 px
        flat = (a + b) < FLAT_ZONE * np.abs(c0) + 2e3 * floor
        flat_rel = (a + b) < FLAT_ZONE * np.abs(c0) + 2e3 * TIE_ATOL
        rep.sub_flat += int((viol & flat).sum())
        rep.sub_flat_floor += int((viol & flat & ~flat_rel).sum())
        hard = viol & ~flat
        rep.sub_bad += int(hard.sum())
        if hard.any():
            i = int(np.argwhere(hard)[0][0])
            rep.notes.append(f"sub bad at {i}: gpu={sg[i]!r} oracle={so[i]!r} "
                             f"(a+b)/A={(a[i] + b[i]) / max(abs(c0[i]), 1e-300):.3g}")
    return rep
