"""Seeded synthetic rectified stereo pairs.

This module only produces inputs: textured piecewise-planar scenes rendered
into a left and a right view, plus the ground-truth left disparity.  It holds
no stereo-matching arithmetic (no matching cost, no support weight, no
aggregation), so both the GPU path and the CPU oracle can take their inputs
from it without sharing any of the method's computation.

Geometry follows the paper's setting of a rectified pair (Section I): a scene
point seen at column x in the left view appears at column x - d in the right
view, on the same row, where d >= 0 is its disparity.

Scenes
------
* ``fronto``  - a few fronto-parallel planes with distinct integer disparities;
  texture is uniform uint8 noise smoothed by a 3x3 box.
* ``slanted`` - slanted planes d = dc + gx*(x-cx) + gy*(y-cy), |g| <= 0.1,
  textured by multi-octave value noise; the right view is a linear
  (along-x) backward warp, so disparities are subpixel.
* ``rich``    - ``slanted`` planes plus ellipse-shaped foreground blobs with
  larger disparities, RGB, and low-texture patches (texture amplitude 2).

Planes partition the left view by a seeded Voronoi diagram; blobs are drawn
on top.  In the right view each surface claims the pixels it projects to and
the largest disparity wins (z-buffer).  Right pixels that no surface claims
(regions occluded in the left view) get fresh texture noise.  Gaussian noise
is added to both views before rounding to uint8.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Workload", "StereoPair", "make_pair", "WORKLOADS", "workload",
    "batched_workloads", "surrogate_workload",
]


@dataclass(frozen=True)
class Workload:
    """A stereo-matching problem: image shape, search range, window and weights."""

    name: str
    width: int
    height: int
    channels: int
    d_min: int
    d_max: int
    radius: int
    sigma_s: float          # gamma_d of the spatial weight
    sigma_r: float          # gamma_r of the range weight
    cost_cap: float         # tau of the truncated absolute difference
    scene: str              # 'fronto' | 'slanted' | 'rich'
    seed: int
    noise_sigma: float = 2.0
    n_planes: int = 3
    n_blobs: int = 0
    lowtex_frac: float = 0.0

    @property
    def n_disp(self) -> int:
        return self.d_max - self.d_min + 1

    @property
    def taps(self) -> int:
        return (2 * self.radius + 1) ** 2

    @property
    def work_taps(self) -> int:
        """Pixel x disparity x tap count of the aggregation (one frame)."""
        return self.width * self.height * self.n_disp * self.taps

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


@dataclass
class StereoPair:
    left: np.ndarray        # uint8 [H][W] (gray) or [H][W][3] (RGB)
    right: np.ndarray       # same shape as left
    gt_disp: np.ndarray     # float64 [H][W], left-view disparity of the scene
    occluded: np.ndarray    # bool [H][W], left pixels with no visible match


# The five workloads: a tiny fronto-parallel case, a 450x375 slanted-plane case
# (the quarter-size Middlebury shape), a 1400x1000 RGB case, and the scene
# recipes for the batched and learned-surrogate workloads.
WORKLOADS = {
    "tiny": Workload("fronto3_64x48_gray_d0-15_r4", 64, 48, 1, 0, 15, 4, 4.0, 10.0, 40.0,
                     scene="fronto", seed=1, noise_sigma=2.0, n_planes=3),
    "mid": Workload("slanted8_450x375_gray_d0-63_r7", 450, 375, 1, 0, 63, 7, 7.0, 10.0, 40.0,
                    scene="slanted", seed=2, noise_sigma=2.0, n_planes=8),
    "large": Workload("rich25_1400x1000_rgb_d0-159_r10", 1400, 1000, 3, 0, 159, 10, 10.0, 12.0,
                      60.0, scene="rich", seed=3, noise_sigma=3.0, n_planes=20, n_blobs=5,
                      lowtex_frac=0.05),
}


def workload(key: str) -> Workload:
    return WORKLOADS[key]


BATCH_SIZES = [(320, 240), (450, 375), (640, 480), (960, 720), (1280, 960)]
BATCH_DRANGES = [32, 64, 96, 128]
BATCH_RADII = [5, 7, 10]


def batched_workloads(n: int = 64, base_seed: int = 1000) -> List[Workload]:
    """The uneven batch: per pair a size, disparity range and radius drawn uniformly."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(base_seed + i)
        w, h = BATCH_SIZES[int(rng.integers(len(BATCH_SIZES)))]
        nd = BATCH_DRANGES[int(rng.integers(len(BATCH_DRANGES)))]
        r = BATCH_RADII[int(rng.integers(len(BATCH_RADII)))]
        out.append(Workload(f"batch{i}_{w}x{h}_d0-{nd - 1}_r{r}", w, h, 1, 0, nd - 1, r,
                            float(r), 10.0, 40.0, scene="slanted", seed=base_seed + i,
                            noise_sigma=2.0, n_planes=8))
    return out


def surrogate_workload(seed: int, radius: int = 10) -> Workload:
    """640x480 gray, 96 disparities, slanted-plane scene (learned-surrogate data)."""
    return Workload(f"surr_{seed}_640x480_d0-95_r{radius}", 640, 480, 1, 0, 95, radius,
                    float(radius), 10.0, 40.0, scene="slanted", seed=seed, noise_sigma=2.0,
                    n_planes=8)


# --------------------------------------------------------------------------------------
# texture generators


def _box3(img: np.ndarray) -> np.ndarray:
    """3x3 box mean with edge replication (texture smoothing only)."""
    p = np.pad(img, ((1, 1), (1, 1)), mode="edge")
    acc = np.zeros_like(img, dtype=np.float64)
    for dy in range(3):
        for dx in range(3):
            acc += p[dy:dy + img.shape[0], dx:dx + img.shape[1]]
    return acc / 9.0


def _value_noise(rng: np.random.Generator, h: int, w: int,
                 periods=(64, 32, 16, 8, 4), persistence: float = 0.5) -> np.ndarray:
    """Multi-octave value noise in roughly [-1, 1] (smoothstep-interpolated lattice)."""
    out = np.zeros((h, w), dtype=np.float64)
    amp, total = 1.0, 0.0
    for period in periods:
        gh, gw = h // period + 3, w // period + 3
        grid = rng.uniform(-1.0, 1.0, size=(gh, gw))
        oy, ox = rng.uniform(0.0, period, size=2)
        ys = (np.arange(h) + oy) / period
        xs = (np.arange(w) + ox) / period
        iy = np.floor(ys).astype(np.int64)
        ix = np.floor(xs).astype(np.int64)
        fy = ys - iy
        fx = xs - ix
        fy = fy * fy * (3.0 - 2.0 * fy)
        fx = fx * fx * (3.0 - 2.0 * fx)
        g00 = grid[iy][:, ix]
        g01 = grid[iy][:, ix + 1]
        g10 = grid[iy + 1][:, ix]
        g11 = grid[iy + 1][:, ix + 1]
        top = g00 * (1 - fx)[None, :] + g01 * fx[None, :]
        bot = g10 * (1 - fx)[None, :] + g11 * fx[None, :]
        out += amp * (top * (1 - fy)[:, None] + bot * fy[:, None])
        total += amp
        amp *= persistence
    return out / total * 1.6


# --------------------------------------------------------------------------------------
# surfaces


@dataclass
class _Surface:
    dc: float
    gx: float
    gy: float
    cx: float
    cy: float
    ox: int      # texture-canvas offset of this surface
    oy: int

    def disp(self, x, y):
        return self.dc + self.gx * (x - self.cx) + self.gy * (y - self.cy)

    def left_x(self, u, y):
        """Left column x whose point lands on right column u: x - disp(x, y) = u."""
        return (u + self.dc - self.gx * self.cx + self.gy * (y - self.cy)) / (1.0 - self.gx)


def _fit_plane(rng, dlo: float, dhi: float, xs, ys, cx, cy, slanted: bool,
               integer: bool) -> Tuple[float, float, float]:
    """Pick (dc, gx, gy) so the plane's disparity stays in [dlo, dhi] over its pixels."""
    if integer:
        return float(rng.integers(int(np.ceil(dlo)), int(np.floor(dhi)) + 1)), 0.0, 0.0
    dc = rng.uniform(dlo + 2.0, dhi - 2.0)
    if not slanted or xs.size == 0:
        return dc, 0.0, 0.0
    ang = rng.uniform(0.0, 2.0 * np.pi)
    mag = rng.uniform(0.0, 0.1)
    gx, gy = mag * np.cos(ang), mag * np.sin(ang)
    for _ in range(60):
        d = dc + gx * (xs - cx) + gy * (ys - cy)
        if d.min() >= dlo and d.max() <= dhi:
            break
        gx *= 0.8
        gy *= 0.8
    else:
        gx = gy = 0.0
    return dc, gx, gy


def make_pair(wl: Workload, seed: Optional[int] = None) -> StereoPair:
    """Render the seeded scene of ``wl`` (``seed`` overrides ``wl.seed``)."""
    rng = np.random.default_rng(wl.seed if seed is None else seed)
    H, W, C = wl.height, wl.width, wl.channels
    integer = wl.scene == "fronto"
    # Disparities of visible surfaces stay strictly inside the search range so that
    # Eq. (10)'s neighbours d-1 and d+1 exist at the true match.
    dlo = max(wl.d_min + 1.0, 2.0)
    dhi = wl.d_max - 1.0
    if integer:
        dhi = min(dhi, 14.0) if wl.d_max >= 15 else dhi

    # texture canvas, shared by all surfaces at distinct offsets
    CH, CW = 2 * H + 8, 2 * W + 8
    if wl.scene == "fronto":
        canv = [_box3(rng.integers(0, 256, size=(CH, CW)).astype(np.float64))
                for _ in range(C)]
    else:
        canv = [128.0 + 100.0 * _value_noise(rng, CH, CW) for _ in range(C)]
    canv = np.stack(canv, axis=-1)                                   # [CH][CW][C]
    amp_mask = np.ones((H, W), dtype=np.float64)
    if wl.lowtex_frac > 0:
        target = wl.lowtex_frac * H * W
        covered = np.zeros((H, W), dtype=bool)
        while covered.sum() < target:
            ph = int(rng.integers(H // 20 + 4, H // 6 + 5))
            pw = int(rng.integers(W // 20 + 4, W // 6 + 5))
            y0 = int(rng.integers(0, H - ph))
            x0 = int(rng.integers(0, W - pw))
            covered[y0:y0 + ph, x0:x0 + pw] = True
        amp_mask[covered] = 2.0 / 100.0   # texture amplitude 2 (vs ~100) in the patches

    # left-view labels: Voronoi partition of the planes, blobs on top
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    n_pl = wl.n_planes
    seeds = np.stack([rng.uniform(0, W, n_pl), rng.uniform(0, H, n_pl)], axis=1)
    d2 = (xx[None] - seeds[:, 0, None, None]) ** 2 + (yy[None] - seeds[:, 1, None, None]) ** 2
    label = np.argmin(d2, axis=0).astype(np.int64)
    surfaces: List[_Surface] = []
    used_ints = set()
    for k in range(n_pl):
        m = label == k
        if integer:
            while True:
                dc = float(rng.integers(int(dlo), int(dhi) + 1))
                if dc not in used_ints or len(used_ints) >= int(dhi - dlo + 1):
                    break
            used_ints.add(dc)
            gx = gy = 0.0
        else:
            dc, gx, gy = _fit_plane(rng, dlo, dhi * 0.8 + dlo * 0.2, xx[m], yy[m],
                                    seeds[k, 0], seeds[k, 1], True, False)
        oy = int(rng.integers(0, CH - H))
        ox = int(rng.integers(0, CW - W))
        surfaces.append(_Surface(dc, gx, gy, seeds[k, 0], seeds[k, 1], ox, oy))
    cur_d = None
    for b in range(wl.n_blobs):
        k = n_pl + b
        cx, cy = rng.uniform(0.15 * W, 0.85 * W), rng.uniform(0.15 * H, 0.85 * H)
        ax, ay = rng.uniform(0.04, 0.12) * W, rng.uniform(0.04, 0.12) * H
        inside = ((xx - cx) / ax) ** 2 + ((yy - cy) / ay) ** 2 <= 1.0
        # foreground: disparities in the upper part of the range
        dc, gx, gy = _fit_plane(rng, dlo + 0.75 * (dhi - dlo), dhi, xx[inside], yy[inside],
                                cx, cy, True, False)
        oy = int(rng.integers(0, CH - H))
        ox = int(rng.integers(0, CW - W))
        s = _Surface(dc, gx, gy, cx, cy, ox, oy)
        if cur_d is None:
            cur_d = np.zeros((H, W))
            for j, sj in enumerate(surfaces):
                m = label == j
                cur_d[m] = sj.disp(xx[m], yy[m])
        sd = s.disp(xx, yy)
        front = inside & (sd > cur_d)
        label[front] = k
        cur_d[front] = sd[front]
        surfaces.append(s)

    def tex(k: int, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        """Surface k's texture at left column x (float, linear along x), row y (int)."""
        s = surfaces[k]
        x = np.clip(x, 0.0, W - 1.0)
        x0 = np.floor(x).astype(np.int64)
        x1 = np.minimum(x0 + 1, W - 1)
        f = (x - x0)[..., None]
        yi = y.astype(np.int64)
        t0 = canv[yi + s.oy, x0 + s.ox]
        t1 = canv[yi + s.oy, x1 + s.ox]
        a0 = amp_mask[yi, x0][..., None]
        a1 = amp_mask[yi, x1][..., None]
        v0 = 128.0 + a0 * (t0 - 128.0)
        v1 = 128.0 + a1 * (t1 - 128.0)
        return v0 * (1.0 - f) + v1 * f

    # left view
    left = np.zeros((H, W, C), dtype=np.float64)
    gt = np.zeros((H, W), dtype=np.float64)
    for k, s in enumerate(surfaces):
        m = label == k
        if not m.any():
            continue
        left[m] = tex(k, xx[m], yy[m])
        gt[m] = s.disp(xx[m], yy[m])

    # right view: every surface claims the right pixels it projects to; larger d wins
    right_d = np.full((H, W), -np.inf)
    right_k = np.full((H, W), -1, dtype=np.int64)
    for k, s in enumerate(surfaces):
        xl = s.left_x(xx, yy)                       # left column seen at right (u, y)
        xr = np.rint(xl).astype(np.int64)
        ok = (xl >= 0.0) & (xl <= W - 1.0)
        xr_c = np.clip(xr, 0, W - 1)
        ok &= label[yy.astype(np.int64), xr_c] == k
        dk = xl - xx
        win = ok & (dk > right_d)
        right_d[win] = dk[win]
        right_k[win] = k
    right = np.zeros((H, W, C), dtype=np.float64)
    for k, s in enumerate(surfaces):
        m = right_k == k
        if not m.any():
            continue
        right[m] = tex(k, s.left_x(xx[m], yy[m]), yy[m])
    holes = right_k < 0
    if holes.any():
        if wl.scene == "fronto":
            fresh = np.stack([_box3(rng.integers(0, 256, size=(H, W)).astype(np.float64))
                              for _ in range(C)], axis=-1)
        else:
            fresh = np.stack([128.0 + 100.0 * _value_noise(rng, H, W) for _ in range(C)],
                             axis=-1)
        right[holes] = fresh[holes]

    # left pixels whose match is off-image or hidden in the right view
    ur = np.rint(xx - gt).astype(np.int64)
    occ = ur < 0
    urc = np.clip(ur, 0, W - 1)
    occ |= right_k[yy.astype(np.int64), urc] != label

    left += rng.normal(0.0, wl.noise_sigma, size=left.shape)
    right += rng.normal(0.0, wl.noise_sigma, size=right.shape)
    L8 = np.clip(np.rint(left), 0, 255).astype(np.uint8)
    R8 = np.clip(np.rint(right), 0, 255).astype(np.uint8)
    if C == 1:
        L8, R8 = L8[..., 0], R8[..., 0]
    return StereoPair(np.ascontiguousarray(L8), np.ascontiguousarray(R8), gt, occ)


def textured_fronto_pair(width: int, height: int, d0: int, seed: int,
                         channels: int = 1) -> Tuple[np.ndarray, np.ndarray]:
    """Noise-free pair of one fronto-parallel plane at integer disparity d0.

    R(x, y) = L(x + d0, y), so every left pixel with x >= d0 matches exactly at d0.
    Columns of R that see past the right edge of the texture get fresh noise.
    """
    rng = np.random.default_rng(seed)
    shape = (height, width + d0) + ((channels,) if channels > 1 else ())
    tex = rng.integers(0, 256, size=shape).astype(np.uint8)
    left = np.ascontiguousarray(tex[:, :width])
    right = np.ascontiguousarray(tex[:, d0:d0 + width])
    return left, right
