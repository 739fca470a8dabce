"""Fast bilateral stereo on MI355X (gfx950).

The compute path is the HIP library ``libfbs.so`` behind the C ABI of
``include/fbs.h``; :mod:`._lib` binds it with ctypes.  The helpers here only
allocate outputs with torch and forward to the C ABI: every step of the
stereo path runs in the library's kernels.  Importing the package loads
nothing; the first call loads ``libfbs.so`` and raises if it is missing.
"""
from __future__ import annotations

from typing import Optional, Tuple

__all__ = ["params_for", "run", "cost", "aggregate", "wta_subpixel", "workspace", "run_lr",
           "cost_lr", "lrc", "wmf", "guided_ranges", "run_ranged"]


def params_for(wl, cost_type: int = 0, ncc_radius: int = 1, flags: int = 0):
    """fbs_params for a :class:`scenes.Workload`."""
    from . import _lib
    return _lib.make_params(wl.width, wl.height, wl.channels, wl.d_min, wl.d_max, wl.radius,
                            wl.sigma_s, wl.sigma_r, wl.cost_cap, cost_type, ncc_radius, flags)


def _dev(t):
    return t.device


def workspace(p, device):
    """Workspace tensor for fbs_cost / fbs_run (None when none is needed)."""
    import torch
    from . import _lib
    n = _lib.fbs_workspace_bytes(p)
    if n == 0:
        return None
    return torch.empty(n, dtype=torch.uint8, device=device)


def run(p, left, right, want_agg: bool = False, stream=None):
    """fbs_run on device images -> (disp int32, disp_sub float32[, agg float32])."""
    import torch
    from . import _lib
    H, W, D = p.height, p.width, p.d_max - p.d_min + 1
    dev = _dev(left)
    disp = torch.empty((H, W), dtype=torch.int32, device=dev)
    sub = torch.empty((H, W), dtype=torch.float32, device=dev)
    agg = torch.empty((D, H, W), dtype=torch.float32, device=dev) if want_agg else None
    _lib.fbs_run(p, left, right, disp, sub, agg, workspace(p, dev), stream)
    return (disp, sub, agg) if want_agg else (disp, sub)


def cost(p, left, right, stream=None):
    import torch
    from . import _lib
    D = p.d_max - p.d_min + 1
    out = torch.empty((D, p.height, p.width), dtype=torch.float32, device=_dev(left))
    _lib.fbs_cost(p, left, right, out, workspace(p, _dev(left)), stream)
    return out


def aggregate(p, left, cost_vol, stream=None):
    import torch
    from . import _lib
    out = torch.empty_like(cost_vol)
    _lib.fbs_aggregate(p, left, cost_vol, out, stream)
    return out


def wta_subpixel(p, agg, stream=None):
    import torch
    from . import _lib
    H, W = agg.shape[1], agg.shape[2]
    disp = torch.empty((H, W), dtype=torch.int32, device=agg.device)
    sub = torch.empty((H, W), dtype=torch.float32, device=agg.device)
    _lib.fbs_wta_subpixel(p, agg, disp, sub, stream)
    return disp, sub


def run_lr(p, left, right, max_diff: int = 0, stream=None):
    """fbs_run_lr -> (disp_left, disp_right int32, valid uint8, disp_sub float32)."""
    import torch
    from . import _lib
    H, W = p.height, p.width
    dev = _dev(left)
    dl = torch.empty((H, W), dtype=torch.int32, device=dev)
    dr = torch.empty((H, W), dtype=torch.int32, device=dev)
    valid = torch.empty((H, W), dtype=torch.uint8, device=dev)
    sub = torch.empty((H, W), dtype=torch.float32, device=dev)
    ws = torch.empty(_lib.fbs_lr_workspace_bytes(p), dtype=torch.uint8, device=dev)
    _lib.fbs_run_lr(p, left, right, max_diff, dl, dr, valid, sub, ws, stream)
    return dl, dr, valid, sub


def cost_lr(p, left, right, stream=None):
    """fbs_cost_lr -> (cost_left, cost_right) float32 [D][H][W]."""
    import torch
    from . import _lib
    D = p.d_max - p.d_min + 1
    cl = torch.empty((D, p.height, p.width), dtype=torch.float32, device=_dev(left))
    cr = torch.empty_like(cl)
    _lib.fbs_cost_lr(p, left, right, cl, cr, workspace(p, _dev(left)), stream)
    return cl, cr


def lrc(p, disp_left, disp_right, max_diff: int = 0, disp_sub=None, stream=None):
    """fbs_lrc -> valid uint8 [H][W]; disp_sub (if given) gets -1 where it fails."""
    import torch
    from . import _lib
    valid = torch.empty(disp_left.shape, dtype=torch.uint8, device=disp_left.device)
    _lib.fbs_lrc(p, disp_left, disp_right, max_diff, valid, disp_sub, stream)
    return valid


def wmf(p, reference, disp_in, stream=None):
    """fbs_wmf -> int32 [H][W] weighted median of disp_in."""
    import torch
    from . import _lib
    out = torch.empty_like(disp_in)
    _lib.fbs_wmf(p, reference, disp_in, out, stream)
    return out


def guided_ranges(p, disp_seed, valid, halo: int, margin: int, stream=None):
    """fbs_guided_ranges -> int32 [tiles_y][tiles_x][2] ranges."""
    import torch
    from . import _lib
    tw, th = _lib.fbs_range_tile(p)
    out = torch.empty(((p.height + th - 1) // th, (p.width + tw - 1) // tw, 2),
                      dtype=torch.int32, device=disp_seed.device)
    _lib.fbs_guided_ranges(p, disp_seed, valid, halo, margin, out, stream)
    return out


def run_ranged(p, left, right, ranges, stream=None):
    """fbs_run_ranged -> (disp int32, disp_sub float32)."""
    import torch
    from . import _lib
    disp = torch.empty((p.height, p.width), dtype=torch.int32, device=left.device)
    sub = torch.empty((p.height, p.width), dtype=torch.float32, device=left.device)
    _lib.fbs_run_ranged(p, left, right, ranges, disp, sub, stream)
    return disp, sub
