"""Parameter sweeps of the paper's evaluation (Section IV-A, Eqs. 11-12,
Figs. 4-6; Section IV-B, Fig. 7) on seeded synthetic scenes with ground truth.

e_PEP (Eq. 11) is the share of evaluated pixels whose estimated disparity is
more than eps_d = 2 away from the ground truth (Eq. 12's delta), in percent.
It is computed over three regions of the left view, as in the paper:

* non_occ          pixels with a visible match (the scene's occlusion mask);
* non_occ_textl    non_occ without texture-less pixels: those whose squared
                   horizontal intensity gradient, averaged over the 3x3
                   neighbourhood, is below 4 (intensity units squared);
* non_occ_discont  non_occ without pixels within 2 px (a 5x5 neighbourhood)
                   of a ground-truth disparity jump larger than 2.

Estimates come from the library's full path with the left-right check
(fbs_run_lr: Eq. 9 then Eq. 10; a pixel whose match the check removed has no
estimate and counts as an error), and from the left-view path alone (fbs_run,
every pixel estimated).  The sweep varies gamma_d, gamma_r and rho one at a
time around a base point and times the fused path per rho.

Run:  python -m paper_1807_02044_amd.sweeps [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import time
from typing import Dict, Iterable, Optional

import numpy as np

EPS_D = 2.0


def pep(est: np.ndarray, gt: np.ndarray, mask: np.ndarray, eps_d: float = EPS_D) -> float:
    """Eq. 11: 100 * (1/N) * sum over the N pixels of `mask` of delta(|est - gt|,
    eps_d), with delta = 1 when the difference exceeds eps_d (Eq. 12).
    Pixels without an estimate (est < 0) are errors."""
    m = np.asarray(mask, dtype=bool)
    n = int(m.sum())
    if n == 0:
        return 0.0
    e = np.asarray(est, dtype=np.float64)[m]
    g = np.asarray(gt, dtype=np.float64)[m]
    err = (e < 0) | (np.abs(e - g) > eps_d)
    return 100.0 * float(err.sum()) / n


def textureless(left: np.ndarray, thresh: float = 4.0) -> np.ndarray:
    """Pixels whose squared horizontal gradient, averaged over 3x3, is below
    `thresh` (gray: the image; RGB: the channel mean)."""
    img = np.asarray(left, dtype=np.float64)
    if img.ndim == 3:
        img = img.mean(axis=2)
    gx = np.zeros_like(img)
    gx[:, 1:-1] = 0.5 * (img[:, 2:] - img[:, :-2])
    g2 = gx * gx
    pad = np.pad(g2, 1, mode="edge")
    H, W = img.shape
    avg = sum(pad[dy:dy + H, dx:dx + W] for dy in range(3) for dx in range(3)) / 9.0
    return avg < thresh


def discontinuities(gt: np.ndarray, gap: float = 2.0, width: int = 2) -> np.ndarray:
    """Pixels within `width` px (a (2*width+1)^2 neighbourhood) of a jump of
    more than `gap` between horizontally or vertically adjacent ground-truth
    disparities."""
    g = np.asarray(gt, dtype=np.float64)
    H, W = g.shape
    jump = np.zeros((H, W), dtype=bool)
    jx = np.abs(g[:, 1:] - g[:, :-1]) > gap
    jy = np.abs(g[1:, :] - g[:-1, :]) > gap
    jump[:, 1:] |= jx
    jump[:, :-1] |= jx
    jump[1:, :] |= jy
    jump[:-1, :] |= jy
    pad = np.pad(jump, width, mode="constant")
    out = np.zeros((H, W), dtype=bool)
    for dy in range(2 * width + 1):
        for dx in range(2 * width + 1):
            out |= pad[dy:dy + H, dx:dx + W]
    return out


def regions(pair) -> Dict[str, np.ndarray]:
    non_occ = ~np.asarray(pair.occluded, dtype=bool)
    return {
        "non_occ": non_occ,
        "non_occ_textl": non_occ & ~textureless(pair.left),
        "non_occ_discont": non_occ & ~discontinuities(pair.gt_disp),
    }


def evaluate(est: np.ndarray, pair) -> Dict[str, float]:
    return {k: pep(est, pair.gt_disp, m) for k, m in regions(pair).items()}


def run_point(wl, pair, dev, radius: int, gamma_d: float, gamma_r: float,
              timed_steps: int = 0, max_diff: int = 0):
    """One parameter point through the library: e_PEP per region, LRC share,
    and (timed_steps > 0) the fused left-view run time in ms."""
    import torch
    from . import _lib as L
    import paper_1807_02044_amd as fbs
    p = L.make_params(wl.width, wl.height, wl.channels, wl.d_min, wl.d_max, radius, gamma_d,
                      gamma_r, wl.cost_cap)
    Ld = torch.from_numpy(pair.left).to(dev)
    Rd = torch.from_numpy(pair.right).to(dev)
    dl, dr, valid, sub = fbs.run_lr(p, Ld, Rd, max_diff)
    _, sub_left = fbs.run(p, Ld, Rd)
    torch.cuda.synchronize()
    out = {"rho": radius, "gamma_d": gamma_d, "gamma_r": gamma_r,
           "e_pep": evaluate(sub.cpu().numpy(), pair),
           "e_pep_left": evaluate(sub_left.cpu().numpy(), pair),
           "lrc_kept": float(valid.float().mean().item())}
    if timed_steps > 0:
        disp = torch.empty((wl.height, wl.width), dtype=torch.int32, device=dev)
        s = torch.empty((wl.height, wl.width), dtype=torch.float32, device=dev)
        for _ in range(3):
            L.fbs_run(p, Ld, Rd, disp, s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(timed_steps):
            L.fbs_run(p, Ld, Rd, disp, s)
        e1.record()
        torch.cuda.synchronize()
        out["fbs_run_ms"] = e0.elapsed_time(e1) / timed_steps
        out["fbs_run_variant"] = L.fbs_run_variant(p)
    return out


def sweep(wl=None, seeds: Iterable[int] = (2, 12, 22), rhos=(1, 2, 3, 4, 5, 6, 7, 8, 9, 10),
          gammas_d=(1, 2, 4, 7, 10, 15, 25), gammas_r=(2, 5, 10, 15, 20, 30, 50),
          base=(7, 7.0, 10.0), timed_steps: int = 20, dev=None) -> dict:
    """e_PEP vs gamma_d, gamma_r and rho (one varied at a time around `base`
    = (rho, gamma_d, gamma_r)), averaged over the seeded scenes, and the
    fused run time vs rho on the first scene."""
    import torch
    from . import scenes
    wl = wl or scenes.workload("mid")
    dev = dev or torch.device("cuda:0")
    pairs = [scenes.make_pair(wl, seed=s) for s in seeds]
    rho0, gd0, gr0 = base

    def avg(points):
        keys = points[0]["e_pep"].keys()
        res = dict(points[0])
        res["e_pep"] = {k: float(np.mean([p["e_pep"][k] for p in points])) for k in keys}
        res["e_pep_left"] = {k: float(np.mean([p["e_pep_left"][k] for p in points])) for k in keys}
        res["lrc_kept"] = float(np.mean([p["lrc_kept"] for p in points]))
        return res

    def grid(name, values, make):
        rows = []
        for v in values:
            rho, gd, gr = make(v)
            pts = [run_point(wl, pr, dev, rho, gd, gr,
                             timed_steps=timed_steps if (name == "rho" and i == 0) else 0)
                   for i, pr in enumerate(pairs)]
            rows.append(avg(pts) if name != "rho" else {**avg(pts), **{
                k: pts[0][k] for k in ("fbs_run_ms", "fbs_run_variant") if k in pts[0]}})
        return rows

    t0 = time.perf_counter()
    out = {
        "workload": wl.name, "seeds": list(seeds), "eps_d": EPS_D,
        "base": {"rho": rho0, "gamma_d": gd0, "gamma_r": gr0},
        "gamma_d": grid("gamma_d", gammas_d, lambda v: (rho0, float(v), gr0)),
        "gamma_r": grid("gamma_r", gammas_r, lambda v: (rho0, gd0, float(v))),
        "rho": grid("rho", rhos, lambda v: (int(v), gd0, gr0)),
    }
    out["wall_s"] = time.perf_counter() - t0
    return out


def table(res: dict) -> str:
    lines = [f"workload {res['workload']}, seeds {res['seeds']}, eps_d {res['eps_d']}, "
             f"base {res['base']}"]
    for name in ("gamma_d", "gamma_r", "rho"):
        lines.append("")
        hdr = (f"{name:>8} {'non_occ':>9} {'textl':>9} {'discont':>9} {'kept':>6} "
               f"{'left:non_occ':>13} {'textl':>9} {'discont':>9}")
        if name == "rho":
            hdr += f" {'fbs_run_ms':>11}"
        lines.append(hdr)
        for r in res[name]:
            e, f = r["e_pep"], r["e_pep_left"]
            row = (f"{r[name]:>8} {e['non_occ']:9.2f} {e['non_occ_textl']:9.2f} "
                   f"{e['non_occ_discont']:9.2f} {r['lrc_kept']:6.3f} {f['non_occ']:13.2f} "
                   f"{f['non_occ_textl']:9.2f} {f['non_occ_discont']:9.2f}")
            if name == "rho" and "fbs_run_ms" in r:
                row += f" {r['fbs_run_ms']:11.4f}"
            lines.append(row)
    return "\n".join(lines)


def main(argv: Optional[list] = None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="write the JSON result here")
    ap.add_argument("--seeds", type=int, nargs="*", default=[2, 12, 22])
    args = ap.parse_args(argv)
    res = sweep(seeds=args.seeds)
    print(table(res), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
