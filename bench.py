#!/usr/bin/env python3
"""Benchmark of the fused fast-bilateral-stereo path on one MI355X.

One step = one ``fbs_run`` (cost, weights, Eq. 6 aggregation, WTA, Eq. 10)
over the 450x375 gray, 64-disparity, 15x15-window slanted-plane pair, with
both images already resident in HBM.  Prints ONE JSON line with frames/s,
pixel*disparity*tap rate, the roofline of the fused kernel measured live with
HIP events on the stream it runs on, and the FP64 CPU oracle timed on the
host's cores as a reported baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frames/s and Gpix*disp*tap/s, plain FBS vs surrogate/batched, at bad-1px<=2%"

# MI355X peaks (dense): HBM3E bandwidth and the compute ceilings of each unit.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VALU_TFLOPS = 157.3      # published fp32 vector peak (counts packed FP32)
PEAK_FP16_MFMA_TFLOPS = 2500.0     # dense fp16 matrix peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="mid", choices=["tiny", "mid", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--force-valu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    return ap.parse_args()


def cpu_baseline(wl, pair, target_s: float):
    """The FP64 oracle, as it stands, on full frames of the same workload."""
    import oracle
    from oracle import Problem
    pb = Problem.from_workload(wl)
    t0 = time.perf_counter()
    oracle.fbs(pb, pair.left, pair.right)
    t1 = time.perf_counter() - t0
    reps = 1
    if t1 < target_s:
        extra = max(0, min(500, int(target_s / max(t1, 1e-3)) - 1))
        t0 = time.perf_counter()
        for _ in range(extra):
            oracle.fbs(pb, pair.left, pair.right)
        t_extra = time.perf_counter() - t0
        if extra:
            reps, t1 = 1 + extra, t1 + t_extra
    fps = reps / t1
    return {
        "value": fps, "unit": "frames/s", "cores": oracle.threads(), "kind": "oracle",
        "gpix_disp_tap_per_s": wl.work_taps * fps / 1e9,
        "sample": f"{reps} full {wl.width}x{wl.height} frame(s), D={wl.n_disp}, "
                  f"r={wl.radius}, {t1:.1f} s total",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the fused path is a "
              "single-GPU kernel and no multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1807_02044_amd import _lib as L
    from paper_1807_02044_amd import scenes
    import paper_1807_02044_amd as fbs

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = scenes.workload(args.workload)
    pair = scenes.make_pair(wl)
    flags = L.FBS_F_FORCE_VALU if args.force_valu else 0
    p = fbs.params_for(wl, flags=flags)
    variant = L.fbs_run_variant(p)
    Ld = torch.from_numpy(pair.left).to(dev)
    Rd = torch.from_numpy(pair.right).to(dev)
    disp = torch.empty((wl.height, wl.width), dtype=torch.int32, device=dev)
    sub = torch.empty((wl.height, wl.width), dtype=torch.float32, device=dev)
    ws = fbs.workspace(p, dev)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            L.fbs_run(p, Ld, Rd, disp, sub, None, ws, stream)
        stream.synchronize()
        # per-launch events on the kernel's own stream
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            ev[i][0].record(stream)
            L.fbs_run(p, Ld, Rd, disp, sub, None, ws, stream)
            ev[i][1].record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    kern_ms = sorted(a.elapsed_time(b) for a, b in ev)
    avg_ms = sum(kern_ms) / len(kern_ms)
    ms_per_step = wall * 1e3 / args.steps
    fps = args.steps / wall
    taps = wl.work_taps
    # algorithmic work of the fused kernel per launch: one multiply-add (2 flops)
    # per (pixel, disparity, tap) of Eq. 6
    flops = 2.0 * taps
    achieved_tflops = flops / (avg_ms * 1e-3) / 1e12
    if variant == 1:
        roof = {"bound": "mfma", "peak": PEAK_FP16_MFMA_TFLOPS}
        dtype = "f16x2-split/f32acc"
        kname = "k_fbs_mfma"
    else:
        roof = {"bound": "alu", "peak": PEAK_FP32_VALU_TFLOPS}
        dtype = "f32"
        kname = "k_valu"
    roof.update({"achieved": achieved_tflops, "unit": "TFLOP/s",
                 "frac": achieved_tflops / roof["peak"], "traffic": None,
                 "kernel": kname, "kernel_avg_ms": avg_ms,
                 "kernel_p10_ms": kern_ms[len(kern_ms) // 10],
                 "kernel_p90_ms": kern_ms[(9 * len(kern_ms)) // 10],
                 "flops_per_launch": flops})
    out = {
        "metric": METRIC,
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": wl.name, "width": wl.width, "height": wl.height,
            "channels": wl.channels, "disparities": wl.n_disp, "radius": wl.radius,
            "sigma_s": wl.sigma_s, "sigma_r": wl.sigma_r, "cost_cap": wl.cost_cap,
            "path": "fbs_run", "kernel": kname, "parallelism": "single-gpu",
        },
        "gpix_disp_tap_per_s": taps * fps / 1e9,
        "mde_per_s": wl.width * wl.height * wl.n_disp * fps / 1e6,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, pair, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
