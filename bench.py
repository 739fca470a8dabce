#!/usr/bin/env python3
"""Benchmark of the fused fast-bilateral-stereo path on one MI355X.

One step = one ``fbs_run`` (cost, weights, Eq. 6 aggregation, WTA, Eq. 10)
over the 1400x1000 RGB, 160-disparity, 21x21-window scene of 20 slanted
planes and 5 blobs (the largest single-GPU workload), with both images already
resident in HBM.  Prints ONE JSON line with frames/s, pixel*disparity*tap
rate, the roofline of the fused kernel measured live with HIP events on the
stream it runs on, and the FP64 CPU oracle timed on the host's cores as a
reported baseline.  Extra keys: the two smaller single-pair workloads, the
end-to-end rate with the host transfers, the left-right path (Eq. 9), the
64-pair batched plan and the learned surrogate.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frames/s and Gpix*disp*tap/s, plain FBS vs surrogate/batched, at bad-1px<=2%"

# MI355X peaks (dense): HBM3E bandwidth and the compute ceilings of each unit.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VALU_TFLOPS = 157.3      # published fp32 vector peak (counts packed FP32)
PEAK_FP16_MFMA_TFLOPS = 2500.0     # dense fp16 matrix peak

# HBM bytes per launch of the fused kernel from two rocprofv3 PMC runs
# (FETCH_SIZE, WRITE_SIZE), each scaled by what the counter reads for a
# 1 GiB device copy.  Valid only for the kernel source they were taken on.
MEASURED_TRAFFIC = {
    "rich25_1400x1000_rgb_d0-159_r10": {
        "sources": ["paper_1807_02044_amd/csrc/mfma_tile.h", "paper_1807_02044_amd/csrc/k_mfma.hip"],
        "sha256": "e61133e20c18c875cf646b532e16ca7437c1a726c31764a60fff1aad25b7b6a1",
        # FETCH_SIZE 27086.7 KiB x 2.0 + WRITE_SIZE 10937.5 KiB x 1.0
        "bytes_per_launch": 66.67e6,
    },
}


# Counter-derived utilisation of the fused kernel (rocprofv3 PMC runs of the
# profiled command): VALU issue and matrix-pipe busy shares of the SIMD time
# of one launch.  Valid only for the kernel source they were taken on.
MEASURED_UTIL = {
    "rich25_1400x1000_rgb_d0-159_r10": {
        "sources": ["paper_1807_02044_amd/csrc/mfma_tile.h", "paper_1807_02044_amd/csrc/k_mfma.hip"],
        "sha256": "e61133e20c18c875cf646b532e16ca7437c1a726c31764a60fff1aad25b7b6a1",
        # SQ_INSTS_VALU x 4 cycles and SQ_VALU_MFMA_BUSY_CYCLES over the SIMD-cycles
        # of a 1.290 ms launch (1024 SIMDs at 2.4 GHz); SQ_LDS_BANK_CONFLICT over
        # SQ_LDS_IDX_ACTIVE
        "valu_issue_frac": 0.498,
        "mfma_busy_frac": 0.160,
        "lds_bank_conflict_frac": 0.244,
        "counters_kernel_avg_ms": 1.290,
    },
    "slanted8_450x375_gray_d0-63_r7": {
        "sources": ["paper_1807_02044_amd/csrc/mfma_tile.h", "paper_1807_02044_amd/csrc/k_mfma.hip"],
        "sha256": "e61133e20c18c875cf646b532e16ca7437c1a726c31764a60fff1aad25b7b6a1",
        "valu_issue_frac": 0.528,
        "mfma_busy_frac": 0.134,
        "counters_kernel_avg_ms": 0.05006,
    },
}


def _sources_sha(sources):
    import hashlib
    h = hashlib.sha256()
    try:
        for src in sources:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    return h.hexdigest()


def measured_utilisation(workload: str):
    m = MEASURED_UTIL.get(workload)
    if not m or _sources_sha(m["sources"]) != m["sha256"]:
        return None
    return {k: v for k, v in m.items() if k not in ("sources", "sha256")}


def measured_traffic(workload: str):
    m = MEASURED_TRAFFIC.get(workload)
    if not m or _sources_sha(m["sources"]) != m["sha256"]:
        return None
    return m["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large", choices=["tiny", "mid", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--force-valu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-pair batched-plan comparison")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned-surrogate comparison")
    ap.add_argument("--surrogate-frames", type=int, default=200,
                    help="held-out pairs of the surrogate evaluation")
    ap.add_argument("--no-two-streams", action="store_true",
                    help="skip the two-frames-in-flight leg (profiles of single-stream launches)")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="skip the smaller single-pair workloads")
    ap.add_argument("--no-e2e", action="store_true",
                    help="skip the end-to-end leg with host transfers")
    ap.add_argument("--no-lr", action="store_true",
                    help="skip the left-right path (both views and Eq. 9)")
    ap.add_argument("--lr-steps", type=int, default=20)
    ap.add_argument("--no-guided", action="store_true",
                    help="skip the guided-search-range leg")
    ap.add_argument("--guided-frames", type=int, default=32)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed loop, copy this many MiB device to device once "
                         "(a kernel of known traffic that calibrates rocprofv3 byte counters)")
    ap.add_argument("--tune-cache", default=os.path.join(tempfile.gettempdir(),
                                                          "fbs_tune_gfx950.json"))
    return ap.parse_args()


def _gen_pair(wl):
    from paper_1807_02044_amd import scenes
    p = scenes.make_pair(wl)
    return p.left, p.right


def batched(args, dev):
    """64 uneven pairs: one graph launch of a tuned plan vs 64 fbs_run calls."""
    import concurrent.futures as cf

    import torch
    from paper_1807_02044_amd import _lib as L
    from paper_1807_02044_amd import scenes
    import paper_1807_02044_amd as fbs

    wls = scenes.batched_workloads()
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(workers) as ex:
        imgs = list(ex.map(_gen_pair, wls))
    gen_s = time.perf_counter() - t0
    params = [fbs.params_for(wl) for wl in wls]
    Ls = [torch.from_numpy(a).to(dev) for a, _ in imgs]
    Rs = [torch.from_numpy(b).to(dev) for _, b in imgs]
    Ds = [torch.empty((w.height, w.width), dtype=torch.int32, device=dev) for w in wls]
    Ss = [torch.empty((w.height, w.width), dtype=torch.float32, device=dev) for w in wls]
    Ds_seq = [torch.empty_like(t) for t in Ds]
    Ss_seq = [torch.empty_like(t) for t in Ss]
    # persistent plan: fbs_run's heuristic configurations (most resident waves);
    # per-tile plan: tuned ones.  The tuner times each shape alone, and its
    # per-shape optimum helps the per-tile launch but not the persistent one,
    # whose classes share the GPU with each other.
    t0 = time.perf_counter()
    plan = L.FbsPlan(params, tune_cache=args.tune_cache)
    plan_s = time.perf_counter() - t0
    stream = torch.cuda.Stream(device=dev)
    taps = sum(w.work_taps for w in wls)

    def timed(fn):
        with torch.cuda.stream(stream):
            fn()
            stream.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.batch_steps):
                fn()
            e1.record(stream)
            stream.synchronize()
        return e0.elapsed_time(e1) / args.batch_steps

    def graph():
        plan.launch(Ls, Rs, Ds, Ss, stream)

    def sequential():
        for i in range(len(wls)):
            L.fbs_run(params[i], Ls[i], Rs[i], Ds_seq[i], Ss_seq[i], None, None, stream)

    def equal_pairs():
        """Pairs whose graph outputs equal the sequential ones bit for bit."""
        torch.cuda.synchronize()
        return sum(int(torch.equal(Ds[i], Ds_seq[i]) and
                       torch.equal(Ss[i].view(torch.int32), Ss_seq[i].view(torch.int32)))
                   for i in range(len(wls)))

    ms_graph = timed(graph)
    ms_seq = timed(sequential)
    eq_persistent = equal_pairs()
    t0 = time.perf_counter()
    plan_pt = L.FbsPlan(params, tune_cache=args.tune_cache, tune=True, per_tile=True)
    plan_pt_s = time.perf_counter() - t0

    def graph_per_tile():
        plan_pt.launch(Ls, Rs, Ds, Ss, stream)

    for t in Ds + Ss:
        t.fill_(-1)
    ms_graph_pt = timed(graph_per_tile)
    eq_per_tile = equal_pairs()
    plan_pt.close()
    if eq_persistent != len(wls) or eq_per_tile != len(wls):
        raise RuntimeError(f"batched outputs differ from fbs_run: persistent {eq_persistent}, "
                           f"per-tile {eq_per_tile} of {len(wls)} pairs bit-identical")
    cfgs = [plan.pair_config(i) for i in range(len(wls))]
    launches = plan.num_launches()
    plan.close()
    n = len(wls)
    return {
        "pairs": n, "taps": taps, "megapixels": sum(w.width * w.height for w in wls) / 1e6,
        "graph_ms": ms_graph, "sequential_ms": ms_seq,
        "frames_per_s_graph": n / (ms_graph * 1e-3),
        "frames_per_s_sequential": n / (ms_seq * 1e-3),
        "gpix_disp_tap_per_s_graph": taps / (ms_graph * 1e-3) / 1e9,
        "gpix_disp_tap_per_s_sequential": taps / (ms_seq * 1e-3) / 1e9,
        "speedup": ms_seq / ms_graph, "host_launches_graph": launches,
        "per_tile_graph_ms": ms_graph_pt, "per_tile_speedup": ms_seq / ms_graph_pt,
        "host_launches_sequential": n,
        "bitwise_equal_pairs": {"persistent": eq_persistent, "per_tile": eq_per_tile},
        "waves_per_wg": sorted({c[1] for c in cfgs}), "slab_blocks": sorted({c[2] for c in cfgs}),
        "scene_gen_s": gen_s, "plan_create_s": plan_s, "per_tile_plan_create_s": plan_pt_s,
        "configs": "persistent: fbs_run heuristic; per-tile: tuned (FBS_PLAN_TUNE)",
        "scenes": "64 seeded slanted-plane pairs, sizes/ranges/radii drawn per pair",
    }


def surrogate(args, dev):
    """Plain full-radius FBS vs the learned surrogate (cheap run + net + gate)
    on held-out 640x480, 96-disparity pairs; quality against the plain run."""
    import concurrent.futures as cf

    import numpy as np
    import torch
    from paper_1807_02044_amd import _lib as L
    from paper_1807_02044_amd import surrogate as SG
    import paper_1807_02044_amd as fbs

    if not os.path.exists(SG.WEIGHTS):
        return {"skipped": "no trained weights"}
    summary = json.load(open(SG.SUMMARY)) if os.path.exists(SG.SUMMARY) else {}
    calib = summary.get("gate_calibrated", {}).get("gate_frac")
    seeds = [SG.EVAL_SEED0 + 100 + i for i in range(args.surrogate_frames)]
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(workers) as ex:
        imgs = list(ex.map(SG._gen, seeds))
    cw, fw = SG.workloads(seeds[0])
    pc, pf = fbs.params_for(cw), fbs.params_for(fw)
    W, H, D = cw.width, cw.height, cw.n_disp
    Ls = [torch.from_numpy(a).to(dev) for a, _ in imgs]
    Rs = [torch.from_numpy(b).to(dev) for _, b in imgs]
    sur = L.FbsSurrogate(W, H, D)
    sur.set_params(np.load(SG.WEIGHTS))
    stream = torch.cuda.Stream(device=dev)
    n = len(seeds)
    plain = [torch.empty((H, W), dtype=torch.float32, device=dev) for _ in range(n)]
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    cheap = torch.empty((H, W), dtype=torch.float32, device=dev)
    feat = torch.empty((H, W, 32), dtype=torch.int16, device=dev)

    def timed(fn):
        with torch.cuda.stream(stream):
            for i in range(n):
                fn(i)
            stream.synchronize()
            t0 = time.perf_counter()
            for i in range(n):
                fn(i)
            stream.synchronize()
        return (time.perf_counter() - t0) / n

    streams2 = [torch.cuda.Stream(device=dev) for _ in range(2)]

    def timed2(fn):
        """Frames alternate over two streams (two frames in flight); the first
        pass warms up, the second is timed."""
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(n):
                fn(i, streams2[i % 2])
            torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    def run_plain(i):
        L.fbs_run(pf, Ls[i], Rs[i], None, plain[i], None, None, stream)

    def run_net(i):
        sur.cheap_run(pc, Ls[i], Rs[i], cheap, feat, stream)
        sur.forward(W, H, feat, cheap, out, stream)

    fb = {}

    def run_gated(frac):
        def f(i):
            fb[i] = sur.run(pc, pf, Ls[i], Rs[i], out, 1.0, frac, stream)
        return f

    t_plain = timed(run_plain)
    t_net = timed(run_net)
    bad, mae = [], []
    with torch.cuda.stream(stream):
        for i in range(n):
            run_net(i)
            e = (out - plain[i]).abs()
            bad.append(float((e > 1.0).float().mean().item()))
            mae.append(float(e.mean().item()))
    res = {
        "frames": n, "workload": f"{W}x{H} gray, d {cw.d_min}..{cw.d_max}, "
                                 f"cheap r={cw.radius} vs plain r={fw.radius}",
        "plain_frames_per_s": 1.0 / t_plain,
        "plain_gpix_disp_tap_per_s": fw.work_taps / t_plain / 1e9,
        "net_path_frames_per_s": 1.0 / t_net,
        "net_bad1_vs_plain": float(np.mean(bad)), "net_mae_vs_plain": float(np.mean(mae)),
    }
    for name, frac in (("specified", 0.05), ("calibrated", calib)):
        if frac is None:
            continue
        t = timed(run_gated(frac))
        rate = float(np.mean([fb[i] for i in range(n)]))
        b = float(np.mean([0.0 if fb[i] else bad[i] for i in range(n)]))
        res[f"gate_{name}"] = {"gate_px": 1.0, "gate_frac": frac, "frames_per_s": 1.0 / t,
                               "fallback_rate": rate, "bad1_vs_plain": b,
                               "speedup_vs_plain": t_plain / t}
    # per-tile fallback (fbs_surrogate_run_tiled), gate calibrated on training pairs
    tg = summary.get("gate_tiles")
    if tg:
        gpx, tfrac = float(tg["gate_px"]), float(tg["tile_frac"])
        t = timed(lambda i: sur.run_tiled(pc, pf, Ls[i], Rs[i], out, gpx, tfrac, stream))
        tb, teq = [], []
        with torch.cuda.stream(stream):
            for i in range(n):
                sur.run_tiled(pc, pf, Ls[i], Rs[i], out, gpx, tfrac, stream)
                tb.append(float(((out - plain[i]).abs() > 1.0).float().mean().item()))
                teq.append(float((out == plain[i]).float().mean().item()))
        # two frames in flight, for plain FBS and the tile-gated path alike
        sur2 = L.FbsSurrogate(W, H, D)
        sur2.set_params(np.load(SG.WEIGHTS))
        outs = [out, torch.empty_like(out)]
        surs = [sur, sur2]
        t2_plain = timed2(lambda i, s: L.fbs_run(pf, Ls[i], Rs[i], None, plain[i], None, None, s))
        t2 = timed2(lambda i, s: surs[i % 2].run_tiled(pc, pf, Ls[i], Rs[i], outs[i % 2], gpx,
                                                       tfrac, s))
        sur2.close()
        res["gate_tiles"] = {"gate_px": gpx, "tile_frac": tfrac, "frames_per_s": 1.0 / t,
                             "bad1_vs_plain": float(np.mean(tb)),
                             "bad1_vs_plain_max": float(np.max(tb)),
                             "pixels_equal_to_plain": float(np.mean(teq)),
                             "speedup_vs_plain": t_plain / t,
                             "two_streams": {"plain_frames_per_s": 1.0 / t2_plain,
                                             "frames_per_s": 1.0 / t2,
                                             "speedup_vs_plain": t2_plain / t2},
                             "calibration": {k: tg[k] for k in ("train_frames", "target_bad1",
                                                                "train_bad1_p90")}}
    sur.close()
    return res


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


def time_fused(L, p, Ld, Rd, disp, sub, ws, stream, steps, warmup):
    """Wall time of `steps` fbs_run calls bracketed by synchronisations, then
    per-launch kernel times from HIP events on the kernel's stream over a
    second pass of the same launches."""
    import torch
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            L.fbs_run(p, Ld, Rd, disp, sub, None, ws, stream)
        stream.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            L.fbs_run(p, Ld, Rd, disp, sub, None, ws, stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for i in range(steps):
            ev[i][0].record(stream)
            L.fbs_run(p, Ld, Rd, disp, sub, None, ws, stream)
            ev[i][1].record(stream)
        stream.synchronize()
    kern_ms = sorted(a.elapsed_time(b) for a, b in ev)
    return wall, kern_ms


def extra_config(name, args, dev, force_valu, cost_type=0):
    """One smaller single-pair workload: frames/s and the kernel time
    (cost_type 1: the paper's NCC cost, Eqs. 1-3, block radius 1: matrix-core
    kernel, or the vector-ALU kernel with force_valu)."""
    import torch
    from paper_1807_02044_amd import _lib as L
    from paper_1807_02044_amd import scenes
    import paper_1807_02044_amd as fbs
    wl = scenes.workload(name)
    pair = scenes.make_pair(wl)
    p = fbs.params_for(wl, cost_type=cost_type,
                       flags=L.FBS_F_FORCE_VALU if force_valu else 0)
    Ld = torch.from_numpy(pair.left).to(dev)
    Rd = torch.from_numpy(pair.right).to(dev)
    disp = torch.empty((wl.height, wl.width), dtype=torch.int32, device=dev)
    sub = torch.empty((wl.height, wl.width), dtype=torch.float32, device=dev)
    stream = torch.cuda.Stream(device=dev)
    steps = max(20, min(200, args.steps * 10))
    wall, kern_ms = time_fused(L, p, Ld, Rd, disp, sub, fbs.workspace(p, dev), stream, steps, 10)
    avg = sum(kern_ms) / len(kern_ms)
    mfma = L.fbs_run_variant(p) == 1
    tflops = 2.0 * wl.work_taps / (avg * 1e-3) / 1e12
    peak = PEAK_FP16_MFMA_TFLOPS if mfma else PEAK_FP32_VALU_TFLOPS
    # the counter figures were taken on the TAD kernel
    util = measured_utilisation(wl.name) if mfma and cost_type != 1 else None
    kernel = ("k_fbs_mfma_ncc" if cost_type == 1 else "k_fbs_mfma") if mfma else "k_valu"
    return {"workload": wl.name, "cost": "ncc" if cost_type == 1 else "tad", **(util or {}),
            "frames_per_s": steps / wall,
            "gpix_disp_tap_per_s": wl.work_taps * steps / wall / 1e9,
            "kernel_avg_ms": avg, "kernel": kernel,
            "achieved_tflops": tflops, "peak_tflops": peak, "frac": tflops / peak,
            "steps": steps}


def end_to_end(args, dev, wl, pair, p, stream):
    """Images from pinned host memory to HBM, the fused run, both maps back."""
    import torch
    from paper_1807_02044_amd import _lib as L
    import paper_1807_02044_amd as fbs
    Lh = torch.from_numpy(pair.left).pin_memory()
    Rh = torch.from_numpy(pair.right).pin_memory()
    Ld, Rd = torch.empty_like(Lh, device=dev), torch.empty_like(Rh, device=dev)
    disp = torch.empty((wl.height, wl.width), dtype=torch.int32, device=dev)
    sub = torch.empty((wl.height, wl.width), dtype=torch.float32, device=dev)
    disp_h = torch.empty(disp.shape, dtype=torch.int32).pin_memory()
    sub_h = torch.empty(sub.shape, dtype=torch.float32).pin_memory()
    ws = fbs.workspace(p, dev)
    steps = max(5, args.steps)

    def step():
        Ld.copy_(Lh, non_blocking=True)
        Rd.copy_(Rh, non_blocking=True)
        L.fbs_run(p, Ld, Rd, disp, sub, None, ws, stream)
        disp_h.copy_(disp, non_blocking=True)
        sub_h.copy_(sub, non_blocking=True)

    with torch.cuda.stream(stream):
        for _ in range(3):
            step()
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        stream.synchronize()
        wall = time.perf_counter() - t0
    nbytes = 2 * Lh.numel() + 8 * wl.width * wl.height
    return {"frames_per_s": steps / wall, "ms_per_frame": wall * 1e3 / steps,
            "host_bytes_per_frame": nbytes, "steps": steps,
            "includes": "H2D of both images (pinned), fbs_run, D2H of disp and disp_sub, "
                        "one stream, frames back to back"}


def left_right(args, dev, wl, pair):
    """The paper's path for both views: right run, left run, Eq. 9, Eq. 10."""
    import torch
    from paper_1807_02044_amd import _lib as L
    import paper_1807_02044_amd as fbs
    p = fbs.params_for(wl)
    Ld = torch.from_numpy(pair.left).to(dev)
    Rd = torch.from_numpy(pair.right).to(dev)
    H, W = wl.height, wl.width
    dl = torch.empty((H, W), dtype=torch.int32, device=dev)
    dr = torch.empty_like(dl)
    valid = torch.empty((H, W), dtype=torch.uint8, device=dev)
    sub = torch.empty((H, W), dtype=torch.float32, device=dev)
    ws = torch.empty(L.fbs_lr_workspace_bytes(p), dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)
    steps = max(3, args.lr_steps)
    with torch.cuda.stream(stream):
        for _ in range(2):
            L.fbs_run_lr(p, Ld, Rd, 0, dl, dr, valid, sub, ws, stream)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            L.fbs_run_lr(p, Ld, Rd, 0, dl, dr, valid, sub, ws, stream)
        stream.synchronize()
        wall = time.perf_counter() - t0
    kept = float(valid.float().mean().item())
    return {"workload": wl.name, "frames_per_s": steps / wall,
            "gpix_disp_tap_per_s": 2 * wl.work_taps * steps / wall / 1e9,
            "mde_per_s": W * H * wl.n_disp * steps / wall / 1e6,
            "lrc_kept_fraction": kept, "max_diff": 0, "steps": steps,
            "includes": "fbs_run_lr: image mirror, right-reference run, left-reference run, "
                        "Eq. 9 and Eq. 10 (two volumes' work)"}


def guided(args, dev):
    """Search ranges suggested by reliable pixels (the paper's future work)
    against the plain full-range run, on held-out 640x480 pairs (D=96, r=10):
    seeds from a cheap radius-3 left-right run, per-tile ranges (halo 10,
    margin 3), the full-radius run over the ranges only."""
    import concurrent.futures as cf

    import numpy as np
    import torch
    from paper_1807_02044_amd import _lib as L
    from paper_1807_02044_amd import surrogate as SG
    import paper_1807_02044_amd as fbs

    seeds = [SG.EVAL_SEED0 + 100 + i for i in range(args.guided_frames)]
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(workers) as ex:
        imgs = list(ex.map(SG._gen, seeds))
    cw, fw = SG.workloads(seeds[0])
    pc, pf = fbs.params_for(cw), fbs.params_for(fw)
    W, H = fw.width, fw.height
    Ls = [torch.from_numpy(a).to(dev) for a, _ in imgs]
    Rs = [torch.from_numpy(b).to(dev) for _, b in imgs]
    n = len(seeds)
    stream = torch.cuda.Stream(device=dev)
    tw, th = L.fbs_range_tile(pf)
    plain = [torch.empty((H, W), dtype=torch.float32, device=dev) for _ in range(n)]
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    dl = torch.empty((H, W), dtype=torch.int32, device=dev)
    valid = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ws = torch.empty(L.fbs_lr_workspace_bytes(pc), dtype=torch.uint8, device=dev)
    rg = torch.empty(((H + th - 1) // th, (W + tw - 1) // tw, 2), dtype=torch.int32, device=dev)
    halo, margin = fw.radius, 3

    def run_plain(i):
        L.fbs_run(pf, Ls[i], Rs[i], None, plain[i], None, None, stream)

    def run_guided(i):
        L.fbs_run_lr(pc, Ls[i], Rs[i], 0, dl, None, valid, None, ws, stream)
        L.fbs_guided_ranges(pf, dl, valid, halo, margin, rg, stream)
        L.fbs_run_ranged(pf, Ls[i], Rs[i], rg, None, out, stream)

    def timed(fn):
        with torch.cuda.stream(stream):
            for i in range(n):
                fn(i)
            stream.synchronize()
            t0 = time.perf_counter()
            for i in range(n):
                fn(i)
            stream.synchronize()
        return (time.perf_counter() - t0) / n

    t_plain = timed(run_plain)
    t_guided = timed(run_guided)
    bad, width = [], []
    with torch.cuda.stream(stream):
        for i in range(n):
            run_guided(i)
            bad.append(float(((out - plain[i]).abs() > 1.0).float().mean().item()))
            width.append(float((rg[..., 1] - rg[..., 0] + 1).float().mean().item()))
    b = np.asarray(bad)
    return {"frames": n, "workload": f"{W}x{H} gray, d {fw.d_min}..{fw.d_max}, r={fw.radius}; "
                                     f"seeds from r={cw.radius} left-right run",
            "halo": halo, "margin": margin, "tile": [tw, th],
            "plain_frames_per_s": 1.0 / t_plain, "guided_frames_per_s": 1.0 / t_guided,
            "speedup_vs_plain": t_plain / t_guided,
            "bad1_vs_plain_mean": float(b.mean()), "bad1_vs_plain_max": float(b.max()),
            "mean_range_width": float(np.mean(width))}


def guided_headline(args, dev, wl, pair):
    """The guided-range pipeline on the headline pair (wider disparity range):
    seeds from a radius-3 left-right run of the same pair, per-tile ranges
    (halo = the full radius, margin 3), the full-radius run over the ranges;
    against the plain full-range run.  Per-stage times from HIP events on the
    pipeline's stream."""
    import torch
    from paper_1807_02044_amd import _lib as L
    import paper_1807_02044_amd as fbs
    pf = fbs.params_for(wl)
    pc = fbs.params_for(wl.with_(radius=3, sigma_s=3.0))
    Ld = torch.from_numpy(pair.left).to(dev)
    Rd = torch.from_numpy(pair.right).to(dev)
    H, W = wl.height, wl.width
    tw, th = L.fbs_range_tile(pf)
    dl = torch.empty((H, W), dtype=torch.int32, device=dev)
    valid = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ws = torch.empty(L.fbs_lr_workspace_bytes(pc), dtype=torch.uint8, device=dev)
    rg = torch.empty(((H + th - 1) // th, (W + tw - 1) // tw, 2), dtype=torch.int32, device=dev)
    plain = torch.empty((H, W), dtype=torch.float32, device=dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    halo, margin = wl.radius, 3
    stream = torch.cuda.Stream(device=dev)
    steps = max(3, args.lr_steps)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def run_plain():
        L.fbs_run(pf, Ld, Rd, None, plain, None, None, stream)

    def run_guided(marks=None):
        if marks:
            marks[0].record(stream)
        L.fbs_run_lr(pc, Ld, Rd, 0, dl, None, valid, None, ws, stream)
        if marks:
            marks[1].record(stream)
        L.fbs_guided_ranges(pf, dl, valid, halo, margin, rg, stream)
        if marks:
            marks[2].record(stream)
        L.fbs_run_ranged(pf, Ld, Rd, rg, None, out, stream)
        if marks:
            marks[3].record(stream)

    def timed(fn):
        with torch.cuda.stream(stream):
            for _ in range(2):
                fn()
            stream.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            stream.synchronize()
        return (time.perf_counter() - t0) / steps

    t_plain = timed(run_plain)
    t_guided = timed(run_guided)
    stages = [[], [], []]
    with torch.cuda.stream(stream):
        for _ in range(steps):
            m = [ev() for _ in range(4)]
            run_guided(m)
            stream.synchronize()
            for k in range(3):
                stages[k].append(m[k].elapsed_time(m[k + 1]))
        run_plain()
        stream.synchronize()
    bad = float(((out - plain).abs() > 1.0).float().mean().item())
    width = float((rg[..., 1] - rg[..., 0] + 1).float().mean().item())
    return {"workload": wl.name, "steps": steps, "halo": halo, "margin": margin,
            "tile": [tw, th], "seed_radius": 3,
            "plain_frames_per_s": 1.0 / t_plain, "guided_frames_per_s": 1.0 / t_guided,
            "speedup_vs_plain": t_plain / t_guided,
            "seeds_ms": sum(stages[0]) / steps, "ranges_ms": sum(stages[1]) / steps,
            "ranged_run_ms": sum(stages[2]) / steps,
            "bad1_vs_plain": bad, "mean_range_width": width}


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

    wall, kern_ms = time_fused(L, p, Ld, Rd, disp, sub, ws, stream, args.steps, args.warmup)
    two_streams = None
    if not args.no_two_streams:
        # the same steps with two frames in flight (alternating streams, own
        # outputs): what a serving loop sees once one frame's last tiles
        # overlap the next frame's first
        st2 = [torch.cuda.Stream(device=dev) for _ in range(2)]
        outs2 = [(torch.empty_like(disp), torch.empty_like(sub), fbs.workspace(p, dev))
                 for _ in range(2)]
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.steps):
                d2, s2, w2 = outs2[i % 2]
                L.fbs_run(p, Ld, Rd, d2, s2, None, w2, st2[i % 2])
            torch.cuda.synchronize()
            wall2 = time.perf_counter() - t0
        two_streams = {"frames_per_s": args.steps / wall2,
                       "gpix_disp_tap_per_s": wl.work_taps * args.steps / wall2 / 1e9}
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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
    traffic = measured_traffic(wl.name) if variant == 1 else None
    roof.update({"achieved": achieved_tflops, "unit": "TFLOP/s",
                 "frac": achieved_tflops / roof["peak"],
                 "traffic": traffic,
                 "kernel": kname, "kernel_avg_ms": avg_ms,
                 "kernel_p10_ms": kern_ms[len(kern_ms) // 10],
                 "kernel_p90_ms": kern_ms[(9 * len(kern_ms)) // 10],
                 "flops_per_launch": flops,
                 "algorithmic_bytes_per_launch": (2 * wl.channels + 8) * wl.width * wl.height})
    if traffic:
        roof["hbm_gbs"] = traffic / (avg_ms * 1e-3) / 1e9
        roof["hbm_frac"] = roof["hbm_gbs"] / PEAK_HBM_GBS
    util = measured_utilisation(wl.name) if variant == 1 else None
    if util:
        roof.update(util)
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
    if two_streams:
        out["two_streams"] = two_streams
    if not args.no_extra_configs:
        out["other_configs"] = [extra_config(n, args, dev, args.force_valu)
                                for n in ("tiny", "mid") if n != args.workload]
        # the paper's own cost (NCC, block radius 1) on the 450x375 pair
        out["other_configs"].append(extra_config("mid", args, dev, False, cost_type=1))
        out["other_configs"].append(extra_config("mid", args, dev, True, cost_type=1))
    if not args.no_e2e:
        out["end_to_end"] = end_to_end(args, dev, wl, pair, p, stream)
    if not args.no_lr:
        out["left_right"] = left_right(args, dev, wl, pair)
    if not args.no_guided:
        out["guided"] = guided(args, dev)
        out["guided"]["headline_pair"] = guided_headline(args, dev, wl, pair)
    if not args.no_batched:
        out["batched"] = batched(args, dev)
    if not args.no_surrogate:
        out["surrogate"] = surrogate(args, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, pair, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
