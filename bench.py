#!/usr/bin/env python
"""Benchmark of the editable-Gaussian rasterizer on one MI355X.

Headline: fwd+bwd iterations/s at 1M Gaussians.  One step is one pass of the
whole hot path over one view: compose the basic models under their edits,
project, bin + depth sort, composite, L1 loss against the view's target, and
the backward through the autograd Function (recompute, no per-pixel state).
The scene is 4 nested isosurface shells of 250k Gaussians (1M total), 800x800,
100 Fibonacci-sphere cameras at radius 4, one view per step; inputs are
resident in HBM before timing starts.

Also reported: forward Mpix/s on the composed 8 x 150k scene at 1024x1024
(60 orbit views), the roofline position of the dominant kernel (its average
duration from HIP events recorded around every launch in the timed region),
and the CPU oracle timed on a bounded sample of the same step.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import dataclasses
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s fwd and fwd+bwd iters/s at 1M Gaussians; culled vs plain speedup at ≤0.1 dB"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK = 78.6      # TFLOP/s without packed FP32 (256 CU x 64 FMA lanes x 2 x 2.4 GHz)
FP32_VALU_PEAK_PACKED = 157.3

# Algorithmic work per unit.
FWD_FLOP_EVAL, FWD_FLOP_COMP = 13, 10     # recount: per evaluated / extra per composited pair
BWD_FLOP_EVAL, BWD_FLOP_COMP = 13, 59
# the scope table's algorithmic work per evaluated pixel-Gaussian pair
# (recompute and chain counted as a whole; the exp is extra)
FWD_FLOP_PAIR_SCOPE, BWD_FLOP_PAIR_SCOPE = 25, 80
SORT_BYTES_PAIR = 4 + 4 + 4 + 4 + 4       # scatter write key+id, sort read key+id, write id
PROJECT_BYTES_G = 84 + 56                  # 21 planes read, record + rect written
DEPTH_SORT_BYTES_G = 12 + 8 + 3 * 24       # key read, (key, id) written, 3 digit passes of 8 B in + 8 B out (+ hist)
SCATTER_BYTES_G = 4 + 8 + 48               # order entry, rect, record per Gaussian; then 4 B per pair written
PROJECT_FLOP_G = 250                       # rotation, covariance, EWA, inverse, shading, bbox
PROJECT_BWD_FLOP_G = 500

# HBM bytes per launch measured with hardware counters (FETCH_SIZE and
# WRITE_SIZE, scaled by the same counters on a plain copy of known size),
# valid only for the kernel source they were measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
KERNEL_SOURCES = {
    "render_fwd": ["render.hip"], "render_bwd": ["render.hip"], "project": ["project.hip"],
    "project_bwd": ["project.hip"], "compose": ["project.hip"], "tile_count": ["binsort.hip"],
    "scatter": ["binsort.hip"], "depth_sort": ["binsort.hip"],
}


def source_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_17954_amd", "csrc")
    for f in KERNEL_SOURCES.get(kernel, []) + ["common.hpp", "launch.hpp"]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """Bytes per launch from the committed counter summary, or None when the
    kernel's source has changed since it was measured (or none exists)."""
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 3 and parts[0] == kernel and not line.startswith("#"):
                    fields = dict(p.split("=", 1) for p in parts[1:] if "=" in p)
                    if fields.get("source") == source_digest(kernel):
                        return int(float(fields["bytes_per_launch"]))
    except (OSError, ValueError, KeyError):
        pass
    return None


def settle():
    """Collect, then freeze the surviving objects out of the cyclic garbage
    collector: a full collection over the setup's objects (a few hundred
    thousand; tens of milliseconds) would otherwise land inside a timed loop
    as a host pause that has nothing to do with the GPU work."""
    gc.collect()
    gc.freeze()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--models", type=int, default=4)
    ap.add_argument("--width", type=int, default=800)
    ap.add_argument("--views", type=int, default=100)
    ap.add_argument("--fwd-px", type=int, default=0)
    ap.add_argument("--bwd-px", type=int, default=0)
    ap.add_argument("--sort-chunk", type=int, default=0,
                    help="records per binning chunk with --fwd-px/--bwd-px (0: the library's choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-culler", action="store_true")
    ap.add_argument("--no-explore", action="store_true")
    ap.add_argument("--no-vq", action="store_true")
    ap.add_argument("--no-sh", action="store_true")
    ap.add_argument("--no-editable", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB five times (counter calibration)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy kernel of known size: reading FETCH_SIZE / WRITE_SIZE for
    it gives the scale between those counters and bytes moved."""
    import torch
    n = 64 * 1024 * 1024  # float32 elements = 256 MiB
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": 4 * n, "dispatches": 5}), flush=True)


def h2_scene(n_total, k):
    from paper_2504_17954_amd import inputs as I
    levels = np.linspace(-0.12, 0.12, k)
    per = n_total // k
    models = [I.isosurface_model(per, I.SEED_SCENE + 2 + 100 * m, float(lv)) for m, lv in enumerate(levels)]
    edits = [I.identity_edit(m) for m in models]
    return models, edits


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}): the library has no multi-GPU "
              "path; how the path would shard is described with the design notes.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2504_17954_amd import inputs as I
    from paper_2504_17954_amd import losses as LS
    from paper_2504_17954_amd import native as N
    from paper_2504_17954_amd import raster as R

    N.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W = H = args.width

    # ---------------------------------------------------------------- setup
    t0 = time.time()
    models, edits = h2_scene(args.n, args.models)
    cams = I.cameras_at(I.fibonacci_sphere(args.views), W, H)
    log(f"scene: {sum(m.n for m in models)} Gaussians in {len(models)} models ({time.time() - t0:.1f}s)")
    mdev = [{k: torch.from_numpy(v).to(dev) for k, v in m.planes.items()} for m in models]
    n = sum(m.n for m in models)
    composed = {k: torch.empty((d, n), dtype=torch.float32, device=dev) for k, d in R.PLANE_DIMS.items()}
    mid = torch.empty(n, dtype=torch.int32, device=dev)
    edits_t = R.edit_table(edits, dev)
    cams_t = R.camera_table(cams, dev)
    jobs = [R.Jobs.single(n, camera=v) for v in range(args.views)]
    g = torch.Generator(device=dev)
    g.manual_seed(I.SEED_TARGET + 2)
    targets = torch.rand((args.views, 1, 4, H, W), generator=g, device=dev)
    settings = R.Settings(W, H, fwd_px=args.fwd_px, bwd_px=args.bwd_px, sort_chunk=args.sort_chunk)
    rnd = R.Renderer(settings, capacity=1 << 24, check="sync")

    # pair capacity from a pass over every view (sync mode grows it)
    R.compose_into(mdev, edits, composed, mid)
    max_pairs = 0
    for v in range(args.views):
        rnd.forward(composed, cams_t, jobs[v], model_id=mid, edits_t=edits_t)
        max_pairs = max(max_pairs, rnd.pairs())
    rnd.grow(int(max_pairs * 1.1) + 4096)
    rnd.check = "defer"
    for k in R.PLANES:
        composed[k].requires_grad_(True)
    tuned = {"fwd_px": args.fwd_px, "bwd_px": args.bwd_px, "sort_chunk": args.sort_chunk}
    if not (args.fwd_px or args.bwd_px):
        # launch shape (results do not depend on it): pixels per lane, records
        # per binning chunk, persistent render kernels; each candidate timed
        # on a few fwd+bwd steps of this workload
        from paper_2504_17954_amd import autotune as A
        base = rnd.settings

        def make(cfg):
            def run():
                rnd.settings = A.apply(base, cfg)
                for v in range(3):
                    rgba = R.rasterize(composed, cams_t, jobs[v], rnd, model_id=mid, edits_t=edits_t)
                    LS.l1(rgba, targets[v]).backward()
                for kk in R.PLANES:
                    composed[kk].grad = None
            return run
        best, times = A.tune(make, W, H, 1, n, reps=3, use_cache=False)
        rnd.settings = A.apply(base, best)
        tuned = {"choice": best, "ms_per_3_steps": {A.describe(c): round(times[i], 3)
                                                      for i, c in enumerate(A.CANDIDATES)}}
        log(f"fwd+bwd autotune (ms per 3 steps): {tuned['ms_per_3_steps']} -> {best}")

    def step(v):
        with torch.no_grad():
            R.compose_into(mdev, edits, composed, mid)
        rgba = R.rasterize(composed, cams_t, jobs[v], rnd, model_id=mid, edits_t=edits_t)
        loss = LS.l1(rgba, targets[v])
        loss.backward()
        for k in R.PLANES:
            composed[k].grad = None
        return loss

    settle()
    for i in range(args.warmup):
        step(i % args.views)
    torch.cuda.synchronize()

    # ------------------------------------------- per-kernel times (untimed)
    # Every launch bracketed by HIP events: the per-kernel averages and the
    # kernel with the largest total.  Two event records per launch slow the
    # step by ~10 %, so the timed region below brackets only that kernel.
    cal_steps = max(1, min(10, args.steps))
    N.ivrgs_timing_enable(True)
    for i in range(cal_steps):
        step((args.warmup + i) % args.views)
    kern = N.ivrgs_timing_read()
    N.ivrgs_timing_enable(False)
    dominant = max((k for k in KERNEL_SOURCES if kern[k][1] > 0), key=lambda k: kern[k][0])

    # ---------------------------------------------------------------- timed
    views = [(args.warmup + cal_steps + i) % args.views for i in range(args.steps)]
    N.ivrgs_timing_enable([dominant])
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for v in views:
        step(v)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    kern_timed = N.ivrgs_timing_read()
    N.ivrgs_timing_enable(False)
    rnd.verify()
    elapsed = t_end - t_start
    ms_step = elapsed / args.steps * 1e3
    value = args.steps / elapsed
    log(f"fwd+bwd: {ms_step:.3f} ms/step, {value:.1f} it/s")

    # --------------------------------------------- algorithmic counts per view
    # per view of the timed region (the rates below), and over every step of
    # the run, warm-up and per-kernel pass included (what a profiler's
    # per-dispatch averages over the whole run divide by)
    counts = {"pairs": [], "evaluated": [], "composited": []}
    cnt_settings = R.Settings(**{**rnd.settings.__dict__})
    cnt_settings.flags = N.FLAG_COUNT_EVAL
    cnt = R.Renderer(cnt_settings, capacity=rnd.capacity, check="sync")
    run_views = [i % args.views for i in range(args.warmup + cal_steps)] + views
    by_view = {}
    with torch.no_grad():
        for v in sorted(set(run_views)):
            cnt.forward({k: t.detach() for k, t in composed.items()}, cams_t, jobs[v], model_id=mid,
                        edits_t=edits_t)
            st = cnt.status.cpu().numpy()
            by_view[v] = (int(st[0]), int(st[2]), int(st[3]))
    for v in views:
        counts["pairs"].append(by_view[v][0])
        counts["evaluated"].append(by_view[v][1])
        counts["composited"].append(by_view[v][2])
    per_view = {k: float(np.mean(v)) for k, v in counts.items()}
    evaluated_run = float(np.mean([by_view[v][1] for v in run_views]))
    avg = {k: (ms / max(nl, 1), nl) for k, (ms, nl) in kern.items()}
    log("kernels (avg ms, launches; untimed pass): " + ", ".join(f"{k} {a:.4f}/{nl}" for k, (a, nl) in avg.items()
                                                                 if nl))
    dom_ms, dom_n = kern_timed[dominant]
    dom_avg_ms = dom_ms / max(dom_n, 1)
    log(f"{dominant} in the timed region: {dom_avg_ms:.4f} ms average over {dom_n} launches")

    work = {
        "render_bwd": ("alu", (BWD_FLOP_EVAL * per_view["evaluated"] + BWD_FLOP_COMP * per_view["composited"]) / 1e12,
                       "TFLOP/s", FP32_VALU_PEAK),
        "render_fwd": ("alu", (FWD_FLOP_EVAL * per_view["evaluated"] + FWD_FLOP_COMP * per_view["composited"]) / 1e12,
                       "TFLOP/s", FP32_VALU_PEAK),
        "depth_sort": ("hbm", DEPTH_SORT_BYTES_G * n / 1e9, "GB/s", HBM_PEAK_GBS),
        "tile_count": ("hbm", SCATTER_BYTES_G * n / 1e9, "GB/s", HBM_PEAK_GBS),
        "scatter": ("hbm", (SCATTER_BYTES_G * n + 4 * per_view["pairs"]) / 1e9, "GB/s", HBM_PEAK_GBS),
        "project": ("hbm", PROJECT_BYTES_G * n / 1e9, "GB/s", HBM_PEAK_GBS),
        "project_bwd": ("hbm", (84 + 36 + 84) * n / 1e9, "GB/s", HBM_PEAK_GBS),
        "compose": ("hbm", (84 + 88) * n / 1e9, "GB/s", HBM_PEAK_GBS),
    }
    scope_flops = {"render_bwd": BWD_FLOP_PAIR_SCOPE * per_view["evaluated"],
                   "render_fwd": FWD_FLOP_PAIR_SCOPE * per_view["evaluated"]}
    bound, amount, unit, peak = work[dominant]
    dur_s = dom_avg_ms / 1e3
    traffic = measured_traffic(dominant)
    if bound == "alu":
        # the scope table's flops per evaluated pair against the published
        # FP32 vector peak; the instruction-level recount and the unpacked
        # rate beside it
        achieved = scope_flops[dominant] / 1e12 / dur_s
        recount = amount / dur_s
        roofline = {"kernel": dominant, "bound": bound, "achieved": round(achieved, 3),
                    "peak": FP32_VALU_PEAK_PACKED, "unit": unit, "frac": round(achieved / FP32_VALU_PEAK_PACKED, 4),
                    "traffic": traffic, "avg_ms": round(dom_avg_ms, 4), "launches": dom_n,
                    "flop_per_evaluated_pair": BWD_FLOP_PAIR_SCOPE if dominant == "render_bwd" else FWD_FLOP_PAIR_SCOPE,
                    "frac_vs_unpacked_peak": round(achieved / FP32_VALU_PEAK, 4),
                    "recount": {"achieved": round(recount, 3), "frac": round(recount / FP32_VALU_PEAK_PACKED, 4),
                                "flop": "13 per evaluated pair + " + ("59" if dominant == "render_bwd" else "10")
                                        + " per composited pair"}}
    else:
        achieved = amount / dur_s
        roofline = {"kernel": dominant, "bound": bound, "achieved": round(achieved, 3), "peak": peak,
                    "unit": unit, "frac": round(achieved / peak, 4), "traffic": traffic,
                    "avg_ms": round(dom_avg_ms, 4), "launches": dom_n}
    if traffic is not None:
        roofline["traffic_unit"] = "bytes per launch"
        roofline["traffic_gbs"] = round(traffic / dur_s / 1e9, 1)

    # whole-step roofline: each stage at the larger of its HBM time and its
    # FP32 VALU time for its algorithmic work, summed, over the measured step
    stage_flops = {  # per launch
        "project": PROJECT_FLOP_G * n, "project_bwd": PROJECT_BWD_FLOP_G * n,
        "render_fwd": (FWD_FLOP_EVAL * per_view["evaluated"] + FWD_FLOP_COMP * per_view["composited"]),
        "render_bwd": (BWD_FLOP_EVAL * per_view["evaluated"] + BWD_FLOP_COMP * per_view["composited"]),
    }
    ideal_s = 0.0
    for kname, (_, nl) in kern.items():
        if not nl or kname not in work and kname not in stage_flops:
            continue
        launches_per_step = nl / cal_steps
        t_hbm = work[kname][1] / HBM_PEAK_GBS if kname in work and work[kname][0] == "hbm" else 0.0
        t_alu = stage_flops.get(kname, 0.0) / (FP32_VALU_PEAK * 1e12)
        ideal_s += launches_per_step * max(t_hbm, t_alu)
    step_roofline = {"ideal_ms": round(ideal_s * 1e3, 4), "measured_ms": round(ms_step, 4),
                     "frac": round(ideal_s * 1e3 / ms_step, 4),
                     "definition": "sum over stages of max(algorithmic bytes / 8 TB/s, algorithmic flop / "
                                   "78.6 TFLOP/s) per step, over the measured step time"}

    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"isosurface-{len(models)}shells-{n}-{W}px-fwd+bwd",
                   "gaussians": n, "models": len(models), "width": W, "height": H,
                   "views": args.views, "views_per_step": 1,
                   "pairs_per_view": round(per_view["pairs"]),
                   "evaluated_per_view": round(per_view["evaluated"]),
                   "evaluated_per_step_of_run": round(evaluated_run),
                   "composited_per_view": round(per_view["composited"]),
                   "launch_shape": tuned},
        "roofline": roofline,
        "step_roofline": step_roofline,
        "kernels_avg_ms": {k: round(a, 4) for k, (a, nl) in avg.items() if nl},
        "kernels_timing": f"kernels_avg_ms from {cal_steps} untimed steps with every launch bracketed by HIP "
                          f"events; the timed region brackets only {dominant}",
    }

    if not args.no_secondary:
        result["secondary"] = {"composed_forward": secondary_fwd(dev)}
        if not args.no_batched:
            result["secondary"]["batched"] = secondary_batched(dev)
        if not args.no_culler:
            result["secondary"]["culler"] = secondary_culler(dev)
        if not args.no_explore:
            result["secondary"]["inverse_exploration"] = secondary_explore(dev)
        if not args.no_vq:
            result["secondary"]["vq"] = secondary_vq(dev)
        if not args.no_sh:
            result["secondary"]["base_3dgs_sh"] = secondary_sh(dev)
        if not args.no_editable:
            result["secondary"]["editable_training"] = secondary_editable(dev)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(models, edits, cams, W, H, views[0], args.cpu_seconds)

    print(json.dumps(result), flush=True)


def secondary_fwd(dev):
    """Forward Mpix/s on the composed scene: 8 nested shells x 150k Gaussians
    with recolour / opacity / light edits, 1024x1024, 60 orbit views
    (project + bin_sort + render_fwd per view; compose once per edit)."""
    import torch
    from paper_2504_17954_amd import inputs as I
    from paper_2504_17954_amd import raster as R
    t0 = time.time()
    w = I.c3()
    log(f"composed scene generated ({time.time() - t0:.1f}s)")
    mdev = [{k: torch.from_numpy(v).to(dev) for k, v in m.planes.items()} for m in w.models]
    planes, mid = R.compose(mdev, w.edits, dev)
    edits_t = R.edit_table(w.edits, dev)
    cams_t = R.camera_table(w.cameras, dev)
    n = mid.numel()
    jobs = [R.Jobs.single(n, camera=v) for v in range(len(w.cameras))]
    rnd = R.Renderer(R.Settings(w.width, w.height), capacity=1 << 25, check="sync")
    out = torch.empty((1, 4, w.height, w.width), dtype=torch.float32, device=dev)
    mx = 0
    for v in range(len(w.cameras)):
        rnd.forward(planes, cams_t, jobs[v], model_id=mid, edits_t=edits_t, out=out, fwd_only=True)
        mx = max(mx, rnd.pairs())
    rnd.grow(int(mx * 1.1) + 4096)
    rnd.check = "defer"
    # launch shape (results do not depend on it): pixels per lane and
    # records per binning chunk, timed on the first views
    from paper_2504_17954_amd import autotune as A
    base = rnd.settings
    cands = [c for c in A.CANDIDATES if not c["persistent"] and c["bwd_px"] == 1]

    def make(cfg):
        def run():
            rnd.settings = A.apply(base, cfg)
            for v in range(4):
                rnd.forward(planes, cams_t, jobs[v], model_id=mid, edits_t=edits_t, out=out, fwd_only=True)
        return run
    best, times = A.tune(make, w.width, w.height, 1, n, candidates=cands, reps=3, use_cache=False)
    rnd.settings = A.apply(base, best)
    log(f"composed forward autotune (ms per candidate): {times} -> {best}")
    settle()
    for v in range(5):
        rnd.forward(planes, cams_t, jobs[v], model_id=mid, edits_t=edits_t, out=out, fwd_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v in range(len(w.cameras)):
        rnd.forward(planes, cams_t, jobs[v], model_id=mid, edits_t=edits_t, out=out, fwd_only=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rnd.verify()
    nv = len(w.cameras)
    mpix = nv * w.width * w.height / dt / 1e6
    log(f"composed forward: {dt / nv * 1e3:.3f} ms/view, {mpix:.1f} Mpix/s")
    return {"fwd_mpix_s": round(mpix, 2), "fwd_ms_per_view": round(dt / nv * 1e3, 4),
            "workload": f"compose-{len(w.models)}x{w.models[0].n}-{w.width}px-{nv}views-fwd",
            "launch_shape": {k: best[k] for k in ("fwd_px", "sort_chunk")}}


VQ_BYTES = 3 * 4 + 3 * 4 + 15       # stored per quantised Gaussian: exact mean and normal, 15 one-byte indices
OUT_BYTES = 21 * 4 + 4              # written per composed Gaussian: 21 FP32 attributes and the model id
FLOAT_BYTES = 21 * 4                # read per Gaussian by the float compose


def secondary_vq(dev, k=256, iters=10, reps=20):
    """Vector quantisation (Sec. 4.4) of the four 250k-Gaussian shells of the
    main workload (eight codebooks per model, k = 256, 10 Lloyd iterations),
    then compose of the quantised models with the decode fused, against the
    float compose; the forward render of one view from both composed sets
    gives the PSNR cost of quantisation."""
    import torch
    from paper_2504_17954_amd import inputs as I
    from paper_2504_17954_amd import native as N
    from paper_2504_17954_amd import raster as R
    from paper_2504_17954_amd import vq as V
    models, edits = h2_scene(1_000_000, 4)
    mdev = [{kk: torch.from_numpy(v).to(dev) for kk, v in m.planes.items()} for m in models]
    n = sum(m.n for m in models)
    for m in mdev[:1]:
        V.quantize(m, k, iters)  # warm-up
    torch.cuda.synchronize()
    settle()
    t0 = time.perf_counter()
    qs = [V.quantize(m, k, iters) for m in mdev]
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    for _ in range(3):
        V.compose(qs, edits, dev)
        R.compose(mdev, edits, dev)
    torch.cuda.synchronize()
    N.ivrgs_timing_enable(["vq", "compose"])
    for _ in range(reps):
        planes_q, mid_q = V.compose(qs, edits, dev)
        planes_f, mid_f = R.compose(mdev, edits, dev)
    t = N.ivrgs_timing_read()
    N.ivrgs_timing_enable(0)
    ms_q = t["vq"][0] / max(t["vq"][1], 1)
    ms_f = t["compose"][0] / max(t["compose"][1], 1)
    gbs_q = n * (VQ_BYTES + OUT_BYTES) / (ms_q * 1e-3) / 1e9
    gbs_f = n * (FLOAT_BYTES + OUT_BYTES) / (ms_f * 1e-3) / 1e9
    cams = I.cameras_at(I.fibonacci_sphere(100), 800, 800)
    cams_t = R.camera_table(cams, dev)
    edits_t = R.edit_table(edits, dev)
    rnd = R.Renderer(R.Settings(800, 800), capacity=1 << 24, check="sync")
    job = R.Jobs.single(n, camera=3)
    a = rnd.forward(planes_f, cams_t, job, model_id=mid_f, edits_t=edits_t, fwd_only=True).clone()
    b = rnd.forward(planes_q, cams_t, job, model_id=mid_q, edits_t=edits_t, fwd_only=True)
    mse = float(((a[:, :3] - b[:, :3]) ** 2).mean())
    psnr = 10 * np.log10(1.0 / max(mse, 1e-20))
    stored_q = sum(q.nbytes() for q in qs)
    stored_f = n * FLOAT_BYTES
    log(f"vq: quantise 4x250k in {t_fit * 1e3:.1f} ms; compose quantised {ms_q:.4f} ms ({gbs_q:.0f} GB/s) "
        f"vs float {ms_f:.4f} ms ({gbs_f:.0f} GB/s); {stored_f / stored_q:.2f}x smaller; PSNR {psnr:.1f} dB")
    return {"quantize_ms": round(t_fit * 1e3, 3), "compose_vq_ms": round(ms_q, 4), "compose_float_ms": round(ms_f, 4),
            "compose_vq_roofline": {"bound": "hbm", "achieved": round(gbs_q, 1), "peak": 8000.0, "unit": "GB/s",
                                    "frac": round(gbs_q / 8000.0, 4),
                                    "bytes_per_gaussian": VQ_BYTES + OUT_BYTES},
            "compose_float_gbs": round(gbs_f, 1), "compression": round(stored_f / stored_q, 3),
            "psnr_quantised_vs_float_db": round(psnr, 2),
            "workload": f"vq-4x250k-k{k}-iters{iters}-compose-800px-view3"}


SH_FWD_BYTES = 48 * 4 + 12 + 12            # per Gaussian: coefficients and mean read, colour written
SH_BWD_BYTES = 48 * 4 + 12 + 12 + 48 * 4 + 24  # + dL/dcolour read, dL/dsh written, dL/dmean read and written


def secondary_sh(dev, steps=20, warmup=3):
    """Base 3DGS (Sec. 4.2), degree-3 SH colour on the 1M Gaussians of the
    main workload: the SH colour and backward kernels on their own, and a
    training step (SH colour -> rasterize -> L1 -> backward through both) at
    800x800, one view per step cycling the 100 cameras."""
    import torch
    from paper_2504_17954_amd import inputs as I
    from paper_2504_17954_amd import losses as LS
    from paper_2504_17954_amd import native as N
    from paper_2504_17954_amd import raster as R
    from paper_2504_17954_amd import sh as SH
    models, edits = h2_scene(1_000_000, 4)
    mdev = [{kk: torch.from_numpy(v).to(dev) for kk, v in m.planes.items()} for m in models]
    planes, _ = R.compose(mdev, edits, dev)
    n = planes["mean"].shape[1]
    planes["shade"] = SH.base_shade(n, dev)
    g = torch.Generator(device=dev)
    g.manual_seed(I.SEED_SCENE + 91)
    sh = (torch.randn((48, n), generator=g, device=dev) * 0.15).contiguous()
    sh[0:3] = (torch.rand((3, n), generator=g, device=dev) - 0.5) / 0.28209479177387814
    cams = I.cameras_at(I.fibonacci_sphere(100), 800, 800)
    cams_t = R.camera_table(cams, dev)
    gcol = torch.rand((3, n), generator=g, device=dev) - 0.5
    gm = torch.zeros((3, n), device=dev)
    for _ in range(3):
        SH.color(sh, planes["mean"], cams[0], 3)
        SH.color_bwd(sh, planes["mean"], cams[0], 3, gcol, gm)
    N.ivrgs_timing_enable(["sh"])
    for v in range(10):
        SH.color(sh, planes["mean"], cams[v], 3)
    t_f = N.ivrgs_timing_read()["sh"]
    N.ivrgs_timing_enable(["sh"])
    for v in range(10):
        SH.color_bwd(sh, planes["mean"], cams[v], 3, gcol, gm)
    t_b = N.ivrgs_timing_read()["sh"]
    N.ivrgs_timing_enable(0)
    ms_f, ms_b = t_f[0] / t_f[1], t_b[0] / t_b[1]
    gbs_f = n * SH_FWD_BYTES / (ms_f * 1e-3) / 1e9
    gbs_b = n * SH_BWD_BYTES / (ms_b * 1e-3) / 1e9
    rnd = R.Renderer(R.Settings(800, 800), capacity=1 << 24, check="sync")
    jobs = R.Jobs.single(n)
    mean = planes["mean"].clone().requires_grad_(True)
    shp = sh.clone().requires_grad_(True)
    tg = torch.Generator(device=dev)
    tg.manual_seed(I.SEED_TARGET + 91)
    targets = [torch.rand((4, 800, 800), generator=tg, device=dev) for _ in range(4)]

    def step(v):
        pl = dict(planes, mean=mean, color=SH.SHColor.apply(shp, mean, cams[v % 100], 3))
        out = R.rasterize(pl, cams_t[v % 100:v % 100 + 1], jobs, rnd)[0]
        loss = LS.l1(out, targets[v % 4])
        mean.grad = shp.grad = None
        loss.backward()

    settle()
    for v in range(warmup):
        step(v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v in range(steps):
        step(v)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    log(f"base 3DGS SH: colour {ms_f:.4f} ms ({gbs_f:.0f} GB/s), backward {ms_b:.4f} ms ({gbs_b:.0f} GB/s); "
        f"training step {dt * 1e3:.3f} ms ({1 / dt:.1f} it/s)")
    return {"sh_color_ms": round(ms_f, 4), "sh_color_bwd_ms": round(ms_b, 4),
            "sh_color_roofline": {"bound": "hbm", "achieved": round(gbs_f, 1), "peak": 8000.0, "unit": "GB/s",
                                  "frac": round(gbs_f / 8000.0, 4), "bytes_per_gaussian": SH_FWD_BYTES},
            "sh_color_bwd_roofline": {"bound": "hbm", "achieved": round(gbs_b, 1), "peak": 8000.0, "unit": "GB/s",
                                      "frac": round(gbs_b / 8000.0, 4), "bytes_per_gaussian": SH_BWD_BYTES},
            "train_step_ms": round(dt * 1e3, 4), "train_iters_per_s": round(1 / dt, 2),
            "workload": "base3dgs-sh3-1000000-800px-fwd+bwd"}


def secondary_editable(dev, steps=20, warmup=3):
    """Editable-Gaussian training step of one basic model (Sec. 4.3): 300k
    Gaussians, 800x800, one view per step: the image and the eleven
    auxiliary maps (depth, unit normal, delta-c, k_a, k_d, k_s, beta), the
    full loss (L1 + SSIM, normal consistency, opacity L1, sparsity,
    bilateral smoothness) and the backward through both renders."""
    import torch
    from paper_2504_17954_amd import aux as AX
    from paper_2504_17954_amd import inputs as I
    from paper_2504_17954_amd import losses as LS
    from paper_2504_17954_amd import native as N
    from paper_2504_17954_amd import raster as R
    m = I.isosurface_model(300_000, I.SEED_SCENE + 2, 0.0)
    planes = {k: torch.from_numpy(v).to(dev).requires_grad_(True) for k, v in I.plain_planes(m).items()}
    n = m.n
    cams = I.cameras_at(I.fibonacci_sphere(100), 800, 800)
    cams_t = R.camera_table(cams, dev)
    tg = torch.Generator(device=dev)
    tg.manual_seed(I.SEED_TARGET + 93)
    targets = [torch.rand((4, 800, 800), generator=tg, device=dev) for _ in range(4)]
    rnd = R.Renderer(R.Settings(800, 800), capacity=1 << 24, check="sync")
    jobs = R.Jobs.single(n)
    edits = R.default_edits(dev)

    def step(v):
        rgba, maps = AX.render_editable(planes, cams_t[v % 100:v % 100 + 1], jobs, rnd, edits_t=edits)
        loss = LS.editable_loss(rgba.squeeze(0), targets[v % 4], maps.squeeze(0), planes["opacity"], cams[v % 100])
        for t in planes.values():
            t.grad = None
        loss.backward()
        return loss

    settle()
    for v in range(warmup):
        step(v)
    rnd.check = "defer"  # the warm-up sized the pair capacity; verified after the timed steps
    torch.cuda.synchronize()
    N.ivrgs_timing_enable(["aux"])
    t0 = time.perf_counter()
    for v in range(steps):
        loss = step(v)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    t_aux = N.ivrgs_timing_read()["aux"]
    N.ivrgs_timing_enable(0)
    rnd.verify()
    log(f"editable training step (300k, 800x800, image + 11 maps + full loss): {dt * 1e3:.3f} ms "
        f"({1 / dt:.1f} it/s); aux kernels {t_aux[0] / steps:.3f} ms per step; loss {float(loss):.4f}")
    return {"train_step_ms": round(dt * 1e3, 4), "train_iters_per_s": round(1 / dt, 2),
            "aux_kernels_ms_per_step": round(t_aux[0] / steps, 4),
            "workload": "editable-300000-800px-image+11maps-fullloss-fwd+bwd"}


EXPLORE_N = 1_484_642  # composed primitives of the paper's largest-timed exploration example


def secondary_explore(dev, iters=100, warmup=5):
    """Inverse volume exploration iterations/s: 5 nested shells composed to
    1,484,642 Gaussians, 800x800, orbital light.  The target is the render
    under reference parameters; the loop starts from perturbed parameters
    and learns palettes, opacity scales, lambda, b and the light angles on
    the paper's L1 + SSIM objective (compose, project, bin_sort, render_fwd,
    SSIM and the photometric gradient, render_bwd, compose_bwd, light_bwd,
    Adam step per iteration, all on the device; the pair count is checked
    once, after the timed iterations)."""
    import torch
    from paper_2504_17954_amd import explore as E
    from paper_2504_17954_amd import inputs as I
    from paper_2504_17954_amd import raster as R
    K, W = 5, 800
    sizes = [EXPLORE_N // K + (1 if m < EXPLORE_N % K else 0) for m in range(K)]
    t0 = time.time()
    levels = np.linspace(-0.2, 0.1, K)
    models = [I.isosurface_model(n, I.SEED_SCENE + 7 + 100 * m, float(lv)) for m, (n, lv) in
              enumerate(zip(sizes, levels))]
    log(f"exploration scene generated ({time.time() - t0:.1f}s)")
    mdev = [{k: torch.from_numpy(v).to(dev) for k, v in m.planes.items()} for m in models]
    rng = np.random.default_rng(I.SEED_SCENE + 77)
    base = np.zeros((K, 16), np.float32)  # orbital light for every model
    truth = E.initial_theta(rng.uniform(0.1, 0.8, (K, 3)), rng.uniform(0.5, 1.5, K), (1.2, 0.9, 1.1, 1.0),
                            (0.05, -0.05, 0.02, 0.0), 1.1, 0.6)
    start = truth.copy()
    start[:3 * K] = np.clip(start[:3 * K] + rng.uniform(-0.2, 0.2, 3 * K), 0, 1)
    start[3 * K:4 * K] = 1.0
    start[4 * K:4 * K + 8] = (1, 1, 1, 1, 0, 0, 0, 0)
    start[4 * K + 8:] = (0.8, 0.2)
    cam = I.cameras_at(I.fibonacci_sphere(100), W, W)[17]
    ref = E.Explorer(mdev, base, truth, cam, torch.zeros((4, W, W), device=dev), R.Settings(W, W), lr=0.0)
    ref.step()
    target = ref.rgba.clone()
    del ref
    ex = E.Explorer(mdev, base, start, cam, target, R.Settings(W, W), lr=0.01)
    settle()
    for _ in range(warmup):
        ex.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ex.run(iters, verify=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ex.verify()  # no binning of the timed iterations overflowed
    ex2 = E.Explorer(mdev, base, start, cam, target, R.Settings(W, W), lr=0.01)
    ex2.step()
    loss0 = ex2.loss()
    ex.step()
    loss1 = ex.loss()
    it_s = iters / dt
    log(f"inverse exploration: {dt / iters * 1e3:.3f} ms/iteration, {it_s:.1f} it/s; "
        f"loss (0.8 L1 + 0.2 (1 - SSIM)) {loss0:.5f} -> {loss1:.5f} after {ex.iterations} iterations")
    return {"iters_per_s": round(it_s, 2), "ms_per_iteration": round(dt / iters * 1e3, 4),
            "objective": "0.8 L1 + 0.2 (1 - SSIM), RGBA",
            "loss_start": round(loss0, 6), f"loss_after_{ex.iterations}": round(loss1, 6),
            "workload": f"explore-{K}models-{EXPLORE_N}-{W}px-orbital-lr0.01-l1ssim",
            "paper_context": "48 s / 1000 iterations (20.8 it/s) at 1,484,642 primitives with L1+SSIM on the "
                             "paper's GPU (RTX 4090; image size not stated)"}


def secondary_batched(dev):
    """Batched training step: 4 basic models of 50k / 120k / 250k / 500k
    Gaussians (nested shells) x 32 Fibonacci views at 800x800 = 128 jobs in
    one launch sequence with persistent render kernels; launch shape chosen by
    the autotuner; eager steps and replays of the captured graph."""
    import torch
    from paper_2504_17954_amd import autotune as A
    from paper_2504_17954_amd import batch as B
    from paper_2504_17954_amd import inputs as I
    from paper_2504_17954_amd import raster as R
    t0 = time.time()
    w = I.c4()
    log(f"batched scene generated ({time.time() - t0:.1f}s)")
    sizes = [m.n for m in w.models]
    planes = {k: torch.from_numpy(np.concatenate([I.plain_planes(m)[k] for m in w.models], 1)).to(dev)
              for k in R.PLANES}
    cams_t = R.camera_table(w.cameras, dev)
    jobs = R.Jobs.models_by_views(sizes, len(w.cameras))
    g = torch.Generator(device=dev)
    g.manual_seed(I.SEED_TARGET + 4)
    targets = torch.rand((jobs.n_jobs, 4, w.height, w.width), generator=g, device=dev)
    step = B.BatchStep(planes, cams_t, jobs, targets, B.batch_settings(w.width, w.height))
    base = step.renderer.settings

    def make(cfg):
        def run():
            step.renderer.settings = A.apply(base, cfg)
            step.step()
        return run
    best, times = A.tune(make, w.width, w.height, jobs.n_jobs, jobs.n_records, reps=3, use_cache=False)
    step.renderer.settings = A.apply(base, best)
    log(f"autotune (ms per candidate): {times} -> {best}")
    settle()
    for _ in range(2):
        step.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        step.step()
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / reps
    step.capture()
    step.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step.replay()
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) / reps
    pairs = step.verify()
    log(f"batched: eager {eager * 1e3:.2f} ms/step, graph {graph * 1e3:.2f} ms/step, {pairs} pairs")
    return {"workload": f"batched-{len(sizes)}models-{len(w.cameras)}views-{w.width}px-fwd+bwd",
            "jobs": jobs.n_jobs, "records": jobs.n_records, "pairs": int(pairs),
            "steps_s_eager": round(1.0 / eager, 3), "steps_s_graph": round(1.0 / graph, 3),
            "images_s_graph": round(jobs.n_jobs / graph, 1), "launch_shape": best}


def secondary_culler(dev):
    """Learned culling on the 300k isosurface scene: labels from 200 random
    training views (the rasterizer's max T*alpha >= 1/255), MLP training,
    threshold calibrated for 99.9 % recall on training views, then 60
    held-out views at 1024x1024: plain vs culled forward time and the PSNR of
    culled against plain (the loss against ground truth it implies for a model
    at the paper's best basic-scene PSNR, 36.44 dB)."""
    import torch
    from paper_2504_17954_amd import cull as CU
    from paper_2504_17954_amd import inputs as I
    from paper_2504_17954_amd import raster as R
    t0 = time.time()
    m = I.isosurface_model(300_000, I.SEED_SCENE + 2)
    planes = {k: torch.from_numpy(v).to(dev) for k, v in I.plain_planes(m).items()}
    train_c, test_c = I.c5_views()
    W = H = train_c[0].width
    tr_t, te_t = R.camera_table(train_c, dev), R.camera_table(test_c, dev)
    n = m.n
    labels = CU.collect_labels(planes, tr_t, W, H)
    model, mean, std = CU.train(planes, tr_t, labels, steps=1500)
    wts = CU.pack(model, mean, std)
    culler = CU.Culler(wts, n)
    recall = 0.999
    wts.threshold = CU.calibrate_threshold(culler, planes, tr_t, labels, recall=recall, views=range(0, 200, 5))
    log(f"culler trained ({time.time() - t0:.1f}s), visible fraction {labels.float().mean().item():.3f}, "
        f"threshold {wts.threshold:.3f}")
    plain = R.Renderer(R.Settings(W, H), capacity=1 << 24, check="sync")
    culled = R.Renderer(R.Settings(W, H), capacity=1 << 24, check="sync")
    edits = R.default_edits(dev)
    views = list(range(len(test_c)))
    jobs_p = [R.Jobs.single(n, camera=v) for v in views]
    jobs_c = [R.Jobs.single(n, camera=v) for v in views]
    ref = [plain.forward(planes, te_t, jobs_p[v], edits_t=edits, fwd_only=True).clone() for v in views]
    got = [culler.render(culled, planes, te_t, jobs_c[v], v).clone() for v in views]
    q = [min(CU.psnr(a[0], b[0]), 120.0) for a, b in zip(got, ref)]  # identical images: capped
    kept = float(np.mean([int(j.device[0, 2].item()) for j in jobs_c])) / n
    plain.check = culled.check = "defer"
    out = torch.empty((1, 4, H, W), dtype=torch.float32, device=dev)

    def timed(fn):
        """Eager wall time per view (includes the host's launch overhead)."""
        for v in views[:3]:
            fn(v)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for v in views:
            fn(v)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / len(views)

    def graphed(fn):
        """GPU time per view: each view's launches captured once as a HIP
        graph, all views replayed back to back between two events."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for v in views[:3]:
                fn(v)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graphs = []
        for v in views:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                fn(v)
            graphs.append(g)
        for g in graphs[:3]:
            g.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for g in graphs:
            g.replay()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / len(views)

    render_plain = lambda v: plain.forward(planes, te_t, jobs_p[v], edits_t=edits, out=out, fwd_only=True)
    render_cull = lambda v: culler.render(culled, planes, te_t, jobs_c[v], v, out=out)
    # records per binning chunk (a launch shape; results do not depend on
    # it), chosen for each pipeline on its own eager renders
    chunks = {}
    for name, rnd_, fn in (("plain", plain, render_plain), ("culled", culled, render_cull)):
        base = rnd_.settings
        best = None
        for c in (0, 64, 128, 256):
            rnd_.settings = dataclasses.replace(base, sort_chunk=c)
            t = timed(fn)
            if best is None or t < best[1]:
                best = (c, t)
        rnd_.settings = dataclasses.replace(base, sort_chunk=best[0])
        chunks[name] = best[0]
    e_plain, e_cull = timed(render_plain), timed(render_cull)
    t_plain, t_cull = graphed(render_plain), graphed(render_cull)
    plain.verify()
    culled.verify()
    # the graphs rendered the same views: the last one must still match its eager image
    last = views[-1]
    assert torch.equal(out, got[last]), "graph replay differs from the eager culled render"
    qmin = float(np.min(q))
    log(f"culler: records per binning chunk {chunks}")
    log(f"culler: plain {t_plain * 1e3:.3f} ms, culled {t_cull * 1e3:.3f} ms per view (graphs); eager "
        f"{e_plain * 1e3:.3f} / {e_cull * 1e3:.3f} ms; kept {kept:.3f}, PSNR mean {np.mean(q):.2f} min {qmin:.2f}")
    return {"workload": f"cull-isosurface-{n}-{W}px-60views-fwd", "speedup": round(t_plain / t_cull, 3),
            "plain_ms": round(t_plain * 1e3, 4), "culled_ms": round(t_cull * 1e3, 4),
            "timing": "per-view HIP graphs replayed back to back", "sort_chunk": chunks,
            "eager_plain_ms": round(e_plain * 1e3, 4), "eager_culled_ms": round(e_cull * 1e3, 4),
            "kept_fraction": round(kept, 4), "visible_fraction_train": round(labels.float().mean().item(), 4),
            "psnr_mean_db": round(float(np.mean(q)), 2), "psnr_min_db": round(qmin, 2),
            "loss_db_at_36.44": round(CU.loss_from_psnr(qmin), 4), "recall_target": recall}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(models, edits, cams, W, H, view, seconds):
    """The CPU oracle on a bounded sample of one step: compose, then forward
    and backward of the L1 loss restricted to a random pixel sample; the
    per-pixel cost is scaled to the full image, the per-step fixed cost
    (projection and sort of every Gaussian) is counted once per pass."""
    import oracle as O
    O.build()
    rows = np.stack([e.row() for e in edits])
    t0 = time.perf_counter()
    planes, mid = O.compose([m.planes for m in models], rows)
    t_compose = time.perf_counter() - t0
    cam = cams[view]
    prm = O.Params(W, H)
    rng = np.random.default_rng(0)

    def run(npx):
        pix = np.stack([rng.integers(0, W, npx), rng.integers(0, H, npx)], 1)
        t = time.perf_counter()
        ref = O.render(planes, cam, prm, model_id=mid, edits=rows, pix=pix)
        tgt = rng.uniform(0, 1, ref["rgba"].shape)
        dl = np.sign(ref["rgba"] - tgt) / (4.0 * W * H)
        O.backward(planes, cam, prm, dl, model_id=mid, edits=rows, pix=pix)
        return time.perf_counter() - t

    t_fixed = run(1)
    t_small = run(512)
    per_px = max((t_small - t_fixed) / 511, 1e-7)
    npx = int(np.clip((seconds - t_fixed) / per_px, 64, W * H))
    t_sample = run(npx)
    per_px = max((t_sample - t_fixed) / max(npx - 1, 1), 1e-9)
    t_step = t_compose + t_fixed + per_px * W * H
    log(f"cpu oracle: fixed {t_fixed:.2f}s, {npx} px in {t_sample:.2f}s -> {t_step:.1f}s per step")
    return {"value": round(1.0 / t_step, 6), "unit": "iters/s", "cores": O.num_threads(),
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"one step of the same workload (view {view}): compose, then forward+backward "
                      f"of {npx} random pixels of {W}x{H}; per-pixel time scaled to the full image, "
                      f"projection/sort counted once ({t_sample:.1f}s measured)"}


if __name__ == "__main__":
    main()
