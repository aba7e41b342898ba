#!/usr/bin/env python3
"""Benchmark of the removal-effect scoring path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step = one pass of the whole path over one view of the single-view
workload (500,000 clustered splats, one 1280x720 view): zero the scores,
project, bin, sort, blend, score. Inputs are resident in HBM before the timed
region. Prints one JSON line.

The roofline entry is for the kernel that takes the most time; its duration is
measured with HIP events on the stream the library launches on, around the one
library call that launches only that kernel. Algorithmic work per launch:
  k_score: 13 flops per visited (pixel, list entry) + 30 per blended one
  k_blend: 13 flops per visited + 12 per blended
  k_project: 288 bytes per splat-view (236 read, 52 written)
The CPU baseline is the FP64 oracle on the same view (project, tile lists,
compositing and removal scores), timed on the host.
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

METRIC = "splat-view removal scores/s (Gsplat·views/s) + fwd+bwd ms/view, % HBM peak"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
FLOPS_VISIT = {"score": 13.0, "blend": 13.0}
FLOPS_BLEND = {"score": 30.0, "blend": 12.0}
PROJECT_BYTES_PER_SPLAT_VIEW = 236 + 48 + 4


def cpu_baseline(scene, cams, s):
    import oracle
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    r = oracle.render(scene, cams[0], s, threads=threads, want=("image", "score_l1"))
    dt = time.perf_counter() - t0
    return {"value": scene.n * 1 / dt / 1e9, "unit": "Gsplat·views/s", "cores": threads, "kind": "oracle",
            "sample": (f"the full first view ({scene.n} splats, {cams[0].width}x{cams[0].height}): FP64 "
                       f"projection and tile lists (1 thread) + compositing and removal scores "
                       f"({threads} threads); {dt:.2f} s"),
            "seconds": dt, "pairs": int(len(r["bins"][1]))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); multi-GPU scoring shards by view "
              f"and is not built here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2601_14821_amd import raster, synth

    scene, cams = synth.workload_single_view()
    s = synth.RenderSettings()
    ds = raster.to_device(scene)
    rz = raster.Rasterizer(s)
    N, V = scene.n, len(cams)
    scores = torch.zeros(N, dtype=torch.float32, device="cuda")
    stages = ("project", "bin", "sort", "blend", "score")
    stage_ms = {k: 0.0 for k in stages}
    stream = torch.cuda.current_stream()

    def step(timed: bool):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] if timed else None
        if timed:
            ev[0].record(stream)
        scores.zero_()
        vb = rz.project(ds, cams)
        if timed:
            ev[1].record(stream)
        rz.bin(vb, cams)
        if timed:
            ev[2].record(stream)
        rz.sort(vb, cams)
        if timed:
            ev[3].record(stream)
        rz.blend(vb, cams)
        if timed:
            ev[4].record(stream)
        rz.score(vb, cams, scores=scores)
        if timed:
            ev[5].record(stream)
        return ev

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step(True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for ev in evs:
        for i, k in enumerate(stages):
            stage_ms[k] += ev[i].elapsed_time(ev[i + 1]) / args.steps
    ms = (t1 - t0) * 1000.0 / args.steps

    # work counts of the measured view (outside the timed region)
    vb = rz.project(ds, cams)
    rz.bin(vb, cams)
    rz.sort(vb, cams)
    rz.blend(vb, cams, count_blended=True)
    visited = int(vb.n_walk.sum().item())
    blended = int(vb.n_blend.sum().item())
    torch.cuda.synchronize()

    work = {
        "score": ("alu", (FLOPS_VISIT["score"] * visited + FLOPS_BLEND["score"] * blended) / 1e12),
        "blend": ("alu", (FLOPS_VISIT["blend"] * visited + FLOPS_BLEND["blend"] * blended) / 1e12),
        "project": ("hbm", PROJECT_BYTES_PER_SPLAT_VIEW * N * V / 1e9),
    }
    dom = max(("project", "blend", "score"), key=lambda k: stage_ms[k])
    bound, amount = work[dom]
    sec = stage_ms[dom] / 1000.0
    if bound == "hbm":
        achieved, peak, unit = amount / sec, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = amount / sec, FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": None, "kernel": f"k_{dom}",
                "kernel_ms": round(stage_ms[dom], 4)}

    out = {
        "metric": METRIC,
        "value": round(N * V / (ms / 1000.0) / 1e9, 4),
        "unit": "Gsplat·views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single-view removal scoring: 500k clustered splats, one 1280x720 view",
                   "splats": N, "views": V, "width": cams[0].width, "height": cams[0].height,
                   "tile": f"{s.tile_w}x{s.tile_h}", "lds_batch": s.lds_batch, "t_min": s.t_min,
                   "path": "plain per-view launches"},
        "roofline": roofline,
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "work": {"pairs": vb.n_pairs, "visited": visited, "blended": blended},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, cams, s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
