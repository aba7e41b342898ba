#!/usr/bin/env python3
"""Benchmark of the removal-effect scoring path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--main-only]

Main line (the `value`): one step = one pass of the whole path over the
single-view workload (500,000 clustered splats, one 1280x720 view): zero the
scores, project, bin, sort, and the fused composite + removal pass, as plain
per-view launches. Inputs are resident in HBM before the timed region.

Also reported (extra fields):
  batched: 3M clustered splats x 16 of the 200 hemisphere views at 1600x1064,
           plain per-view launches vs one HIP-graph replay of the batched
           persistent scorer (ms per view, Gsplat.views/s);
  multi_scene: 16 clustered scenes of uneven size (50k..2M splats, 8..32
           views each, 640x480 / 1280x720 / 1600x1064): tile shape and LDS
           batch picked by the autotuner on the whole batch, then one HIP-graph
           replay of the batched persistent scorer;
  fwd_bwd: 1M splats x 4 views at 1280x720, forward + L1 loss gradient +
           hand-written backward, ms per view.

Roofline: the kernel that takes the most time in the main line, timed with HIP
events on the library's stream around the one call that launches only it.
Algorithmic work per launch:
  k_render_score: 26 flops per visited (pixel, list entry) + 42 per blended one
                  (blend sweep 13 + 12, removal sweep 13 + 30)
  k_project:      288 bytes per splat-view (236 read, 48 + 4 written)
`traffic` (HBM bytes) and `valu_issue` (VALU instructions over the chip's issue
limit of one wave64 instruction per CU per cycle, for the live kernel time) come
from the committed counter record, null once the kernel's sources differ.
The CPU baseline is the FP64 oracle on the same view, timed on the host.
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
VALU_ISSUE_PER_S = 256 * 2.4e9   # wave64 VALU instructions per second, one per CU per cycle
FUSED_FLOPS_VISIT, FUSED_FLOPS_BLEND = 26.0, 42.0
PROJECT_BYTES_PER_SPLAT_VIEW = 236 + 48 + 4


def measured_counters(kernel: str):
    """The committed counter record of `kernel` (HBM bytes and VALU instructions
    per launch), or None when there is none or the kernel's sources changed since
    it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "render_score_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for p in rec["sources"]:
        try:
            h.update(open(os.path.join(ROOT, p), "rb").read())
        except OSError:
            return None
    return rec if h.hexdigest() == rec["sources_sha256"] else None


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter record, or None."""
    rec = measured_counters(kernel)
    return None if rec is None else int(rec["bytes_per_launch"])


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
            "seconds": round(dt, 3), "pairs": int(len(r["bins"][1]))}


def main_line(args, torch, raster, synth):
    scene, cams = synth.workload_single_view()
    s = synth.RenderSettings()
    ds = raster.to_device(scene)
    rz = raster.Rasterizer(s)
    N, V = scene.n, len(cams)
    scores = torch.zeros(N, dtype=torch.float32, device="cuda")
    stages = ("project", "bin", "sort", "render_score")
    stage_ms = {k: 0.0 for k in stages}
    stream = torch.cuda.current_stream()
    # the pair count of this view, from an untimed pass; the timed steps sort into
    # that many slots without reading the count back (no host synchronisation
    # inside a step), and the last step's count is checked against it afterwards
    cap = rz.bin(rz.project(ds, cams), cams).n_pairs

    def step(timed: bool):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] if timed else None
        if timed:
            ev[0].record(stream)
        scores.zero_()
        vb = rz.project(ds, cams)
        if timed:
            ev[1].record(stream)
        rz.bin(vb, cams, read_count=False)
        if timed:
            ev[2].record(stream)
        rz.sort(vb, cams, capacity=cap)
        if timed:
            ev[3].record(stream)
        rz.render_score(vb, cams, scores=scores)
        if timed:
            ev[4].record(stream)
        return ev, vb

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if not rz.pairs_fit(runs[-1][1]):
        raise RuntimeError("the timed steps ran out of pair slots")
    evs = [r[0] for r in runs]
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
        "render_score": ("alu", (FUSED_FLOPS_VISIT * visited + FUSED_FLOPS_BLEND * blended) / 1e12),
        "project": ("hbm", PROJECT_BYTES_PER_SPLAT_VIEW * N * V / 1e9),
    }
    dom = max(work, key=lambda k: stage_ms[k])
    bound, amount = work[dom]
    sec = stage_ms[dom] / 1000.0
    if bound == "hbm":
        achieved, peak, unit = amount / sec, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = amount / sec, FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    ctr = measured_counters(f"k_{dom}")
    # VALU issue: the record's wave instructions per launch over the chip's issue limit
    # (one wave64 VALU instruction per CU per cycle) for the live kernel time
    valu = ctr.get("valu_insts_per_launch") if ctr else None
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(f"k_{dom}"), "kernel": f"k_{dom}",
                "kernel_ms": round(stage_ms[dom], 4),
                "valu_issue": None if valu is None else round(valu / (VALU_ISSUE_PER_S * sec), 4)}
    out = {
        "value": round(N * V / (ms / 1000.0) / 1e9, 4),
        "ms_per_step": round(ms, 4),
        "config": {"workload": "single-view removal scoring: 500k clustered splats, one 1280x720 view",
                   "splats": N, "views": V, "width": cams[0].width, "height": cams[0].height,
                   "tile": f"{s.tile_w}x{s.tile_h}", "lds_batch": s.lds_batch, "t_min": s.t_min,
                   "path": "plain per-view launches, fused composite + removal pass"},
        "roofline": roofline,
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "work": {"pairs": vb.n_pairs, "visited": visited, "blended": blended},
    }
    return out, (scene, cams, s)


def timed(torch, fn, reps, warm=1):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / reps


def batched_section(torch, raster, synth, batch, n_views=16):
    scene, cams = synth.workload_full_scene(n_views=n_views)
    s = synth.RenderSettings()
    ds = raster.to_device(scene)
    sc = torch.zeros(scene.n, device="cuda")
    rz = raster.Rasterizer(s)

    def plain():
        sc.zero_()
        rz.score_views_fused(ds, cams, views_per_batch=1, scores=sc)

    plain_ms = timed(torch, plain, 2)
    bs = batch.BatchScorer([(ds, cams, sc)], s, views_per_job=8)
    bs.capture()

    def replay():
        sc.zero_()
        bs.replay()

    graph_ms = timed(torch, replay, 3)
    over = bs.overflowed()
    counted, _ = bs.pairs()
    bs.close()
    del bs, rz, ds, sc
    torch.cuda.empty_cache()
    gs = lambda ms: round(scene.n * n_views / (ms / 1000.0) / 1e9, 4)
    return {"workload": f"{scene.n} clustered splats x {n_views} of the 200 hemisphere views at 1600x1064",
            "plain_ms_per_view": round(plain_ms / n_views, 4), "plain_gsplat_views_per_s": gs(plain_ms),
            "batched_graph_ms_per_view": round(graph_ms / n_views, 4), "batched_gsplat_views_per_s": gs(graph_ms),
            "pairs_per_view": int(sum(counted) / n_views), "overflowed_jobs": over}


def multi_scene_section(torch, raster, synth, batch):
    """16 scenes of uneven size (50 k..2 M splats, 8..32 views, three image sizes) scored
    in one batch: the autotuner picks tile shape and LDS batch on the whole batch, then
    per-job project/bin/sort and one persistent render + removal launch are replayed as
    one HIP graph."""
    work = synth.workload_batched()
    items = []
    for scene, cams in work:
        ds = raster.to_device(scene)
        items.append((ds, cams, torch.zeros(scene.n, device="cuda")))
    s, tune = batch.autotune(items, synth.RenderSettings(), reps=1)
    torch.cuda.empty_cache()
    bs = batch.BatchScorer(items, s, views_per_job=8)
    bs.capture()

    def replay():
        for it in items:
            it[2].zero_()
        bs.replay()

    ms = timed(torch, replay, 3)
    over = bs.overflowed()
    counted, _ = bs.pairs()
    bs.close()
    sv = sum(scene.n * len(cams) for scene, cams in work)
    nv = sum(len(cams) for _, cams in work)
    ns = sum(scene.n for scene, _ in work)
    del bs, items
    torch.cuda.empty_cache()
    return {"workload": f"{len(work)} clustered scenes, {ns} splats in all (50k..2M log-uniform), {nv} views "
                        f"(8..32 per scene) at 640x480, 1280x720 and 1600x1064",
            "autotuned": f"{s.tile_w}x{s.tile_h} tiles, LDS batch {s.lds_batch}",
            "autotune_ms": {f"{c['tile']}/{c['lds_batch']}": round(c["ms"], 2) for c in tune["tried"]},
            "ms_per_batch": round(ms, 3), "ms_per_view": round(ms / nv, 4),
            "gsplat_views_per_s": round(sv / (ms / 1000.0) / 1e9, 4),
            "pairs": int(sum(counted)), "overflowed_jobs": over}


def fwd_bwd_section(torch, raster, synth, autograd):
    scene, cams, target_scene = synth.workload_differentiation()
    s = synth.RenderSettings()
    ds = raster.to_device(scene)
    rz = raster.Rasterizer(s)
    with torch.no_grad():
        tgt = raster.Rasterizer(s).render_views(raster.to_device(target_scene), cams).image.clone()
    params = [t.clone().requires_grad_(True) for t in (ds.means, ds.scales, ds.quats, ds.opacities, ds.sh)]

    def step():
        for p in params:
            p.grad = None
        img = autograd.render(*params, cams, rz)
        loss = (img - tgt).abs().mean()
        loss.backward()

    ms = timed(torch, step, 5, warm=2)
    del params, rz, ds, tgt
    torch.cuda.empty_cache()
    return {"workload": f"{scene.n} clustered splats, {len(cams)} views at 1280x720, L1 loss vs a perturbed scene",
            "ms_per_view": round(ms / len(cams), 4), "ms_per_step": round(ms, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--main-only", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); multi-GPU scoring shards by view "
              f"and is not built here", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2601_14821_amd import autograd, batch, raster, synth

    main_out, (scene, cams, s) = main_line(args, torch, raster, synth)
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = {
        "metric": METRIC,
        "value": main_out["value"],
        "unit": "Gsplat·views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_out["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": main_out["config"],
        "roofline": main_out["roofline"],
        "stages_ms": main_out["stages_ms"],
        "work": main_out["work"],
    }
    if not args.main_only:
        out["batched"] = batched_section(torch, raster, synth, batch)
        out["multi_scene"] = multi_scene_section(torch, raster, synth, batch)
        out["fwd_bwd"] = fwd_bwd_section(torch, raster, synth, autograd)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, cams, s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
