"""Batched scoring of many scenes and views (potr_batch_* of include/potr.h).

    bs = BatchScorer([(ds0, cams0, scores0), (ds1, cams1, scores1)], settings)
    bs.run()                  # or: bs.capture(); bs.replay()
    assert bs.overflowed() == 0

An item is (scene, cameras, scores[, importance]) with [N] tensors, or
(scene, cameras, raster.Outputs[, targets[, FineTune]]) for per-view arrays,
weights and dSE sums against target images [V,H,W,3] (outputs may be an empty
Outputs() when the item only runs a fine-tuning step).

Scenes are split into jobs of at most `views_per_job` views (one image size per
job). The library plans pair capacities by counting once at construction, runs
project -> bin -> sort per job and one persistent render + removal launch over
all (view, tile) items, and can record the whole run into one HIP graph.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import json
import os

import torch

import dataclasses

from . import _lib as L
from .raster import DeviceScene, Outputs


@dataclasses.dataclass
class FineTune:
    """The fine-tuning step of an item (Sec. 4.6): the gradients of
    weight * sum |image - target| over the item's views are ADDED into the
    grads (d_means, d_scales, d_quats, d_opac, d_sh: tensors shaped like the
    scene's parameters). weight = 1 / (V H W 3) makes it the mean L1 loss."""
    target: torch.Tensor          # [V, H, W, 3]
    grads: DeviceScene
    weight: float = 1.0


class BatchScorer:
    def __init__(self, scenes, settings, views_per_job: int = 8, margin: float = 0.05, device="cuda"):
        self.s = settings
        self.cfg = L.make_config(settings)
        self.device = torch.device(device)
        self._keep = []
        jobs = []
        for item in scenes:
            ds, cams, out = item[0], item[1], item[2]
            targets, step = None, None
            if isinstance(out, Outputs):
                targets = item[3] if len(item) > 3 else None
                step = item[4] if len(item) > 4 else None
            else:
                out = Outputs(scores=out, importance=item[3] if len(item) > 3 else None)
            if targets is not None:
                targets = targets.contiguous()
                self._keep.append(targets)
            if step is not None:
                step = FineTune(step.target.contiguous(), step.grads, step.weight)
                self._keep.append(step)
            for v0 in range(0, len(cams), views_per_job):
                cb = cams[v0:v0 + views_per_job]
                arr = L.make_cameras(cb)
                self._keep.append(arr)
                j = L.potr_job()
                j.N = ds.n
                j.means, j.scales, j.quats = L.ptr(ds.means), L.ptr(ds.scales), L.ptr(ds.quats)
                j.opac, j.sh = L.ptr(ds.opacities), L.ptr(ds.sh)
                j.V = len(cb)
                j.cams = C.cast(arr, C.POINTER(L.potr_camera))
                j.out = L.make_outputs(out, v0)
                j.target = None if targets is None else targets[v0].data_ptr()
                if step is not None:
                    g = step.grads
                    j.grad_target = step.target[v0].data_ptr()
                    j.grad_weight = float(step.weight)
                    j.d_means, j.d_scales, j.d_quats = L.ptr(g.means), L.ptr(g.scales), L.ptr(g.quats)
                    j.d_opac, j.d_sh = L.ptr(g.opacities), L.ptr(g.sh)
                jobs.append(j)
        self.n_jobs = len(jobs)
        self.jobs = (L.potr_job * self.n_jobs)(*jobs)
        self._handle = C.c_void_p()
        L.call("potr_batch_create", self.jobs, self.n_jobs, C.byref(self.cfg), margin, C.byref(self._handle),
               L.stream_handle())
        b = C.c_size_t(0)
        L.call("potr_batch_workspace_size", self._handle, C.byref(b))
        self.ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=self.device)
        L.call("potr_batch_bind", self._handle, L.ptr(self.ws), self.ws.numel(), L.stream_handle())
        self._graph_stream = None

    def pairs(self):
        counted = (C.c_int64 * self.n_jobs)()
        cap = (C.c_int64 * self.n_jobs)()
        L.call("potr_batch_pairs", self._handle, counted, cap)
        return list(counted), list(cap)

    def run(self) -> None:
        L.call("potr_batch_run", self._handle, L.stream_handle())

    def render(self) -> None:
        """Only the persistent render + removal launch over the lists of the last run."""
        L.call("potr_batch_render", self._handle, L.stream_handle())

    def capture(self) -> None:
        """Record run() into a HIP graph on a side stream (default priority)."""
        if self._graph_stream is None:
            self._graph_stream = torch.cuda.Stream(device=self.device)
        self._graph_stream.wait_stream(torch.cuda.current_stream())
        L.call("potr_batch_capture", self._handle, self._graph_stream.cuda_stream)
        torch.cuda.current_stream().wait_stream(self._graph_stream)

    def replay(self) -> None:
        L.call("potr_batch_replay", self._handle, L.stream_handle())

    def overflowed(self) -> int:
        n = C.c_int32(0)
        L.call("potr_batch_overflow", self._handle, C.byref(n), L.stream_handle())
        return n.value

    def close(self) -> None:
        if self._handle:
            L.lib().potr_batch_destroy(self._handle)
            self._handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _signature(scenes, settings) -> str:
    parts = [(int(ds.n), len(cams), cams[0].width, cams[0].height) for ds, cams, *_ in scenes]
    key = json.dumps([parts, settings.t_min, settings.q_max, settings.alpha_min, settings.sh_degree])
    return hashlib.sha1(key.encode()).hexdigest()


def autotune(scenes, settings, reps: int = 2, views_per_job: int = 8, cache_path: str | None = None):
    """Pick tile shape and LDS batch by timing all candidates on `scenes`.
    Returns (settings with the choice, {"best_ms": ..., "tried": [...]}). Results are
    cached in a JSON file (POTR_AUTOTUNE_CACHE or `cache_path`) keyed by shapes."""
    cache_path = cache_path or os.environ.get("POTR_AUTOTUNE_CACHE")
    sig = _signature(scenes, settings)
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if sig in cache:
            c = cache[sig]
            return settings.replace(tile_w=c["tile_w"], tile_h=c["tile_h"], lds_batch=c["lds_batch"]), c
    jobs = []
    keep = []
    for ds, cams, *_ in scenes:
        for v0 in range(0, len(cams), views_per_job):
            cb = cams[v0:v0 + views_per_job]
            arr = L.make_cameras(cb)
            keep.append(arr)
            j = L.potr_job()
            j.N = ds.n
            j.means, j.scales, j.quats = L.ptr(ds.means), L.ptr(ds.scales), L.ptr(ds.quats)
            j.opac, j.sh = L.ptr(ds.opacities), L.ptr(ds.sh)
            j.V = len(cb)
            j.cams = C.cast(arr, C.POINTER(L.potr_camera))
            jobs.append(j)
    arr = (L.potr_job * len(jobs))(*jobs)
    cfg = L.make_config(settings)
    best = C.c_double(0.0)
    tried = (L.potr_config * 12)()
    tried_ms = (C.c_double * 12)()
    n = C.c_int32(0)
    L.call("potr_autotune", arr, len(jobs), C.byref(cfg), reps, C.byref(best), tried, tried_ms, C.byref(n),
           L.stream_handle())
    info = {"tile_w": cfg.tile_w, "tile_h": cfg.tile_h, "lds_batch": cfg.lds_batch, "best_ms": best.value,
            "tried": [{"tile": f"{tried[k].tile_w}x{tried[k].tile_h}", "lds_batch": tried[k].lds_batch,
                       "ms": tried_ms[k]} for k in range(n.value)]}
    if cache_path:
        cache = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        cache[sig] = info
        json.dump(cache, open(cache_path, "w"), indent=1)
    return settings.replace(tile_w=cfg.tile_w, tile_h=cfg.tile_h, lds_batch=cfg.lds_batch), info
