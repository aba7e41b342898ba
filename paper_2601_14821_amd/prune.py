"""Iterative pruning controller (paper Sec. 4.3) over libpotr.so.

    pc = PruneController(ds, cams, settings)      # target = the unpruned render
    for _ in range(pc.n_iter):
        pc.step()
    survivors = pc.ids                            # original indices of the kept splats

Each iteration scores the surviving splats over every view (dMSE_k against the
target images and importance I_k, normalised as Sec. 4.1 and 4.2 define them,
with the fused render + removal kernel), lets potr_prune_select choose the
splats to remove, and compacts the survivors with potr_prune_compact. The only
host synchronisation per iteration is the read-back of the survivor count.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _lib as L
from .raster import DeviceScene, Rasterizer


def hyperparameters(q: float = 0.5) -> dict:
    """The paper's pruning hyperparameters as functions of the quality
    parameter q (Sec. 5.1, hyperparameter table): dMSE_MAX = 10^(-8.8 - 2q),
    48 iterations; the mapping's a = 10 (Sec. 4.3)."""
    return {"dmse_max": 10.0 ** (-8.8 - 2.0 * q), "n_iter": 48, "a": 10.0}


def _workspace(N: int, device) -> torch.Tensor:
    b = C.c_size_t(0)
    L.call("potr_prune_workspace_size", N, C.byref(b))
    return torch.empty(max(b.value, 256), dtype=torch.uint8, device=device)


def select(dmse: torch.Tensor, importance: torch.Tensor, dmse_max: float, remaining: int, a: float = 10.0,
           ws: torch.Tensor | None = None):
    """potr_prune_select: (remove mask uint8 [N], removed count as a device int64 tensor)."""
    N = dmse.numel()
    dev = dmse.device
    if ws is None:
        ws = _workspace(N, dev)
    remove = torch.empty(max(N, 1), dtype=torch.uint8, device=dev)[:N]
    n = torch.empty(1, dtype=torch.int64, device=dev)
    L.call("potr_prune_select", N, L.ptr(dmse), L.ptr(importance), float(dmse_max), int(remaining), float(a),
           L.ptr(ws), ws.numel(), L.ptr(remove), L.ptr(n), L.stream_handle())
    return remove, n


def compact(ds: DeviceScene, remove: torch.Tensor, ids: torch.Tensor | None = None,
            ws: torch.Tensor | None = None):
    """potr_prune_compact: (surviving scene, their ids, survivor count)."""
    N = ds.n
    dev = ds.means.device
    if ws is None:
        ws = _workspace(N, dev)
    out = DeviceScene(torch.empty_like(ds.means), torch.empty_like(ds.scales), torch.empty_like(ds.quats),
                      torch.empty_like(ds.opacities), torch.empty_like(ds.sh))
    ids_out = torch.empty(max(N, 1), dtype=torch.int32, device=dev)
    n = torch.empty(1, dtype=torch.int64, device=dev)
    L.call("potr_prune_compact", N, L.ptr(remove), L.ptr(ds.means), L.ptr(ds.scales), L.ptr(ds.quats),
           L.ptr(ds.opacities), L.ptr(ds.sh), L.ptr(ids), L.ptr(ws), ws.numel(), L.ptr(out.means),
           L.ptr(out.scales), L.ptr(out.quats), L.ptr(out.opacities), L.ptr(out.sh), L.ptr(ids_out), L.ptr(n),
           L.stream_handle())
    k = int(n.item())
    kept = DeviceScene(out.means[:k], out.scales[:k], out.quats[:k], out.opacities[:k], out.sh[:k])
    return kept, ids_out[:k], k


class PruneController:
    """The iterative controller of Sec. 4.3 over a device scene and its views
    (all of one size). `targets` [V,H,W,3] defaults to the render of the
    unpruned scene (the paper's fixed reference colour c_t)."""

    def __init__(self, ds: DeviceScene, cams, settings, n_iter: int | None = None, dmse_max: float | None = None,
                 a: float | None = None, targets: torch.Tensor | None = None, views_per_batch: int = 8):
        hp = hyperparameters()
        self.n_iter = hp["n_iter"] if n_iter is None else int(n_iter)
        self.dmse_max = hp["dmse_max"] if dmse_max is None else float(dmse_max)
        self.a = hp["a"] if a is None else float(a)
        self.cams = cams
        self.vpb = views_per_batch
        self.rz = Rasterizer(settings, ds.means.device)
        self.ds = ds
        self.ids = torch.arange(ds.n, dtype=torch.int32, device=ds.means.device)
        self.it = 0
        if targets is None:
            targets = self.render(ds)
        self.targets = targets
        self.last = None

    def render(self, ds: DeviceScene) -> torch.Tensor:
        """Images [V,H,W,3] of a scene over the controller's views."""
        imgs = []
        for v0 in range(0, len(self.cams), self.vpb):
            cb = self.cams[v0:v0 + self.vpb]
            imgs.append(self.rz.render_views(ds, cb).image.clone())
        return torch.cat(imgs)

    def statistics(self):
        """(dMSE_k, I_k) of the current survivors."""
        dmse, imp, _ = self.rz.removal_statistics(self.ds, self.cams, self.targets, views_per_batch=self.vpb)
        return dmse, imp

    def step(self) -> int:
        """One iteration; returns how many splats it removed."""
        if self.it >= self.n_iter:
            raise RuntimeError("every iteration has run")
        dmse, imp = self.statistics()
        remove, n = select(dmse, imp, self.dmse_max, self.n_iter - self.it, self.a)
        self.last = {"dmse": dmse, "importance": imp, "remove": remove}
        kept, ids, k = compact(self.ds, remove, self.ids)
        removed = int(n.item())
        if removed < 0:
            raise RuntimeError("importance out of range: the statistics are not normalised")
        self.ds, self.ids = kept, ids
        self.it += 1
        return removed
