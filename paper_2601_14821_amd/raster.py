"""Plain per-view pipeline over libpotr.so: project -> bin -> sort -> blend -> score.

PyTorch supplies device memory and the stream; every step of the pipeline runs
in the library's HIP kernels. The only host synchronisation is the read-back of
the pair count after binning (to size the sort); a caller that reuses the
Rasterizer keeps its buffers, so repeated calls allocate nothing new.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import torch

from . import _lib as L


@dataclasses.dataclass
class DeviceScene:
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opacities: torch.Tensor
    sh: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


def to_device(scene, device="cuda") -> DeviceScene:
    f = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
    return DeviceScene(f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacities), f(scene.sh))


@dataclasses.dataclass
class ViewBatch:
    """Device results for one batch of views (all views share one size)."""
    V: int
    N: int
    proj: torch.Tensor            # uint8 [V*N*48]
    tiles_touched: torch.Tensor   # int32 [V*N]
    order: torch.Tensor | None = None
    n_pairs: int = 0
    sorted_ids: torch.Tensor | None = None
    tile_ranges: torch.Tensor | None = None
    image: torch.Tensor | None = None
    p_final: torch.Tensor | None = None
    t_final: torch.Tensor | None = None
    n_walk: torch.Tensor | None = None
    n_blend: torch.Tensor | None = None


@dataclasses.dataclass
class Outputs:
    """Per-splat reductions of the fused pass (potr_outputs): each tensor is
    optional; view v of a call adds into tensor[v * stride :][:N] (stride 0: all
    views into one [N] array; stride N: a [V, N] array), every partial sum
    multiplied by the weight first."""
    scores: torch.Tensor | None = None
    scores_stride: int = 0
    scores_weight: float = 1.0
    scores_se: torch.Tensor | None = None
    se_stride: int = 0
    se_weight: float = 1.0
    importance: torch.Tensor | None = None
    importance_stride: int = 0
    importance_weight: float = 1.0
    # int64 tensors of fixed-point sums (units of 2^-32; fixed_to_float converts):
    # the same bits on every run
    fixed_point: bool = False

    def any(self) -> bool:
        return self.scores is not None or self.scores_se is not None or self.importance is not None


def fixed_to_float(acc: torch.Tensor) -> torch.Tensor:
    """potr_fixed_to_float: FP32 values of fixed-point sums (int64, units of 2^-32)."""
    out = torch.empty(acc.shape, dtype=torch.float32, device=acc.device)
    L.call("potr_fixed_to_float", L.ptr(acc), acc.numel(), L.ptr(out), L.stream_handle())
    return out


class Rasterizer:
    def __init__(self, settings, device="cuda"):
        self.s = settings
        self.cfg = L.make_config(settings)
        self.device = torch.device(device)
        self._bufs: dict[str, torch.Tensor] = {}
        L.lib()

    # -------------------------------------------------------------- buffers
    def _buf(self, name: str, nbytes: int) -> torch.Tensor:
        b = self._bufs.get(name)
        nbytes = max(int(nbytes), 256)
        if b is None or b.numel() < nbytes:
            b = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._bufs[name] = b
        return b

    def release(self) -> None:
        """Hand every buffer the rasterizer holds over to whoever references it:
        later calls allocate new ones instead of overwriting them."""
        self._bufs = {}

    def _i32(self, name: str, n: int) -> torch.Tensor:
        return self._buf(name, 4 * n)[: 4 * max(n, 1)].view(torch.int32)

    def _f32(self, name: str, n: int) -> torch.Tensor:
        return self._buf(name, 4 * n)[: 4 * max(n, 1)].view(torch.float32)

    def tiles(self, cam):
        return self.s.tiles(cam)

    # -------------------------------------------------------------- stages
    def project(self, ds: DeviceScene, cams, tag: str = "") -> ViewBatch:
        N, V = ds.n, len(cams)
        proj = self._buf("proj" + tag, L.PROJ_BYTES * V * N)[: L.PROJ_BYTES * max(V * N, 1)]
        tt = self._i32("tt" + tag, V * N)
        L.call("potr_project", N, V, L.make_cameras(cams), C.byref(self.cfg), L.ptr(ds.means), L.ptr(ds.scales),
               L.ptr(ds.quats), L.ptr(ds.opacities), L.ptr(ds.sh), L.ptr(proj), L.ptr(tt), L.stream_handle())
        return ViewBatch(V=V, N=N, proj=proj, tiles_touched=tt)

    def bin(self, vb: ViewBatch, cams, read_count: bool = True) -> ViewBatch:
        """Depth order per view and pair counts (potr_bin). With read_count the
        pair count is read back (a host synchronisation); without, vb.n_pairs
        stays None and sort() needs an explicit capacity (see pairs_fit)."""
        N, V = vb.N, vb.V
        cam_arr = L.make_cameras(cams)
        order = self._i32("order", V * N)
        n_pairs = self._buf("n_pairs", 8)[:8].view(torch.int64)
        ws = self._buf("bin_ws", L.bin_workspace_size(N, V, cam_arr, self.cfg))
        L.call("potr_bin", N, V, cam_arr, C.byref(self.cfg), L.ptr(vb.proj), L.ptr(ws), ws.numel(), L.ptr(order),
               L.ptr(n_pairs), L.stream_handle())
        n = None
        if read_count:
            n = int(n_pairs.item())
        vb.order, vb.n_pairs = order, n
        vb._bin_ws = ws
        vb._n_pairs_dev = n_pairs
        return vb

    def sort(self, vb: ViewBatch, cams, capacity: int | None = None) -> ViewBatch:
        """Tile lists in depth order (potr_sort) into a buffer of `capacity` ids
        (default: exactly the counted pairs)."""
        tx, ty = self.tiles(cams[0])
        if capacity is None and vb.n_pairs is None:
            raise ValueError("sort() after bin(read_count=False) needs a capacity")
        cap = vb.n_pairs if capacity is None else int(capacity)
        ids = self._i32("sorted_ids", cap)
        ranges = self._i32("ranges", 2 * vb.V * tx * ty)[: 2 * vb.V * tx * ty]
        sws = self._buf("sort_ws", L.sort_workspace_size(cap))
        L.call("potr_sort", vb.N, vb.V, L.make_cameras(cams), C.byref(self.cfg), L.ptr(vb.proj), L.ptr(vb.order),
               L.ptr(vb._bin_ws), vb._bin_ws.numel(), L.ptr(vb._n_pairs_dev), cap, L.ptr(sws), sws.numel(),
               L.ptr(ids), L.ptr(ranges), L.stream_handle())
        vb.sorted_ids, vb.tile_ranges = ids, ranges
        vb._capacity = cap
        return vb

    @staticmethod
    def pairs_fit(vb: ViewBatch) -> bool:
        """Whether the last sort had room for every pair (reads the count back)."""
        n = int(vb._n_pairs_dev.item())
        if vb.n_pairs is None:
            vb.n_pairs = n
        return 0 <= n <= vb._capacity

    def blend(self, vb: ViewBatch, cams, count_blended: bool = False) -> ViewBatch:
        V, H, W = vb.V, cams[0].height, cams[0].width
        P = V * H * W
        image = self._f32("image", 3 * P)[: 3 * P].view(V, H, W, 3)
        pf = self._f32("p_final", 3 * P)[: 3 * P].view(V, H, W, 3)
        tf = self._f32("t_final", P)[:P].view(V, H, W)
        nw = self._i32("n_walk", P)[:P].view(V, H, W)
        nb = self._i32("n_blend", P)[:P].view(V, H, W) if count_blended else None
        L.call("potr_blend", vb.N, V, L.make_cameras(cams), C.byref(self.cfg), L.ptr(vb.proj), L.ptr(vb.sorted_ids),
               L.ptr(vb.tile_ranges), L.ptr(image), L.ptr(pf), L.ptr(tf), L.ptr(nw), L.ptr(nb), L.stream_handle())
        vb.image, vb.p_final, vb.t_final, vb.n_walk, vb.n_blend = image, pf, tf, nw, nb
        return vb

    def score(self, vb: ViewBatch, cams, scores=None, scores_se=None, importance=None, target=None) -> None:
        L.call("potr_score", vb.N, vb.V, L.make_cameras(cams), C.byref(self.cfg), L.ptr(vb.proj),
               L.ptr(vb.sorted_ids), L.ptr(vb.tile_ranges), L.ptr(vb.p_final), L.ptr(vb.t_final),
               L.ptr(vb.n_walk), L.ptr(target), L.ptr(scores), L.ptr(scores_se), L.ptr(importance),
               L.stream_handle())

    # -------------------------------------------------------------- whole path
    def render_views(self, ds: DeviceScene, cams) -> ViewBatch:
        vb = self.project(ds, cams)
        self.bin(vb, cams)
        self.sort(vb, cams)
        self.blend(vb, cams)
        return vb

    def score_views(self, ds: DeviceScene, cams, views_per_batch: int = 8, scores=None, importance=None,
                    scores_se=None, targets=None, keep_images: bool = False):
        """Removal scores accumulated over all views. Returns (scores, importance, images?)."""
        N = ds.n
        if scores is None:
            scores = torch.zeros(N, dtype=torch.float32, device=self.device)
        images = []
        for v0 in range(0, len(cams), views_per_batch):
            cb = cams[v0:v0 + views_per_batch]
            vb = self.render_views(ds, cb)
            tgt = None if targets is None else targets[v0:v0 + len(cb)].contiguous()
            self.score(vb, cb, scores=scores, scores_se=scores_se, importance=importance, target=tgt)
            if keep_images:
                images.append(vb.image.clone())
        return scores, importance, (torch.cat(images) if keep_images else None)

    # -------------------------------------------------------------- backward
    def backward(self, ds: DeviceScene, vb: ViewBatch, cams, dL_dimage: torch.Tensor, grads=None,
                 grad2d: torch.Tensor | None = None) -> dict:
        """Gradients (+=) of the splat parameters for dL/dimage [V,H,W,3] of the views in `vb`.
        With `grad2d` given ([V*N*9] float32, zeroed by the caller) the screen-space
        gradients are kept there and chained from it."""
        N, V = vb.N, vb.V
        if grads is None:
            grads = {k: torch.zeros_like(getattr(ds, a)) for k, a in
                     (("means", "means"), ("scales", "scales"), ("quats", "quats"), ("opacities", "opacities"),
                      ("sh", "sh"))}
        g = dL_dimage.contiguous()
        cams_arr = L.make_cameras(cams)
        if grad2d is None:
            b = C.c_size_t(0)
            L.call("potr_backward_workspace_size", N, V, C.byref(b))
            ws = self._buf("bwd_ws", b.value)
            L.call("potr_backward", N, V, cams_arr, C.byref(self.cfg), L.ptr(ds.means), L.ptr(ds.scales),
                   L.ptr(ds.quats), L.ptr(ds.opacities), L.ptr(ds.sh), L.ptr(vb.proj), L.ptr(vb.sorted_ids),
                   L.ptr(vb.tile_ranges), L.ptr(vb.p_final), L.ptr(vb.t_final), L.ptr(vb.n_walk), L.ptr(g),
                   L.ptr(ws), ws.numel(), L.ptr(grads["means"]), L.ptr(grads["scales"]), L.ptr(grads["quats"]),
                   L.ptr(grads["opacities"]), L.ptr(grads["sh"]), L.stream_handle())
        else:
            L.call("potr_blend_backward", N, V, cams_arr, C.byref(self.cfg), L.ptr(vb.proj), L.ptr(vb.sorted_ids),
                   L.ptr(vb.tile_ranges), L.ptr(vb.p_final), L.ptr(vb.t_final), L.ptr(vb.n_walk), L.ptr(g),
                   L.ptr(grad2d), L.stream_handle())
            L.call("potr_project_backward", N, V, cams_arr, C.byref(self.cfg), L.ptr(ds.means), L.ptr(ds.scales),
                   L.ptr(ds.quats), L.ptr(ds.opacities), L.ptr(ds.sh), L.ptr(grad2d), L.ptr(grads["means"]),
                   L.ptr(grads["scales"]), L.ptr(grads["quats"]), L.ptr(grads["opacities"]), L.ptr(grads["sh"]),
                   L.stream_handle())
        return grads

    # -------------------------------------------------------------- fused forward + removal
    def render_score(self, vb: ViewBatch, cams, scores=None, importance=None, image=None, scores_se=None,
                     target=None) -> None:
        """potr_render_score: composite and score the views of `vb` in one launch."""
        L.call("potr_render_score", vb.N, vb.V, L.make_cameras(cams), C.byref(self.cfg), L.ptr(vb.proj),
               L.ptr(vb.sorted_ids), L.ptr(vb.tile_ranges), L.ptr(image), L.ptr(target), L.ptr(scores),
               L.ptr(scores_se), L.ptr(importance), L.stream_handle())

    def render_score_out(self, vb: ViewBatch, cams, out: Outputs, v0: int = 0, image=None, target=None) -> None:
        """potr_render_score_out: the views of `vb` are views v0.. of `out`'s arrays."""
        o = L.make_outputs(out, v0)
        L.call("potr_render_score_out", vb.N, vb.V, L.make_cameras(cams), C.byref(self.cfg), L.ptr(vb.proj),
               L.ptr(vb.sorted_ids), L.ptr(vb.tile_ranges), L.ptr(image), L.ptr(target), C.byref(o),
               L.stream_handle())

    def score_views_fused(self, ds: DeviceScene, cams, views_per_batch: int = 8, scores=None, importance=None,
                          out: Outputs | None = None, targets=None):
        """Removal scores over all views with the fused launch (no per-pixel buffers).
        With `out`, its description is used (per-view arrays, weights, dSE with
        `targets` [V,H,W,3]); otherwise scores (and importance) accumulate raw."""
        if out is None:
            if scores is None:
                scores = torch.zeros(ds.n, dtype=torch.float32, device=self.device)
            out = Outputs(scores=scores, importance=importance)
        for v0 in range(0, len(cams), views_per_batch):
            cb = cams[v0:v0 + views_per_batch]
            vb = self.project(ds, cb)
            self.bin(vb, cb)
            self.sort(vb, cb)
            tgt = None if targets is None else targets[v0:v0 + len(cb)].contiguous()
            self.render_score_out(vb, cb, out, v0=v0, target=tgt)
        return out.scores

    def removal_statistics(self, ds: DeviceScene, cams, targets, per_view_importance: bool = False,
                           views_per_batch: int = 8):
        """The pruning controller's inputs, normalised as in the paper: dMSE_k
        (Sec. 4.2, the camera-, pixel- and channel-averaged dSE against the
        target images [V,H,W,3]) and I_k (Sec. 4.1, the camera average of the
        image fraction I_k(s)); with per_view_importance also I_k(s) [V, N].
        Every view must have the same size. Returns (dmse, importance, per_view)."""
        N, V = ds.n, len(cams)
        P = cams[0].width * cams[0].height
        if any(c.width * c.height != P for c in cams):
            raise ValueError("removal_statistics needs views of one size")
        dmse = torch.zeros(N, dtype=torch.float32, device=self.device)
        imp = torch.zeros(N, dtype=torch.float32, device=self.device)
        out = Outputs(scores_se=dmse, se_weight=1.0 / (3.0 * V * P), importance=imp, importance_weight=1.0 / (V * P))
        self.score_views_fused(ds, cams, views_per_batch, out=out, targets=targets)
        per_view = None
        if per_view_importance:
            per_view = torch.zeros(V, N, dtype=torch.float32, device=self.device)
            self.score_views_fused(ds, cams, views_per_batch,
                                   out=Outputs(importance=per_view, importance_stride=N, importance_weight=1.0 / P))
        return dmse, imp, per_view
