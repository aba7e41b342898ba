"""FP64 CPU oracle for the POTR removal-effect rasterizer -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py`
may import this package. It wraps `liboracle.so`, built from `potr_oracle.c` by
`oracle.build_lib()` with gcc; it shares no code with the HIP path.

Every function takes numpy inputs (the FP32 scene and cameras from
`paper_2601_14821_amd.synth`) and returns FP64 numpy outputs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "potr_oracle.c")


def build_lib(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fused contraction, IEEE semantics)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, SRC, "-lm", "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Cam(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class _Cfg(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("eps2d", C.c_float), ("near_z", C.c_float),
                ("jclamp", C.c_float), ("alpha_min", C.c_float), ("alpha_max", C.c_float),
                ("q_max", C.c_float), ("t_min", C.c_float), ("bg", C.c_float * 3), ("sh_degree", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_lib()
        _lib = C.CDLL(LIB_PATH)
        _lib.orc_bin_sort.restype = C.c_int64
        _lib.orc_render.restype = C.c_int64
    return _lib


def _cam(cam) -> _Cam:
    c = _Cam()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).reshape(-1)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32).reshape(-1)]
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    c.width, c.height = cam.width, cam.height
    return c


def _cfg(s) -> _Cfg:
    c = _Cfg()
    c.tile_w, c.tile_h = s.tile_w, s.tile_h
    c.eps2d, c.near_z, c.jclamp = s.eps2d, s.near, s.jclamp
    c.alpha_min, c.alpha_max, c.q_max, c.t_min = s.alpha_min, s.alpha_max, s.q_max, s.t_min
    c.bg[:] = [float(x) for x in s.bg]
    c.sh_degree = s.sh_degree
    return c


def _p(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def sh_basis(lmax: int, d) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros((lmax + 1) ** 2)
    lib().orc_sh_basis(C.c_int32(lmax), _p(d, C.c_double), _p(out, C.c_double))
    return out


def project(scene, cam, s) -> dict:
    n = scene.n
    out = dict(mean2d=np.zeros((n, 2)), cov2d=np.zeros((n, 3)), conic=np.zeros((n, 3)),
               rgb=np.zeros((n, 3)), depth_key=np.zeros(n, np.uint32), rect=np.zeros((n, 4), np.int32),
               tiles_touched=np.zeros(n, np.int32))
    m, sc, q, o, sh = (_f64(a) for a in (scene.means, scene.scales, scene.quats, scene.opacities, scene.sh))
    cm, cf = _cam(cam), _cfg(s)
    lib().orc_project(C.c_int64(n), C.byref(cm), C.byref(cf), _p(m, C.c_double), _p(sc, C.c_double),
                      _p(q, C.c_double), _p(o, C.c_double), _p(sh, C.c_double),
                      _p(out["mean2d"], C.c_double), _p(out["cov2d"], C.c_double),
                      _p(out["conic"], C.c_double), _p(out["rgb"], C.c_double),
                      _p(out["depth_key"], C.c_uint32), _p(out["rect"], C.c_int32),
                      _p(out["tiles_touched"], C.c_int32))
    return out


def bin_sort(rect, depth_key, tiles_x: int, tiles_y: int):
    """Tile lists ordered by (tile, depth key, splat id): (tile, id, tile_ranges[T, 2])."""
    rect = np.ascontiguousarray(rect, np.int32)
    key = np.ascontiguousarray(depth_key, np.uint32)
    n = rect.shape[0]
    L = lib()
    npairs = L.orc_bin_sort(C.c_int64(n), C.c_int32(tiles_x), C.c_int32(tiles_y), _p(rect, C.c_int32),
                            _p(key, C.c_uint32), None, None, None)
    tile = np.zeros(max(npairs, 1), np.int32)
    ids = np.zeros(max(npairs, 1), np.int32)
    ranges = np.zeros((tiles_x * tiles_y, 2), np.int32)
    L.orc_bin_sort(C.c_int64(n), C.c_int32(tiles_x), C.c_int32(tiles_y), _p(rect, C.c_int32),
                   _p(key, C.c_uint32), _p(tile, C.c_int32), _p(ids, C.c_int32), _p(ranges, C.c_int32))
    return tile[:npairs], ids[:npairs], ranges


def default_threads() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def render(scene, cam, s, proj=None, bins=None, target=None, method: int = 0, threads: int | None = None,
           record_f32: bool = False,
           want=("image", "p_final", "t_final", "n_walk", "n_blend", "score_l1", "importance",
                 "magnitude", "flag_mass", "pixel_flag")) -> dict:
    """Composite one view and reduce the removal effect per splat (see potr_oracle.h)."""
    if proj is None:
        proj = project(scene, cam, s)
    tx, ty = s.tiles(cam)
    if bins is None:
        bins = bin_sort(proj["rect"], proj["depth_key"], tx, ty)
    _, ids, ranges = bins
    n, H, W = scene.n, cam.height, cam.width
    shapes = dict(image=((H, W, 3), np.float64), p_final=((H, W, 3), np.float64), t_final=((H, W), np.float64),
                  n_walk=((H, W), np.int32), n_blend=((H, W), np.int32), score_l1=((n,), np.float64),
                  score_se=((n,), np.float64), importance=((n,), np.float64), magnitude=((n,), np.float64),
                  flag_mass=((n,), np.float64), pixel_flag=((H, W), np.uint8))
    out = {k: np.zeros(*shapes[k]) for k in want}
    if "score_se" in want and target is None:
        raise ValueError("score_se needs a target image")
    tgt = None if target is None else _f32(target)
    cm, cf = _cam(cam), _cfg(s)
    ids = np.ascontiguousarray(ids, np.int32)
    ranges = np.ascontiguousarray(ranges, np.int32)
    g = lambda k, ct: _p(out.get(k), ct)
    nflag = lib().orc_render(
        C.c_int64(n), C.byref(cm), C.byref(cf), _p(proj["mean2d"], C.c_double), _p(proj["conic"], C.c_double),
        _p(proj["rgb"], C.c_double), _p(_f64(scene.opacities), C.c_double), _p(ranges, C.c_int32),
        _p(ids, C.c_int32), _p(tgt, C.c_float), C.c_int32(method), C.c_int32(int(record_f32)),
        C.c_int32(threads or default_threads()),
        g("image", C.c_double), g("p_final", C.c_double), g("t_final", C.c_double), g("n_walk", C.c_int32),
        g("n_blend", C.c_int32), g("score_l1", C.c_double), g("score_se", C.c_double),
        g("importance", C.c_double), g("magnitude", C.c_double), g("flag_mass", C.c_double),
        g("pixel_flag", C.c_uint8))
    out["n_flagged"] = int(nflag)
    out["proj"] = proj
    out["bins"] = bins
    return out


def render_without(scene, cam, s, k: int, proj=None, bins=None, record_f32: bool = False) -> np.ndarray:
    """Image [H, W, 3] composited with splat k deleted (the plain definition of removal)."""
    if proj is None:
        proj = project(scene, cam, s)
    tx, ty = s.tiles(cam)
    if bins is None:
        bins = bin_sort(proj["rect"], proj["depth_key"], tx, ty)
    _, ids, ranges = bins
    img = np.zeros((cam.height, cam.width, 3))
    lib().orc_render_without(C.c_int64(scene.n), C.byref(_cam(cam)), C.byref(_cfg(s)),
                             _p(proj["mean2d"], C.c_double), _p(proj["conic"], C.c_double),
                             _p(proj["rgb"], C.c_double), _p(_f64(scene.opacities), C.c_double),
                             _p(np.ascontiguousarray(ranges, np.int32), C.c_int32),
                             _p(np.ascontiguousarray(ids, np.int32), C.c_int32), C.c_int64(k),
                             C.c_int32(int(record_f32)), _p(img, C.c_double))
    return img


def score_views(scene, cams, s, method: int = 0, threads: int | None = None, target_images=None,
                record_f32: bool = False,
                want=("image", "score_l1", "importance", "magnitude", "flag_mass", "pixel_flag")):
    """Accumulate per-splat outputs over several views; returns (totals, per_view list)."""
    tot = {}
    views = []
    for v, cam in enumerate(cams):
        tgt = None if target_images is None else target_images[v]
        r = render(scene, cam, s, target=tgt, method=method, threads=threads, record_f32=record_f32, want=want)
        views.append(r)
        for k in ("score_l1", "score_se", "importance", "magnitude", "flag_mass"):
            if k in r:
                tot[k] = tot.get(k, 0.0) + r[k]
        tot["n_flagged"] = tot.get("n_flagged", 0) + r["n_flagged"]
    return tot, views


def backward(scene, cam, s, dL_dimage, proj=None, bins=None, threads: int | None = None) -> dict:
    """Analytic FP64 gradient of a loss through one view given dL/dimage [H, W, 3]."""
    if proj is None:
        proj = project(scene, cam, s)
    tx, ty = s.tiles(cam)
    if bins is None:
        bins = bin_sort(proj["rect"], proj["depth_key"], tx, ty)
    _, ids, ranges = bins
    n = scene.n
    out = dict(d_means=np.zeros((n, 3)), d_scales=np.zeros((n, 3)), d_quats=np.zeros((n, 4)),
               d_opac=np.zeros(n), d_sh=np.zeros((n, 16, 3)), d_mean2d=np.zeros((n, 2)),
               d_conic=np.zeros((n, 3)), d_rgb=np.zeros((n, 3)))
    m, sc, q, o, sh = (_f64(a) for a in (scene.means, scene.scales, scene.quats, scene.opacities, scene.sh))
    g = _f64(dL_dimage)
    assert g.shape == (cam.height, cam.width, 3)
    d = lambda k: _p(out[k], C.c_double)
    lib().orc_backward(C.c_int64(n), C.byref(_cam(cam)), C.byref(_cfg(s)), _p(m, C.c_double),
                       _p(sc, C.c_double), _p(q, C.c_double), _p(o, C.c_double), _p(sh, C.c_double),
                       _p(proj["mean2d"], C.c_double), _p(proj["conic"], C.c_double), _p(proj["rgb"], C.c_double),
                       _p(np.ascontiguousarray(ranges, np.int32), C.c_int32),
                       _p(np.ascontiguousarray(ids, np.int32), C.c_int32), _p(g, C.c_double),
                       C.c_int32(threads or default_threads()), d("d_means"), d("d_scales"), d("d_quats"),
                       d("d_opac"), d("d_sh"), d("d_mean2d"), d("d_conic"), d("d_rgb"))
    out["proj"] = proj
    out["bins"] = bins
    return out
