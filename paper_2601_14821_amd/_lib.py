"""ctypes binding of libpotr.so (include/potr.h). Argument marshalling only.

Names mirror the C entry points. Buffers are torch tensors on the GPU; their
device pointers are passed as-is. Loading fails loudly if libpotr.so is
missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpotr.so")

POTR_OK, POTR_EINVAL, POTR_ECAPACITY, POTR_EHIP, POTR_EUNSUPPORTED = 0, -1, -2, -3, -4
PROJ_BYTES = 48
# potr_proj as a numpy record (for inspecting device results on the host)
PROJ_DTYPE = np.dtype([("mean2d", "<f4", (2,)), ("conic", "<f4", (3,)), ("opacity", "<f4"), ("rgb", "<f4", (3,)),
                       ("depth", "<f4"), ("rect", "<i2", (4,))])
assert PROJ_DTYPE.itemsize == PROJ_BYTES

# every function the header declares, with its argument and return types
_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t


class potr_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class potr_config(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("lds_batch", C.c_int32),
                ("eps2d", C.c_float), ("near_z", C.c_float), ("jclamp", C.c_float),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("q_max", C.c_float),
                ("t_min", C.c_float), ("bg", C.c_float * 3), ("sh_degree", C.c_int32)]


class potr_outputs(C.Structure):
    _fields_ = [("scores", C.c_void_p), ("scores_stride", C.c_int64), ("scores_weight", C.c_float),
                ("scores_se", C.c_void_p), ("se_stride", C.c_int64), ("se_weight", C.c_float),
                ("importance", C.c_void_p), ("importance_stride", C.c_int64), ("importance_weight", C.c_float),
                ("fixed_point", C.c_int32)]


class potr_job(C.Structure):
    _fields_ = [("N", C.c_int64), ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opac", C.c_void_p), ("sh", C.c_void_p), ("V", C.c_int32), ("cams", C.POINTER(potr_camera)),
                ("out", potr_outputs), ("target", C.c_void_p), ("grad_target", C.c_void_p),
                ("grad_weight", C.c_float), ("d_means", C.c_void_p), ("d_scales", C.c_void_p),
                ("d_quats", C.c_void_p), ("d_opac", C.c_void_p), ("d_sh", C.c_void_p)]


_CAM_P, _CFG_P, _JOB_P = C.POINTER(potr_camera), C.POINTER(potr_config), C.POINTER(potr_job)
_OUT_P = C.POINTER(potr_outputs)

SIGNATURES = {
    "potr_abi_version": (_i32, []),
    "potr_last_error": (C.c_char_p, []),
    "potr_project": (_i32, [_i64, _i32, _CAM_P, _CFG_P, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "potr_bin_workspace_size": (_i32, [_i64, _i32, _CAM_P, _CFG_P, C.POINTER(_sz)]),
    "potr_bin": (_i32, [_i64, _i32, _CAM_P, _CFG_P, _vp, _vp, _sz, _vp, _vp, _vp]),
    "potr_sort_workspace_size": (_i32, [_i64, C.POINTER(_sz)]),
    "potr_sort": (_i32, [_i64, _i32, _CAM_P, _CFG_P, _vp, _vp, _vp, _sz, _vp, _i64, _vp, _sz, _vp, _vp, _vp]),
    "potr_blend": (_i32, [_i64, _i32, _CAM_P, _CFG_P, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "potr_score": (_i32, [_i64, _i32, _CAM_P, _CFG_P, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "potr_blend_backward": (_i32, [_i64, _i32, _CAM_P, _CFG_P, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "potr_project_backward": (_i32, [_i64, _i32, _CAM_P, _CFG_P] + [_vp] * 12),
    "potr_backward_workspace_size": (_i32, [_i64, _i32, C.POINTER(_sz)]),
    "potr_backward": (_i32, [_i64, _i32, _CAM_P, _CFG_P] + [_vp] * 13 + [_sz] + [_vp] * 6),
    "potr_render_score": (_i32, [_i64, _i32, _CAM_P, _CFG_P] + [_vp] * 9),
    "potr_render_score_out": (_i32, [_i64, _i32, _CAM_P, _CFG_P] + [_vp] * 5 + [_OUT_P, _vp]),
    "potr_batch_create": (_i32, [_JOB_P, _i32, _CFG_P, C.c_float, C.POINTER(_vp), _vp]),
    "potr_batch_workspace_size": (_i32, [_vp, C.POINTER(_sz)]),
    "potr_batch_pairs": (_i32, [_vp, C.POINTER(_i64), C.POINTER(_i64)]),
    "potr_batch_bind": (_i32, [_vp, _vp, _sz, _vp]),
    "potr_batch_run": (_i32, [_vp, _vp]),
    "potr_batch_render": (_i32, [_vp, _vp]),
    "potr_batch_capture": (_i32, [_vp, _vp]),
    "potr_batch_replay": (_i32, [_vp, _vp]),
    "potr_batch_overflow": (_i32, [_vp, C.POINTER(_i32), _vp]),
    "potr_batch_destroy": (_i32, [_vp]),
    "potr_prune_workspace_size": (_i32, [_i64, C.POINTER(_sz)]),
    "potr_prune_select": (_i32, [_i64, _vp, _vp, C.c_double, _i32, C.c_double, _vp, _sz, _vp, _vp, _vp]),
    "potr_sh_compact_workspace_size": (_i32, [_i64, _i32, C.POINTER(_sz)]),
    "potr_sh_compact": (_i32, [_i64, _i32, _CAM_P, _i32, _vp, _vp, _vp, _i64, C.c_double, C.c_double, C.c_double,
                               _vp, _sz, _vp, _vp]),
    "potr_codec_workspace_size": (_i32, [_i64, _i32, _i32, C.POINTER(_sz)]),
    "potr_codec_max_bytes": (_i32, [_i64, _i32, _i32, C.POINTER(_sz)]),
    "potr_codec_encode": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _i32, _CAM_P, _i32, _vp, _vp, _sz, _vp, _sz,
                                 C.POINTER(_sz), _vp, _vp]),
    "potr_codec_compress_bound": (_i32, [_sz, C.POINTER(_sz)]),
    "potr_codec_compress": (_i32, [_vp, _sz, _i32, _vp, _sz, C.POINTER(_sz)]),
    "potr_codec_decompressed_size": (_i32, [_vp, _sz, C.POINTER(_sz)]),
    "potr_codec_decompress": (_i32, [_vp, _sz, _vp, _sz, C.POINTER(_sz)]),
    "potr_codec_info": (_i32, [_vp, _sz, C.POINTER(_i64), C.POINTER(_i32)]),
    "potr_codec_decode": (_i32, [_vp, _sz, _vp, _vp, _vp, _vp, _vp]),
    "potr_fixed_to_float": (_i32, [_vp, _i64, _vp, _vp]),
    "potr_prune_select_noalloc": (_i32, [_i64, _vp, _vp, C.c_double, _i32, C.c_double, _vp, _vp, _vp]),
    "potr_prune_compact": (_i32, [_i64] + [_vp] * 7 + [_vp, _sz] + [_vp] * 7 + [_vp]),
    "potr_autotune": (_i32, [_JOB_P, _i32, _CFG_P, _i32, C.POINTER(C.c_double), _CFG_P, C.POINTER(C.c_double),
                             C.POINTER(_i32), _vp]),
}

_lib = None


class PotrError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed ({status}): {msg}")
        self.status = status


def lib():
    """Load libpotr.so (no fallback: a missing library is an error)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_2601_14821_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def call(name: str, *args) -> None:
    st = getattr(lib(), name)(*args)
    if st != POTR_OK:
        raise PotrError(name, st, lib().potr_last_error().decode())


def ptr(t) -> int | None:
    """Device pointer of a torch tensor (None for None)."""
    return None if t is None else t.data_ptr()


def stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def make_cameras(cams):
    arr = (potr_camera * len(cams))()
    for k, c in enumerate(cams):
        arr[k].R[:] = [float(x) for x in np.asarray(c.R, np.float32).reshape(-1)]
        arr[k].t[:] = [float(x) for x in np.asarray(c.t, np.float32).reshape(-1)]
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = c.fx, c.fy, c.cx, c.cy
        arr[k].width, arr[k].height = c.width, c.height
    return arr


def make_config(s) -> potr_config:
    c = potr_config()
    c.tile_w, c.tile_h, c.lds_batch = s.tile_w, s.tile_h, s.lds_batch
    c.eps2d, c.near_z, c.jclamp = s.eps2d, s.near, s.jclamp
    c.alpha_min, c.alpha_max, c.q_max, c.t_min = s.alpha_min, s.alpha_max, s.q_max, s.t_min
    c.bg[:] = [float(x) for x in s.bg]
    c.sh_degree = s.sh_degree
    return c


def make_outputs(o, v0: int = 0) -> potr_outputs:
    """potr_outputs for an `Outputs` description (raster.py), its arrays
    starting at view v0 of theirs."""
    c = potr_outputs()
    fixed = bool(getattr(o, "fixed_point", False))
    elem = 8 if fixed else 4
    for name, stride, weight in (("scores", "scores_stride", "scores_weight"), ("scores_se", "se_stride", "se_weight"),
                                 ("importance", "importance_stride", "importance_weight")):
        t = getattr(o, name)
        st = int(getattr(o, stride))
        if t is not None and t.element_size() != elem:
            raise ValueError(f"{name}: {'int64' if fixed else 'float32'} elements expected")
        setattr(c, name, None if t is None else t.data_ptr() + elem * v0 * st)
        setattr(c, stride, st)
        setattr(c, weight, float(getattr(o, weight)))
    c.fixed_point = 1 if fixed else 0
    return c


def bin_workspace_size(N: int, V: int, cams, cfg) -> int:
    """Bytes of the workspace potr_bin fills and potr_sort reads (cams: a
    make_cameras array, cfg: a potr_config)."""
    b = C.c_size_t(0)
    call("potr_bin_workspace_size", N, V, cams, C.byref(cfg), C.byref(b))
    return b.value


def sort_workspace_size(capacity: int) -> int:
    b = C.c_size_t(0)
    call("potr_sort_workspace_size", capacity, C.byref(b))
    return b.value
