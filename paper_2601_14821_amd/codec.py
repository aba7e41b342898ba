"""The codec of the paper (Sec. 4.5) over libpotr.so. Argument marshalling only.

    raw, order = codec.encode(ds, cams, codec.params(0.5))   # device model -> bytes
    comp = codec.compress(raw)                                # zstd
    model = codec.decode(codec.decompress(comp))             # host arrays, leaf order

The encoder's per-splat work (nearest camera eye, grid cell and Morton code, the
sort into leaf order, leaf depths, quantisation) runs on the device; the octree
bytes, zstd and the decoder run on the host inside the library.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


class potr_codec_params(C.Structure):
    _fields_ = [("beta", C.c_double), ("gamma", C.c_double), ("sf_scale", C.c_double), ("sf_rot", C.c_double),
                ("sf_opac", C.c_double), ("sf_sh", C.c_double), ("max_depth", C.c_int32), ("reserved", C.c_int32)]


def params(q: float = 0.5, max_depth: int = 21, **override) -> potr_codec_params:
    """The codec's hyperparameters at quality q (Sec. 5.1 table): beta = 1.4e-4 q,
    gamma = 5 10^(-3 - 5q), SF_scale = 1 + 4000 q, SF_rotation = 1 + 400 q,
    SF_opacity = 1 + 200 q, SF_SH = 1 + 100 q."""
    p = dict(beta=1.4e-4 * q, gamma=5.0 * 10.0 ** (-3.0 - 5.0 * q), sf_scale=1.0 + 4000.0 * q,
             sf_rot=1.0 + 400.0 * q, sf_opac=1.0 + 200.0 * q, sf_sh=1.0 + 100.0 * q, max_depth=max_depth)
    p.update(override)
    return potr_codec_params(**p, reserved=0)


def _u8(buf) -> C.c_void_p:
    return C.cast(buf, C.c_void_p)


def _src(data):
    """(pointer, length) of a bytes object or a uint8 numpy array."""
    if isinstance(data, np.ndarray):
        data = np.ascontiguousarray(data, np.uint8)
        return C.c_void_p(data.ctypes.data), data.nbytes, data
    return data, len(data), data


def encode(ds, cams, prm: potr_codec_params, sh_degree: int = 3, want_order: bool = False, ws=None):
    """potr_codec_encode: the uncompressed bitstream (a uint8 numpy array over
    pinned host memory) and, if asked, the input index of each coded splat
    (device int64 tensor)."""
    N = ds.n
    dev = ds.means.device
    cam = L.make_cameras(cams)
    b = C.c_size_t(0)
    L.call("potr_codec_workspace_size", N, sh_degree, len(cams), C.byref(b))
    if ws is None or ws.numel() < b.value:
        ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=dev)
    L.call("potr_codec_max_bytes", N, sh_degree, prm.max_depth, C.byref(b))
    # pinned host memory: the attribute streams leave the device in one DMA
    raw = torch.empty(b.value, dtype=torch.uint8, pin_memory=True)
    n = C.c_size_t(0)
    order = torch.empty(max(N, 1), dtype=torch.int32, device=dev)[:N] if want_order else None
    L.call("potr_codec_encode", N, L.ptr(ds.means), L.ptr(ds.scales), L.ptr(ds.quats), L.ptr(ds.opacities),
           L.ptr(ds.sh), sh_degree, cam, len(cams), C.byref(prm), L.ptr(ws), ws.numel(), raw.data_ptr(), b.value,
           C.byref(n), L.ptr(order) if order is not None else None, L.stream_handle())
    out = raw[: n.value].numpy()
    if want_order:
        return out, order.long()
    return out


def compress(raw, level: int = 3) -> bytes:
    """zstd of a bitstream (bytes or uint8 array)."""
    p, size, _keep = _src(raw)
    b = C.c_size_t(0)
    L.call("potr_codec_compress_bound", size, C.byref(b))
    out = (C.c_uint8 * b.value)()
    n = C.c_size_t(0)
    L.call("potr_codec_compress", p, size, level, _u8(out), b.value, C.byref(n))
    return bytes(memoryview(out)[: n.value])


def decompress(comp) -> bytes:
    p, size, _keep = _src(comp)
    b = C.c_size_t(0)
    L.call("potr_codec_decompressed_size", p, size, C.byref(b))
    out = (C.c_uint8 * max(b.value, 1))()
    n = C.c_size_t(0)
    L.call("potr_codec_decompress", p, size, _u8(out), b.value, C.byref(n))
    return bytes(memoryview(out)[: n.value])


def decode(raw) -> dict:
    """potr_codec_decode: the model as host arrays, splats in leaf order."""
    p, size, _keep = _src(raw)
    n = C.c_int64(0)
    deg = C.c_int32(0)
    L.call("potr_codec_info", p, size, C.byref(n), C.byref(deg))
    N = n.value
    out = dict(means=np.zeros((N, 3), np.float32), scales=np.zeros((N, 3), np.float32),
               quats=np.zeros((N, 4), np.float32), opacities=np.zeros(N, np.float32),
               sh=np.zeros((N, 16, 3), np.float32))
    L.call("potr_codec_decode", p, size, out["means"].ctypes.data, out["scales"].ctypes.data,
           out["quats"].ctypes.data, out["opacities"].ctypes.data, out["sh"].ctypes.data)
    out["sh_degree"] = deg.value
    return out
