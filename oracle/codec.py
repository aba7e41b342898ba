"""The codec of the paper (Sec. 4.5) -- TEST INFRASTRUCTURE ONLY.

Plain numpy and Python, FP64, written from the paper's description; only
`tests/` may use it. It shares no code with the HIP path. The octree is built
by literal recursive splitting (pure Python over the nodes: small inputs only).

What the codec computes (Sec. 4.5, hyperparameters from the table of Sec. 5.1):
  * attributes are quantised uniformly, x_hat = floor(1/2 + x SF), and
    dequantised as x_hat / SF; opacity is dequantised off-centre as
    (x_hat + 1/4) / SF; every attribute has its own scale factor SF;
  * DC lighting coefficients are coded differentially, and the real quaternion
    component is left out (recomputed from unit norm);
  * positions go to the centre of an octree leaf; a leaf is split while it
    holds more than one splat or its one splat misses the precision test
    |mu - centre| < max(gamma, beta * min over training cameras s of |mu - eye_s|);
  * the octree is written depth first: on its first visit every node appends
    one occupancy byte (bit c set when octant c has a child node);
  * attributes follow in the leaf order of that traversal, one property after
    another over all splats; the stream is then compressed with zstd.

Readings where the paper is silent (the HIP path takes the same ones):
  * the root is the cube [lo, lo + size)^3 with lo the per-axis minimum of the
    positions and size = (largest per-axis extent) * (1 + 2^-20) (1 when all
    positions coincide); positions are placed on a 2^D grid, X = floor((mu -
    lo) * (2^D / size)) per axis (FP64, clamped to [0, 2^D)), and a node at
    depth L is a cube of the grid cells sharing the top L bits; octant
    c = x_bit | y_bit << 1 | z_bit << 2 of the next bit, children in increasing
    c; at the depth cap D (21 by default) nodes are leaves whatever they hold,
    and such a leaf's splat count is stored (a u32 per leaf at depth D);
  * a node's centre is lo + (cell + 1/2) * (size * 2^-L) per axis, and the test
    is taken on squares: ((dx dx + dy dy) + dz dz) < max(gamma^2, beta^2 * d2min),
    d2min the smallest squared distance to a camera eye (eye = -R^T t), every
    operation correctly rounded in the order written;
  * quantised attributes are the activated scales and opacity of the model, the
    unit quaternion (w, x, y, z) / |q| with w >= 0 (x, y, z kept; a zero
    quaternion counts as the identity), and every SH coefficient with SF_SH;
    the decoder takes w = sqrt(max(0, 1 - (x^2 + y^2 + z^2)));
  * the DC difference of a splat is taken against the previous splat in leaf
    order (the first against zero), on the quantised integers; splats sharing
    a leaf at the depth cap keep their index order;
  * layout, little-endian: header (magic, version, N, D, SH degree, lo, size,
    the four scale factors, node and cap-leaf counts), the node bytes, the
    cap-leaf counts, then int32 streams of N values each: opacity; scale x, y,
    z; rotation x, y, z; SH coefficient j channel r, g, b for j = 0 .. (DEG+1)^2
    - 1 (j = 0 as differences). The decoded model lists the splats in leaf order.
"""
from __future__ import annotations

import ctypes
import struct

import numpy as np

MAGIC = 0x52544F50   # "POTR"
VERSION = 1
HEADER = struct.Struct("<IIQIIddddddddQQ")


def params(q: float, max_depth: int = 21) -> dict:
    """The hyperparameters of the codec as functions of the quality q (Sec. 5.1 table)."""
    return dict(beta=1.4e-4 * q, gamma=5.0 * 10.0 ** (-3.0 - 5.0 * q), sf_scale=1.0 + 4000.0 * q,
                sf_rot=1.0 + 400.0 * q, sf_opac=1.0 + 200.0 * q, sf_sh=1.0 + 100.0 * q, max_depth=max_depth)


def quantise(x, sf: float) -> np.ndarray:
    """x_hat = floor(1/2 + x SF) in FP64 (x in FP32)."""
    return np.floor(0.5 + np.asarray(x, np.float32).astype(np.float64) * sf).astype(np.int64)


def dequantise(xq, sf: float, offset: float = 0.0) -> np.ndarray:
    return (np.asarray(xq, np.int64).astype(np.float64) + offset) / sf


def camera_eyes(cams) -> np.ndarray:
    """eye = -R^T t for each camera (FP64)."""
    out = []
    for c in cams:
        R = np.asarray(c.R, np.float32).astype(np.float64).reshape(3, 3)
        t = np.asarray(c.t, np.float32).astype(np.float64)
        out.append([-(R[0, k] * t[0] + R[1, k] * t[1] + R[2, k] * t[2]) for k in range(3)])
    return np.array(out, np.float64).reshape(-1, 3)


def nearest_eye_d2(means, eyes) -> np.ndarray:
    """Smallest squared distance from each position to a camera eye, ((dx dx + dy dy) + dz dz)."""
    m = np.asarray(means, np.float32).astype(np.float64)
    best = np.full(m.shape[0], np.inf)
    for e in eyes:
        d = m - e
        best = np.minimum(best, (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    return best


def grid(means, D: int):
    """The root cube (lo, size) and each position's grid cell X, Y, Z (int64, D bits)."""
    m = np.asarray(means, np.float32).astype(np.float64)
    if m.shape[0] == 0:
        return np.zeros(3), 1.0, np.zeros((0, 3), np.int64)
    lo = m.min(axis=0)
    ext = float((m.max(axis=0) - lo).max())
    size = ext * (1.0 + 2.0 ** -20) if ext > 0 else 1.0
    scale = float(2 ** D) / size
    cell = np.floor((m - lo) * scale)
    cell = np.clip(cell, 0, 2 ** D - 1).astype(np.int64)
    return lo, size, cell


def _node_centre(lo, size, node_cell, depth):
    """Centre of a node from its coordinates at its own depth (the top `depth` bits of the cells)."""
    step = size * 2.0 ** -depth
    return lo + (np.asarray(node_cell, np.float64) + 0.5) * step


def build_octree(means, thr2, D: int):
    """Recursive splitting (Sec. 4.5): returns (node bytes, cap-leaf counts, leaf
    order of the splats, each splat's leaf depth and leaf cell at that depth),
    plus lo and size of the root."""
    lo, size, X = grid(means, D)
    m = np.asarray(means, np.float32).astype(np.float64)
    n = m.shape[0]
    nodes = bytearray()
    caps: list[int] = []
    order: list[int] = []
    depth_of = np.zeros(n, np.int64)
    cell_of = np.zeros((n, 3), np.int64)
    if n == 0:
        return bytes(nodes), caps, np.zeros(0, np.int64), depth_of, cell_of, lo, size

    def visit(idx, depth, node_cell):
        if depth < D and idx.size == 1:
            i = int(idx[0])
            c = _node_centre(lo, size, node_cell, depth)
            d = m[i] - c
            d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
            if d2 < thr2[i]:
                nodes.append(0)
                order.append(i)
                depth_of[i] = depth
                cell_of[i] = node_cell
                return
        if depth == D:
            nodes.append(0)
            caps.append(int(idx.size))
            order.extend(int(i) for i in idx)
            depth_of[idx] = D
            cell_of[idx] = node_cell
            return
        shift = D - depth - 1
        bits = (X[idx] >> shift) & 1
        octant = bits[:, 0] | (bits[:, 1] << 1) | (bits[:, 2] << 2)
        occ = 0
        for c in range(8):
            if np.any(octant == c):
                occ |= 1 << c
        nodes.append(occ)
        for c in range(8):
            sub = idx[octant == c]
            if sub.size:
                child = np.array([2 * node_cell[0] + (c & 1), 2 * node_cell[1] + ((c >> 1) & 1),
                                  2 * node_cell[2] + ((c >> 2) & 1)], np.int64)
                visit(sub, depth + 1, child)

    visit(np.arange(n, dtype=np.int64), 0, np.zeros(3, np.int64))
    return bytes(nodes), caps, np.array(order, np.int64), depth_of, cell_of, lo, size


def parse_octree(nodes: bytes, caps, D: int, lo, size):
    """Decoder side: the leaf centres (FP64 [N, 3]) in traversal order and each
    leaf's depth, read back from the node bytes."""
    out, depths = [], []
    pos = 0
    ci = 0

    def visit(depth, node_cell):
        nonlocal pos, ci
        b = nodes[pos]
        pos += 1
        if b == 0:
            count = 1
            if depth == D:
                count = caps[ci]
                ci += 1
            c = _node_centre(lo, size, node_cell, depth)
            for _ in range(count):
                out.append(c)
                depths.append(depth)
            return
        for c in range(8):
            if b >> c & 1:
                visit(depth + 1, (2 * node_cell[0] + (c & 1), 2 * node_cell[1] + ((c >> 1) & 1),
                                  2 * node_cell[2] + ((c >> 2) & 1)))

    if len(nodes):
        visit(0, (0, 0, 0))
    if pos != len(nodes) or ci != len(caps):
        raise ValueError("node bytes or cap counts left over")
    return np.array(out, np.float64).reshape(-1, 3), np.array(depths, np.int64)


def unit_quat(quats) -> np.ndarray:
    """(w, x, y, z) / |q| in FP64 with w >= 0; a zero quaternion is the identity."""
    q = np.asarray(quats, np.float32).astype(np.float64)
    n2 = ((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]) + q[:, 3] * q[:, 3]
    nrm = np.sqrt(n2)
    zero = n2 == 0
    u = q / np.where(zero, 1.0, nrm)[:, None]
    u[zero] = [1.0, 0.0, 0.0, 0.0]
    u[u[:, 0] < 0] *= -1.0
    return u


def encode_raw(scene, cams, prm: dict) -> tuple[bytes, dict]:
    """The uncompressed bitstream of Sec. 4.5 and what went into it."""
    D = int(prm["max_depth"])
    N = scene.n
    nsh = scene.sh.shape[1]
    deg = int(round(np.sqrt(nsh))) - 1
    eyes = camera_eyes(cams)
    d2 = nearest_eye_d2(scene.means, eyes)
    thr2 = np.maximum(prm["gamma"] * prm["gamma"], (prm["beta"] * prm["beta"]) * d2)
    nodes, caps, order, depth_of, cell_of, lo, size = build_octree(scene.means, thr2, D)
    sf = (prm["sf_scale"], prm["sf_rot"], prm["sf_opac"], prm["sf_sh"])
    streams = [quantise(scene.opacities[order], prm["sf_opac"])]
    for a in range(3):
        streams.append(quantise(scene.scales[order, a], prm["sf_scale"]))
    u = unit_quat(scene.quats)[order]
    for a in range(1, 4):
        streams.append(np.floor(0.5 + u[:, a] * prm["sf_rot"]).astype(np.int64))
    sh = np.asarray(scene.sh, np.float32)[order]          # [N, nsh, 3]
    for j in range(nsh):
        for ch in range(3):
            qv = quantise(sh[:, j, ch], prm["sf_sh"])
            if j == 0:
                qv = np.diff(qv, prepend=0)
            streams.append(qv)
    head = HEADER.pack(MAGIC, VERSION, N, D, deg, float(lo[0]), float(lo[1]), float(lo[2]), float(size),
                       *[float(x) for x in sf], len(nodes), len(caps))
    body = [head, nodes, np.asarray(caps, "<u4").tobytes()]
    for s in streams:
        if s.size and (s.min() < -2 ** 31 or s.max() >= 2 ** 31):
            raise ValueError("quantised value out of int32 range")
        body.append(s.astype("<i4").tobytes())
    info = dict(order=order, depth=depth_of, cell=cell_of, lo=lo, size=size, thr2=thr2, nodes=nodes, caps=caps)
    return b"".join(body), info


def decode_raw(raw: bytes) -> dict:
    """The model back from the uncompressed bitstream, splats in leaf order (FP32)."""
    (magic, ver, N, D, deg, lx, ly, lz, size, sf_scale, sf_rot, sf_opac, sf_sh, n_nodes, n_caps) = \
        HEADER.unpack_from(raw, 0)
    if magic != MAGIC or ver != VERSION:
        raise ValueError("not a bitstream of this codec")
    p = HEADER.size
    nodes = raw[p:p + n_nodes]
    p += n_nodes
    caps = np.frombuffer(raw, "<u4", n_caps, p).astype(np.int64).tolist()
    p += 4 * n_caps
    nsh = (deg + 1) ** 2
    st = np.frombuffer(raw, "<i4", (7 + 3 * nsh) * N, p).astype(np.int64).reshape(7 + 3 * nsh, N)
    lo = np.array([lx, ly, lz])
    pos, _ = parse_octree(nodes, caps, D, lo, size)
    if pos.shape[0] != N:
        raise ValueError("leaf count differs from N")
    out = dict(means=pos.astype(np.float32))
    out["opacities"] = dequantise(st[0], sf_opac, 0.25).astype(np.float32)
    out["scales"] = np.stack([dequantise(st[1 + a], sf_scale) for a in range(3)], 1).astype(np.float32)
    xyz = np.stack([dequantise(st[4 + a], sf_rot) for a in range(3)], 1)
    n2 = (xyz[:, 0] * xyz[:, 0] + xyz[:, 1] * xyz[:, 1]) + xyz[:, 2] * xyz[:, 2]
    w = np.sqrt(np.maximum(0.0, 1.0 - n2))
    out["quats"] = np.concatenate([w[:, None], xyz], 1).astype(np.float32)
    sh = np.zeros((N, nsh, 3))
    for j in range(nsh):
        for ch in range(3):
            qv = st[7 + 3 * j + ch]
            if j == 0:
                qv = np.cumsum(qv)
            sh[:, j, ch] = dequantise(qv, sf_sh)
    out["sh"] = sh.astype(np.float32)
    out["D"] = D
    out["sh_degree"] = deg
    return out


# ---- zstd (the system's libzstd, a library step of the codec)
_zstd = None


def _lib():
    global _zstd
    if _zstd is None:
        z = ctypes.CDLL("libzstd.so.1")
        z.ZSTD_compressBound.restype = ctypes.c_size_t
        z.ZSTD_compressBound.argtypes = [ctypes.c_size_t]
        z.ZSTD_compress.restype = ctypes.c_size_t
        z.ZSTD_compress.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        z.ZSTD_decompress.restype = ctypes.c_size_t
        z.ZSTD_decompress.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t]
        z.ZSTD_isError.restype = ctypes.c_uint
        z.ZSTD_isError.argtypes = [ctypes.c_size_t]
        z.ZSTD_getFrameContentSize.restype = ctypes.c_ulonglong
        z.ZSTD_getFrameContentSize.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
        _zstd = z
    return _zstd


def zstd_compress(raw: bytes, level: int = 3) -> bytes:
    z = _lib()
    cap = z.ZSTD_compressBound(len(raw))
    out = ctypes.create_string_buffer(cap)
    n = z.ZSTD_compress(out, cap, raw, len(raw), level)
    if z.ZSTD_isError(n):
        raise RuntimeError("zstd compression failed")
    return out.raw[:n]


def zstd_decompress(comp: bytes) -> bytes:
    z = _lib()
    size = z.ZSTD_getFrameContentSize(comp, len(comp))
    if size >= 2 ** 63:
        raise RuntimeError("zstd frame without a content size")
    out = ctypes.create_string_buffer(max(int(size), 1))
    n = z.ZSTD_decompress(out, int(size), comp, len(comp))
    if z.ZSTD_isError(n) or n != size:
        raise RuntimeError("zstd decompression failed")
    return out.raw[:n]
