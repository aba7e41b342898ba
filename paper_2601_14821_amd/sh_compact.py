"""Spherical-harmonics energy compaction (paper Sec. 4.4) over libpotr.so.

    imp = rz.removal_statistics(ds, cams, targets, per_view_importance=True)[2]   # I_k(s) [V, N]
    new_sh = sh_compact.compact(ds, cams, imp)

potr_sh_compact does all of it on the device: the importance-weighted Gram
matrix of every splat's SH basis over the cameras (FP64 matrix cores), the
column selection, the two ridge passes per YCoCg channel and the conversion
back to RGB.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _lib as L
from .raster import DeviceScene


def hyperparameters(q: float = 0.5) -> dict:
    """lambda = 10^-q and alpha = sigmoid(3 q) (Sec. 5.1, hyperparameter table);
    tau = 1 / (2 SF_SH) with SF_SH = 1 + 100 q, the half step of the SH quantiser."""
    return {"lam": 10.0 ** (-q), "alpha": 1.0 / (1.0 + math.exp(-3.0 * q)), "tau": 0.5 / (1.0 + 100.0 * q)}


def compact(ds: DeviceScene, cams, importance: torch.Tensor, degree: int = 3, lam: float | None = None,
            alpha: float | None = None, tau: float | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """New SH coefficients [N, 16, 3] for the splats of `ds` given the per-camera
    importance [V, N] (or [V, stride >= N])."""
    hp = hyperparameters()
    lam = hp["lam"] if lam is None else lam
    alpha = hp["alpha"] if alpha is None else alpha
    tau = hp["tau"] if tau is None else tau
    N, V = ds.n, len(cams)
    if importance.dim() != 2 or importance.shape[0] != V:
        raise ValueError("importance must be [V, N]")
    stride = importance.stride(0)
    b = C.c_size_t(0)
    L.call("potr_sh_compact_workspace_size", N, V, C.byref(b))
    ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=ds.means.device)
    if out is None:
        out = torch.empty_like(ds.sh)
    L.call("potr_sh_compact", N, V, L.make_cameras(cams), degree, L.ptr(ds.means), L.ptr(ds.sh), L.ptr(importance),
           stride, float(lam), float(alpha), float(tau), L.ptr(ws), ws.numel(), L.ptr(out), L.stream_handle())
    return out
