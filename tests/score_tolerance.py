"""Per-splat score comparison against the oracle, shared by the GPU parity tests.

A splat passes when |s_gpu - s_ref| <= rtol |s_ref| + mfloor M_k + F_k: M_k is
the splat's term magnitude (the sum over its pixels of |c alpha T| + alpha/(1 - alpha)
(|P_K| + T_f |bg|), emitted by the oracle), so scores made of cancelling terms get
an FP32-sized absolute floor, and F_k is the oracle's allowance for pixels within a
relative 1e-5 of a threshold (whose decision FP32 may take the other way)."""
import numpy as np

import oracle


def compare_scores(sg, ref, mag, flag_mass, rtol=1e-3, mfloor=1e-5):
    """Assert every splat is within tolerance; return how many needed the flag allowance."""
    base = rtol * np.abs(ref) + mfloor * mag
    tol = base + flag_mass
    d = np.abs(sg.astype(np.float64) - ref)
    bad = d > tol
    assert not bad.any(), (f"{bad.sum()} splats out of tolerance; worst idx {np.argmax(d - tol)} "
                           f"gpu {sg[np.argmax(d - tol)]} ref {ref[np.argmax(d - tol)]}")
    return int((d > base).sum())


def oracle_views(scene, cams, s, target=None):
    """Oracle render of every view: per-view records and the per-splat sums over the views."""
    want = ("image", "score_l1", "importance", "magnitude", "flag_mass", "pixel_flag")
    if target is not None:
        want = want + ("score_se",)
    tot = {}
    views = []
    for v, cam in enumerate(cams):
        r = oracle.render(scene, cam, s, record_f32=True, want=want,
                          target=None if target is None else target[v])
        views.append(r)
        for k in ("score_l1", "importance", "magnitude", "flag_mass", "score_se"):
            if k in r:
                tot[k] = tot.get(k, 0.0) + r[k]
    return tot, views
