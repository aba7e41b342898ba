"""Per-splat score comparison against the oracle, shared by the GPU parity tests.

A splat passes when |s_gpu - s_ref| <= rtol |s_ref| + mfloor M_k + F_k: M_k is
the splat's term magnitude (the sum over its pixels of |c alpha T| + alpha/(1 - alpha)
(|P_K| + T_f |bg|), emitted by the oracle), so scores made of cancelling terms get
an FP32-sized absolute floor, and F_k is the oracle's allowance for pixels within a
relative 1e-5 of a threshold (whose decision FP32 may take the other way)."""
import numpy as np

import oracle


def compare_scores(sg, ref, mag, flag_mass, rtol=1e-3, mfloor=1e-5, stats=None, atol=0.0):
    """Assert every splat is within tolerance; return how many needed the flag
    allowance. With `stats` (a dict) also record, over the splats the oracle
    scores (ref != 0): how many there are, how many needed F_k, how many have
    F_k > 0.1 |s_ref| (for which the check pins little), how many are
    well conditioned (mfloor M_k <= rtol |s_ref|) and how many of those miss the
    plain relative bar rtol |s_ref| (and how many of all scored splats meet it).
    atol: an absolute floor (e.g. for sums of FP32 values below its normal range)."""
    base = rtol * np.abs(ref) + mfloor * mag + atol
    tol = base + flag_mass
    d = np.abs(sg.astype(np.float64) - ref)
    bad = d > tol
    assert not bad.any(), (f"{bad.sum()} splats out of tolerance; worst idx {np.argmax(d - tol)} "
                           f"gpu {sg[np.argmax(d - tol)]} ref {ref[np.argmax(d - tol)]}")
    if stats is not None:
        sc = ref != 0
        good = sc & (mfloor * mag <= rtol * np.abs(ref))
        stats.update(scored=int(sc.sum()), allowance=int((sc & (d > base)).sum()),
                     big_allowance=int((sc & (flag_mass > 0.1 * np.abs(ref))).sum()),
                     conditioned=int(good.sum()), conditioned_off=int((good & (d > rtol * np.abs(ref))).sum()),
                     strict=int((sc & (d <= rtol * np.abs(ref))).sum()))
    return int((d > base).sum())


def assert_allowance_is_rare(stats, use_frac=1e-3, big_frac=0.02, off_frac=1e-3, strict_frac=None):
    """The per-splat bar is carried by its tight terms: at most a thousandth of
    the scored splats need the flip allowance F_k at all, at most 2% have an
    allowance above a tenth of their score (a property of the oracle's bound),
    and at most a thousandth of the well-conditioned splats miss the plain
    relative bar. With strict_frac, at least that fraction of all scored splats
    meets the plain relative bar with neither the M_k floor nor F_k (production
    mode: the early stop keeps every blended T_k >= t_min, so the FP32
    cancellation floor rarely matters; in exact mode splats far down a list have
    scores below FP32's resolution of the colour still to come, and only the
    floor can carry them)."""
    n = max(stats["scored"], 1)
    if strict_frac is not None:
        assert stats["strict"] >= strict_frac * n, stats
    assert stats["allowance"] <= max(5, use_frac * n), stats
    assert stats["big_allowance"] <= max(2, big_frac * n), stats
    assert stats["conditioned_off"] <= max(2, off_frac * max(stats["conditioned"], 1)), stats


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
