"""Iterative pruning controller of the paper (Sec. 4.3) -- TEST INFRASTRUCTURE ONLY.

Plain numpy, FP64, written from the paper's rule; only `tests/` and the
CPU-baseline leg of `bench.py` may use it. It shares no code with the HIP path.

One pruning iteration, given every splat's dMSE_k and importance I_k (Sec. 4.1,
4.2) and the number of iterations still to run (this one included):
  * candidates are the splats with dMSE_k < dMSE_MAX (the controller's aim is to
    remove all of them over the iterations);
  * budget B = (1 / remaining) * sum of I_k over the candidates;
  * candidates are taken in ascending order of m(dMSE_k / dMSE_MAX), with
    m(x) = x for x >= 0 and (sqrt(1 - 2 a x) - 1) / a for x < 0 (a = 10),
    ties by splat index, each added to the removal set S until the budget is
    reached, B <= sum of I_k over S (so the splat that reaches it is removed,
    and nothing is removed when B = 0).

Readings where the paper is silent (the HIP path takes the same ones):
  * S is drawn from the candidates only: a splat with dMSE_k >= dMSE_MAX is
    never removed, even though a strongly negative dMSE can map above 1;
  * the budget arithmetic is exact: each I_k (given in FP32) is rounded to a
    multiple of 2^-52 (an integer Q_k), and the budget is reached at the first
    prefix whose integer sum reaches ceil(sum over candidates of Q_k / remaining),
    so that no summation order can move the cut; the inputs must be normalised
    (each I_k in [0, 1], their sum at most 2), as I_k is an image fraction;
  * x = dMSE_k / dMSE_MAX and m(x) are evaluated in FP64, each operation
    correctly rounded, in the order written above.
"""
from __future__ import annotations

import numpy as np

Q_BITS = 52


def mapping(x, a: float = 10.0):
    """m(x) of Sec. 4.3, elementwise in FP64."""
    x = np.asarray(x, np.float64)
    neg = (np.sqrt(1.0 - (2.0 * a) * np.minimum(x, 0.0)) - 1.0) / a
    return np.where(x >= 0.0, x, neg)


def quantise_importance(imp) -> np.ndarray:
    """Q_k = round-half-even(I_k * 2^52) as int64 (exact for FP32 inputs in [0, 1])."""
    q = np.rint(np.ldexp(np.asarray(imp, np.float32).astype(np.float64), Q_BITS))
    return q.astype(np.int64)


def select(dmse, importance, dmse_max: float, remaining: int, a: float = 10.0):
    """Splats removed by one iteration: a boolean mask over the splats.

    dmse, importance: FP32 arrays [N]; dmse_max > 0; remaining >= 1."""
    dmse = np.asarray(dmse, np.float32)
    imp = np.asarray(importance, np.float32)
    if remaining < 1 or not dmse_max > 0:
        raise ValueError("remaining >= 1 and dmse_max > 0")
    if imp.size and (np.any(~(imp >= 0)) or np.any(imp > 1)):
        raise ValueError("importance must lie in [0, 1]")
    n = dmse.size
    cand = dmse.astype(np.float64) < dmse_max
    q = quantise_importance(imp)
    total = int(q[cand].sum())
    if total > (2 << Q_BITS):
        raise ValueError("importance sums above 2: not normalised")
    remove = np.zeros(n, bool)
    if total == 0:
        return remove
    need = -(-total // int(remaining))            # ceil(total / remaining)
    idx = np.nonzero(cand)[0]
    keys = mapping(dmse[idx].astype(np.float64) / dmse_max, a)
    order = idx[np.argsort(keys, kind="stable")]  # ascending m, ties by index (idx is increasing)
    cum = np.cumsum(q[order])
    p = int(np.searchsorted(cum, need, side="left"))   # first prefix (0-based end) with sum >= need
    remove[order[: p + 1]] = True
    return remove


def select_by_walk(dmse, importance, dmse_max: float, remaining: int, a: float = 10.0):
    """The same rule as a literal walk (one splat at a time), for small inputs:
    used to check `select` itself."""
    dmse = [float(np.float32(d)) for d in dmse]
    imp = [float(np.float32(i)) for i in importance]
    cand = [k for k in range(len(dmse)) if dmse[k] < dmse_max]
    q = {k: int(round(imp[k] * 2.0 ** Q_BITS)) for k in cand}
    total = sum(q.values())
    budget_num = total                             # B = total / remaining, compared exactly
    key = {}
    for k in cand:
        x = dmse[k] / dmse_max
        key[k] = x if x >= 0 else (np.sqrt(1.0 - 2.0 * a * x) - 1.0) / a
    chosen, s = [], 0
    for k in sorted(cand, key=lambda k: (key[k], k)):
        if budget_num <= s * remaining:            # budget reached
            break
        chosen.append(k)
        s += q[k]
    out = np.zeros(len(dmse), bool)
    out[chosen] = True
    return out


def removal_statistics(scene, cams, s, targets, threads=None):
    """dMSE_k and I_k of every splat over the views (Sec. 4.1, 4.2), FP64 from
    the oracle's renders: dMSE_k = sum over views, pixels and channels of dSE_k
    / (3 V P), I_k = sum over views and pixels of T_k alpha_k / (V P)."""
    from . import render
    V = len(cams)
    P = cams[0].width * cams[0].height
    se = np.zeros(scene.n)
    imp = np.zeros(scene.n)
    for v, cam in enumerate(cams):
        r = render(scene, cam, s, target=targets[v], threads=threads, want=("score_se", "importance"))
        se += r["score_se"]
        imp += r["importance"]
    return se / (3.0 * V * P), imp / (V * P)


def run(scene, cams, s, n_iter: int, dmse_max: float, a: float = 10.0, targets=None, iterations=None):
    """The controller over `iterations` (default all n_iter) iterations: scores the
    survivors over all views against the targets (default: the oracle's render
    of the unpruned scene), removes one iteration's choice, and repeats.
    Returns the survivors' original indices after each iteration."""
    from . import render
    if targets is None:
        targets = [render(scene, cam, s, want=("image",))["image"].astype(np.float32) for cam in cams]
    alive = np.arange(scene.n)
    history = []
    for it in range(n_iter if iterations is None else iterations):
        sub = scene.subset(alive)
        dmse, imp = removal_statistics(sub, cams, s, targets)
        rm = select(dmse.astype(np.float32), imp.astype(np.float32), dmse_max, n_iter - it, a)
        alive = alive[~rm]
        history.append(alive.copy())
    return history
