"""Spherical-harmonics energy compaction of the paper (Sec. 4.4) -- TEST INFRASTRUCTURE ONLY.

Plain numpy, FP64, one splat at a time, in the paper's order; only `tests/` and
the CPU-baseline leg of `bench.py` may use it. The SH basis is the oracle's own
(associated-Legendre recurrences in potr_oracle.c). It shares no code with the
HIP path.

For one splat with coefficients L (M x 3, RGB) and the training cameras s:
  1. the colour each camera sees, C(d_s) = sum_i L_i Y_i(d_s), d_s the unit
     vector from the camera centre to the splat centre (Sec. 3): C = Y L;
  2. luminance-chrominance: L and C in YCoCg (Y = R/4 + G/2 + B/4,
     Co = R/2 - B/2, Cg = -R/4 + G/2 - B/4);
  3. importance: every row of Y and C multiplied by the camera's weight w_s;
  4. sparsity: an AC column of the weighted Y is zeroed (its coefficient is 0)
     when the absolute cosine between it and a preceding column that is kept
     exceeds alpha;
  5. ridge regression per channel, L' = (Y^T Y + G^T G)^(-1) Y^T C with
     G = sqrt(lambda_c) diag(0, 1, ..., 1) over the kept columns, lambda_Y =
     lambda, lambda_Co = lambda_Cg = 3 lambda;
  6. two passes: AC coefficients of the first solution with |L'_i| < tau are
     forced to zero and the ridge problem is solved again over the rest;
  7. back to RGB (R = Y + Co - Cg, G = Y + Cg, B = Y - Co - Cg).

Readings where the paper is silent (the HIP path takes the same ones):
  * the colour is the raw SH sum (before the 1/2 offset and the clamp at 0 of
    the renderer), which the paper's linear system states;
  * the camera weights are the per-camera importances I_k(s) divided by the
    splat's largest one (the paper's substitution multiplies rows by I_k(s);
    rescaling them by a per-splat constant keeps the fit's weighting but gives
    lambda a scale that does not depend on how much of an image the splat fills);
  * DC is always kept; a column of zero norm counts as parallel (dropped);
    columns are visited in index order and compared with the kept ones before them;
  * "almost zero" is |L'_i| < tau with tau = 1/(2 SF_SH), the half step of the
    SH quantiser of Sec. 4.5 (SF_SH = 1 + 100 q), i.e. coefficients that the
    codec would quantise to zero;
  * a splat no camera sees (all weights 0) keeps its DC and loses its AC;
  * coefficients beyond the degree in use are set to 0.
"""
from __future__ import annotations

import math

import numpy as np

RGB_TO_YCOCG = np.array([[0.25, 0.5, 0.25], [0.5, 0.0, -0.5], [-0.25, 0.5, -0.25]])
YCOCG_TO_RGB = np.array([[1.0, 1.0, -1.0], [1.0, 0.0, 1.0], [1.0, -1.0, -1.0]])


def hyperparameters(q: float = 0.5) -> dict:
    """lambda = 10^-q, alpha = sigmoid(3 q), SF_SH = 1 + 100 q (hyperparameter table, Sec. 5.1)."""
    sf = 1.0 + 100.0 * q
    return {"lam": 10.0 ** (-q), "alpha": 1.0 / (1.0 + math.exp(-3.0 * q)), "tau": 0.5 / sf}


def basis_matrix(mu, eyes, degree: int) -> np.ndarray:
    """Y [V, M]: the basis at the unit directions from each eye to mu."""
    from . import sh_basis
    M = (degree + 1) ** 2
    rows = []
    for e in np.asarray(eyes, np.float64):
        d = np.asarray(mu, np.float64) - e
        d = d / np.linalg.norm(d)
        rows.append(sh_basis(3, d)[:M])
    return np.array(rows).reshape(-1, M)


def ridge(Yw, c, cols, lam):
    """Minimiser over x (zero outside `cols`) of |Yw x - c|^2 + lam |x_AC|^2 (the
    closed form of Sec. 4.4 on the kept columns)."""
    M = Yw.shape[1]
    x = np.zeros(M)
    if not cols:
        return x
    A = Yw[:, cols]
    reg = np.diag([0.0 if i == 0 else lam for i in cols])
    x[cols] = np.linalg.solve(A.T @ A + reg, A.T @ c)
    return x


def compact_splat(L_rgb, mu, eyes, importance, degree: int, lam: float, alpha: float, tau: float,
                  with_margins: bool = False):
    """New coefficients [16, 3] (RGB) of one splat; with_margins also returns the
    smallest relative distance of any of its decisions (cosine vs alpha,
    |L'| vs tau) from its threshold."""
    L_rgb = np.asarray(L_rgb, np.float64).reshape(16, 3)
    M = (degree + 1) ** 2
    out = np.zeros((16, 3))
    imp = np.asarray(importance, np.float64)
    margin = math.inf
    if not imp.size or imp.max() <= 0.0:
        out[0] = L_rgb[0]
        return (out, margin) if with_margins else out
    Y = basis_matrix(mu, eyes, degree)
    C = Y @ L_rgb[:M]                                  # 1. colours per camera
    Cy = C @ RGB_TO_YCOCG.T                            # 2. YCoCg
    w = imp / imp.max()                                # 3. importance weights
    Yw = w[:, None] * Y
    Cw = w[:, None] * Cy
    kept = [0]                                         # 4. sparsity
    norms = np.linalg.norm(Yw, axis=0)
    for i in range(1, M):
        if norms[i] == 0.0:
            continue
        cos = [abs(Yw[:, j] @ Yw[:, i]) / (norms[j] * norms[i]) for j in kept]
        margin = min(margin, min(abs(c - alpha) / alpha for c in cos)) if alpha <= 1.0 else margin
        if max(cos) <= alpha:
            kept.append(i)
    res = np.zeros((M, 3))
    for ch, lc in enumerate((lam, 3.0 * lam, 3.0 * lam)):
        first = ridge(Yw, Cw[:, ch], kept, lc)         # 5. first pass
        keep2 = [i for i in kept if i == 0 or abs(first[i]) >= tau]
        if tau > 0.0:
            for i in kept[1:]:
                margin = min(margin, abs(abs(first[i]) - tau) / tau)
        res[:, ch] = ridge(Yw, Cw[:, ch], keep2, lc)   # 6. second pass
    out[:M] = res @ YCOCG_TO_RGB.T                     # 7. back to RGB
    return (out, margin) if with_margins else out


def compact(scene, cams, importance, degree: int = 3, lam: float | None = None, alpha: float | None = None,
            tau: float | None = None, idx=None, with_margins: bool = False):
    """compact_splat over the splats `idx` (default all) of a scene; importance
    [V, N] per camera. Returns the new SH array [len(idx), 16, 3] (and margins)."""
    hp = hyperparameters()
    lam = hp["lam"] if lam is None else lam
    alpha = hp["alpha"] if alpha is None else alpha
    tau = hp["tau"] if tau is None else tau
    eyes = np.array([c.eye for c in cams])
    idx = np.arange(scene.n) if idx is None else np.asarray(idx)
    imp = np.asarray(importance, np.float64)
    outs, margins = [], []
    for k in idx:
        o, m = compact_splat(scene.sh[k], scene.means[k], eyes, imp[:, k], degree, lam, alpha, tau, True)
        outs.append(o)
        margins.append(m)
    outs = np.array(outs).reshape(len(idx), 16, 3)
    return (outs, np.array(margins)) if with_margins else outs
