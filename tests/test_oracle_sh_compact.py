"""Pins of the oracle's SH energy compaction (Sec. 4.4) on the CPU: closed
forms, an independent least-squares solve of the ridge problem, the colour
model, the importance weighting, the sparsity rule and the two passes."""
import math

import numpy as np
import pytest

from oracle import sh_compact as shc
from paper_2601_14821_amd import synth


def _eyes(n, seed, r=3.0):
    """Camera centres spread over the sphere around the origin."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    return r * v / np.linalg.norm(v, axis=1, keepdims=True)


def _coeffs(seed, scale_ac=0.3):
    rng = np.random.default_rng(seed)
    L = rng.normal(0, scale_ac, (16, 3))
    L[0] = rng.normal(0, 1.0, 3)
    return L


def test_hyperparameters_of_the_table():
    hp = shc.hyperparameters(0.5)
    assert hp["lam"] == 10 ** -0.5
    assert abs(hp["alpha"] - 1 / (1 + math.exp(-1.5))) < 1e-16
    assert hp["tau"] == 0.5 / 51.0


def test_colour_model_matrices_are_inverse():
    np.testing.assert_array_equal(shc.RGB_TO_YCOCG @ shc.YCOCG_TO_RGB, np.eye(3))
    # grey is pure luminance
    np.testing.assert_array_equal(shc.RGB_TO_YCOCG @ np.ones(3), [1.0, 0.0, 0.0])


def test_no_regularisation_reproduces_the_coefficients():
    """With many spread cameras, lambda = 0, no sparsity (alpha > 1) and tau = 0,
    the fit of C = Y L returns L."""
    L = _coeffs(1)
    eyes = _eyes(40, 2)
    out = shc.compact_splat(L, [0.1, -0.2, 0.05], eyes, np.ones(40), 3, lam=0.0, alpha=1.1, tau=0.0)
    np.testing.assert_allclose(out, L, atol=1e-10)


def test_one_camera_keeps_only_the_dc_and_its_colour():
    """One camera: every column is a single number, so every AC column is
    parallel to the DC one and dropped; the DC is then C(d) / Y_0 = 2 sqrt(pi) C(d)."""
    L = _coeffs(3)
    mu = np.array([0.3, 0.1, -0.4])
    eye = np.array([[2.0, 1.0, 3.0]])
    out = shc.compact_splat(L, mu, eye, [0.7], 3, lam=0.3, alpha=0.8, tau=0.01)
    Y = shc.basis_matrix(mu, eye, 3)
    colour = (Y @ L)[0]
    np.testing.assert_allclose(out[0], 2.0 * math.sqrt(math.pi) * colour, rtol=1e-13)
    assert not out[1:].any()


def test_ridge_equals_augmented_least_squares():
    """The closed form (Y^T Y + G^T G)^-1 Y^T C against numpy's least squares on
    the stacked system [Y; G] x = [C; 0] (an SVD, not the normal equations)."""
    rng = np.random.default_rng(4)
    Yw = rng.normal(size=(25, 16))
    c = rng.normal(size=25)
    cols = [0, 1, 3, 4, 7, 9, 15]
    for lam in (0.3, 3.0, 1e-3):
        x = shc.ridge(Yw, c, cols, lam)
        G = np.diag([0.0 if i == 0 else math.sqrt(lam) for i in cols])
        ref = np.linalg.lstsq(np.vstack([Yw[:, cols], G]), np.concatenate([c, np.zeros(len(cols))]), rcond=None)[0]
        np.testing.assert_allclose(x[cols], ref, rtol=1e-10, atol=1e-12)
        assert not np.delete(x, cols).any()


def test_channels_regularised_as_the_colour_model_says():
    """A grey splat stays grey (no chrominance); a splat with only Co content is
    fitted with 3 lambda, a luminance-only one with lambda."""
    eyes = _eyes(12, 5)
    mu = np.zeros(3)
    Y = shc.basis_matrix(mu, eyes, 3)
    w = np.linspace(0.2, 1.0, 12)
    grey = np.repeat(_coeffs(6)[:, :1], 3, axis=1)
    out = shc.compact_splat(grey, mu, eyes, w, 3, lam=0.3, alpha=1.1, tau=0.0)
    np.testing.assert_allclose(out[:, 0], out[:, 1], atol=1e-14)
    np.testing.assert_allclose(out[:, 0], out[:, 2], atol=1e-14)
    # luminance-only coefficients: the Y channel fit with lambda
    ref = shc.ridge(w[:, None] * Y, w * (Y @ grey[:, 0]), list(range(16)), 0.3)
    np.testing.assert_allclose(out[:, 0], ref, atol=1e-13)
    # Co-only coefficients (R = -B = x, G = 0): fit with 3 lambda
    x = _coeffs(7)[:, 0]
    co = np.stack([x, np.zeros(16), -x], axis=1)
    out = shc.compact_splat(co, mu, eyes, w, 3, lam=0.3, alpha=1.1, tau=0.0)
    # Co of the input is (R - B)/2 = x
    ref = shc.ridge(w[:, None] * Y, w * (Y @ x), list(range(16)), 0.9)
    np.testing.assert_allclose(out[:, 0], ref, atol=1e-13)        # R = Y + Co - Cg = Co
    np.testing.assert_allclose(out[:, 2], -ref, atol=1e-13)
    np.testing.assert_allclose(out[:, 1], 0.0, atol=1e-14)


def test_importance_weighting():
    """A camera of zero importance changes nothing; scaling every importance by
    a constant changes nothing; the weighted fit equals the ridge of the
    row-scaled system."""
    L = _coeffs(8)
    mu = np.array([0.2, 0.3, 0.1])
    eyes = _eyes(10, 9)
    w = np.random.default_rng(10).uniform(0.1, 1.0, 10)
    base = shc.compact_splat(L, mu, eyes, w, 3, lam=0.3, alpha=0.8, tau=0.01)
    extra = np.vstack([eyes, [[0.0, 5.0, 0.0]]])
    np.testing.assert_allclose(shc.compact_splat(L, mu, extra, np.append(w, 0.0), 3, lam=0.3, alpha=0.8, tau=0.01),
                               base, atol=1e-13)
    np.testing.assert_allclose(shc.compact_splat(L, mu, eyes, 7.5 * w, 3, lam=0.3, alpha=0.8, tau=0.01), base,
                               atol=1e-13)


def test_sparsity_drops_parallel_columns():
    """Cameras on a circle in the plane z = mu_z see no z-dependence: Y_2 (~ z) is
    a zero column and dropped; with alpha > 1 nothing else is dropped."""
    mu = np.array([0.0, 0.0, 0.5])
    ang = np.linspace(0, 2 * np.pi, 9)[:-1]
    eyes = np.stack([3 * np.cos(ang), 3 * np.sin(ang), np.full(8, 0.5)], axis=1)
    L = _coeffs(11)
    out = shc.compact_splat(L, mu, eyes, np.ones(8), 1, lam=0.1, alpha=1.1, tau=0.0)
    assert not out[2].any()                      # the z column is gone
    assert out[1].any() and out[3].any()
    # degree 2 on the circle: Y_6 ~ (2 z^2 - x^2 - y^2) = -1 is parallel to the DC column
    out = shc.compact_splat(_coeffs(12), mu, eyes, np.ones(8), 2, lam=0.1, alpha=0.999, tau=0.0)
    assert not out[6].any() and not out[2].any()
    assert not out[9:].any()                     # beyond the degree in use


def test_two_passes_zero_small_coefficients_and_refit():
    L = _coeffs(13)
    L[5] = [2e-3, 2e-3, 2e-3]                     # a grey coefficient the first pass leaves tiny
    mu = np.array([0.1, 0.0, -0.2])
    eyes = _eyes(30, 14)
    w = np.random.default_rng(15).uniform(0.2, 1.0, 30)
    tau, lam = 0.02, 0.005
    out, margin = shc.compact_splat(L, mu, eyes, w, 3, lam=lam, alpha=1.1, tau=tau, with_margins=True)
    assert margin > 1e-3
    assert not out[5].any()
    # the output is the ridge fit over the columns that survived, channel by channel
    # (rows weighted by the importances over their largest)
    w = w / w.max()
    Y = shc.basis_matrix(mu, eyes, 3)
    Cy = (Y @ L) @ shc.RGB_TO_YCOCG.T
    first = [shc.ridge(w[:, None] * Y, w * Cy[:, ch], list(range(16)), lc)
             for ch, lc in enumerate((lam, 3 * lam, 3 * lam))]
    res = np.zeros((16, 3))
    for ch, lc in enumerate((lam, 3 * lam, 3 * lam)):
        cols = [0] + [i for i in range(1, 16) if abs(first[ch][i]) >= tau]
        assert 5 not in cols
        res[:, ch] = shc.ridge(w[:, None] * Y, w * Cy[:, ch], cols, lc)
    np.testing.assert_allclose(out, res @ shc.YCOCG_TO_RGB.T, atol=1e-13)


def test_degenerate_splats():
    L = _coeffs(16)
    # nothing sees it: DC kept, AC dropped
    out = shc.compact_splat(L, np.zeros(3), _eyes(4, 17), np.zeros(4), 3, 0.3, 0.8, 0.01)
    np.testing.assert_array_equal(out[0], L[0])
    assert not out[1:].any()
    # degree 0: the DC is the colour's only coefficient and is reproduced
    out = shc.compact_splat(L, np.zeros(3), _eyes(4, 18), np.ones(4), 0, 0.3, 0.8, 0.01)
    np.testing.assert_allclose(out[0], L[0], rtol=1e-14)
    assert not out[1:].any()


def test_scene_driver_matches_per_splat_calls():
    scene = synth.random_scene(20, 19)
    cams = synth.hemisphere_cameras(6, 64, 48, seed=20)
    imp = np.random.default_rng(21).uniform(0, 1e-3, (6, 20))
    out = shc.compact(scene, cams, imp, idx=[3, 7])
    eyes = np.array([c.eye for c in cams])
    hp = shc.hyperparameters()
    np.testing.assert_array_equal(out[1], shc.compact_splat(scene.sh[7], scene.means[7], eyes, imp[:, 7], 3,
                                                            hp["lam"], hp["alpha"], hp["tau"]))
