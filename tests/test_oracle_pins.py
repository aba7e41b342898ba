"""Pins of the FP64 oracle against facts fixed outside its own code.

Each test ties one part of the oracle to something independent of it: a
hand-worked example (tests/golden), a closed form, an invariant of alpha
compositing (Sec. 3), the plain definition of removal (Sec. 4.2: composite
again without the splat), a library routine (scipy's spherical harmonics,
Python's exact rationals) or brute force on tiny inputs.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2601_14821_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _one_pixel_proj(alphas, colours, W=1, H=1, centre=(0.5, 0.5)):
    """Hand-placed records: every splat centred on the pixel centre, so q = 0 and alpha = o."""
    n = len(alphas)
    proj = dict(mean2d=np.tile(np.array(centre, float), (n, 1)),
                conic=np.tile([1.0, 0.0, 1.0], (n, 1)).astype(float),
                rgb=np.array(colours, float).reshape(n, 3),
                depth_key=np.arange(1, n + 1, dtype=np.uint32),
                rect=np.tile([0, 0, 1, 1], (n, 1)).astype(np.int32),
                tiles_touched=np.ones(n, np.int32))
    scene = synth.Scene(np.zeros((n, 3), np.float32), np.ones((n, 3), np.float32),
                        np.tile(np.float32([1, 0, 0, 0]), (n, 1)), np.array(alphas, np.float32),
                        np.zeros((n, 16, 3), np.float32))
    cam = synth.Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 1.0, 1.0, 0.0, 0.0, W, H)
    return scene, cam, proj


# ---------------------------------------------------------------- hand-worked example
@pytest.mark.parametrize("t_min", [0.0, 1e-4])
@pytest.mark.parametrize("method", [0, 1])
def test_three_splat_pixel(method, t_min):
    g = json.load(open(os.path.join(GOLDEN, "three_splat_pixel.json")))
    for case in g["cases"]:
        scene, cam, proj = _one_pixel_proj(g["alpha"], g["colour"])
        s = synth.RenderSettings(bg=tuple(case["bg"]), t_min=t_min)
        r = oracle.render(scene, cam, s, proj=proj, method=method,
                          want=("image", "t_final", "score_l1", "importance", "n_blend"))
        assert r["n_blend"][0, 0] == 3
        np.testing.assert_array_equal(r["image"][0, 0], case["image"])
        assert r["t_final"][0, 0] == g["t_final"]
        np.testing.assert_array_equal(r["importance"], g["weights"])
        np.testing.assert_allclose(r["score_l1"], case["pd_l1"], rtol=0, atol=1e-15)
        # signed PD per channel from the squared-error change (Sec. 4.2):
        # dSE(target) = |PD|^2 + 2 PD.(c - target); a unit shift of the target in
        # channel ch moves dSE by 2 PD_ch.
        img = np.array(case["image"], np.float32).reshape(1, 1, 3)
        base = oracle.render(scene, cam, s, proj=proj, method=method, target=img, want=("score_se",))
        for ch in range(3):
            t2 = img.copy()
            t2[0, 0, ch] -= 1.0
            sh = oracle.render(scene, cam, s, proj=proj, method=method, target=t2, want=("score_se",))
            pd = (sh["score_se"] - base["score_se"]) / 2.0
            np.testing.assert_allclose(pd, np.array(case["pd"])[:, ch], rtol=0, atol=1e-15)


# ---------------------------------------------------------------- compositing invariants
def _small():
    scene, cams = synth.workload_small()
    return scene, cams


def test_single_splat_removal_is_alpha_times_bg_minus_c():
    # one splat: PD = alpha (bg - c) at every pixel, so its L1 score equals its
    # importance sum_x alpha(x) times |bg - c|_1
    scene, cams = _small()
    sc = scene.subset([7])
    s = synth.RenderSettings(bg=(0.2, 0.7, 0.1))
    for method in (0, 1):
        r = oracle.render(sc, cams[0], s, method=method, want=("score_l1", "importance"))
        c = r["proj"]["rgb"][0]
        expect = r["importance"][0] * np.abs(np.array(s.bg, np.float32).astype(float) - c).sum()
        assert r["importance"][0] > 1.0
        assert abs(r["score_l1"][0] - expect) <= 1e-12 * expect


@pytest.mark.parametrize("t_min", [0.0, 1e-4])
def test_uniform_colour_background_gives_zero_effect(t_min):
    scene, cams = _small()
    proj = oracle.project(scene, cams[1], synth.RenderSettings())
    proj["rgb"][:] = 0.25
    s = synth.RenderSettings(bg=(0.25, 0.25, 0.25), t_min=t_min)
    r = oracle.render(scene, cams[1], s, proj=proj, want=("score_l1", "magnitude"))
    assert r["magnitude"].max() > 1.0
    assert np.all(r["score_l1"] <= 1e-13 * (1.0 + r["magnitude"]))


def test_partition_of_unity():
    # sum_k T_k alpha_k + T_final = 1 at every pixel: with white splats on black,
    # the image equals 1 - T_final, and sum of importances + sum T_final = #pixels
    scene, cams = _small()
    s = synth.RenderSettings()
    proj = oracle.project(scene, cams[2], s)
    proj["rgb"][:] = 1.0
    r = oracle.render(scene, cams[2], s, proj=proj, want=("image", "t_final", "importance"))
    for ch in range(3):
        np.testing.assert_allclose(r["image"][..., ch], 1.0 - r["t_final"], rtol=0, atol=1e-13)
    P = cams[2].width * cams[2].height
    assert abs(r["importance"].sum() + r["t_final"].sum() - P) < 1e-9
    assert np.all(r["t_final"] <= 1.0) and np.all(r["t_final"] >= 0.0)


def test_linear_in_colour_and_background():
    scene, cams = _small()
    s1 = synth.RenderSettings(bg=(0.25, 0.5, 0.125))
    s2 = synth.RenderSettings(bg=(0.5, 1.0, 0.25))
    proj = oracle.project(scene, cams[0], s1)
    r1 = oracle.render(scene, cams[0], s1, proj=proj, want=("score_l1",))
    proj2 = dict(proj)
    proj2["rgb"] = proj["rgb"] * 2.0
    r2 = oracle.render(scene, cams[0], s2, proj=proj2, want=("score_l1",))
    np.testing.assert_allclose(r2["score_l1"], 2.0 * r1["score_l1"], rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- removal = definition
def test_closed_form_equals_literal_deletion_exact_mode():
    """Exact mode (no early stop): the paper's partial-colour closed form equals
    compositing again with splat k deleted, for the first 50 splats of every view."""
    scene, cams = _small()
    s = synth.RenderSettings(t_min=0.0)
    checked = 0
    for cam in cams:
        r = oracle.render(scene, cam, s, method=0, want=("image", "score_l1"))
        for k in range(50):
            img = oracle.render_without(scene, cam, s, k, proj=r["proj"], bins=r["bins"])
            lit = np.abs(img - r["image"]).sum()
            assert abs(lit - r["score_l1"][k]) <= 1e-12 * max(1.0, lit)
            checked += lit > 0
    assert checked > 100


def test_production_mode_closed_form_equals_truncated_definition():
    scene, cams = _small()
    s = synth.RenderSettings()
    for cam in cams:
        a = oracle.render(scene, cam, s, method=0, want=("score_l1",))
        b = oracle.render(scene, cam, s, method=1, want=("score_l1",))
        np.testing.assert_allclose(a["score_l1"], b["score_l1"], rtol=1e-12, atol=1e-13)


def test_removal_equals_minus_alpha_dC_dalpha():
    """C is affine in alpha_k, so PD_k = -alpha_k dC/dalpha_k = -o_k dC/do_k where
    alpha_k = o_k G is unclamped; dC/do_k by a central difference of full renders."""
    scene, cams = _small()
    s = synth.RenderSettings(t_min=0.0)
    cam = cams[0]
    base = oracle.render(scene, cam, s, want=("image", "score_l1"))
    ks = [k for k in range(200) if 0.05 < scene.opacities[k] < 0.95 and base["score_l1"][k] > 1e-3][:8]
    assert len(ks) >= 5
    for k in ks:
        o = scene.opacities[k]
        up, dn = scene.subset(np.arange(scene.n)), scene.subset(np.arange(scene.n))
        up.opacities[k] = np.float32(o * (1 + 4e-6))
        dn.opacities[k] = np.float32(o * (1 - 4e-6))
        iu = oracle.render(up, cam, s, want=("image",))["image"]
        idn = oracle.render(dn, cam, s, want=("image",))["image"]
        dC = (iu - idn) / (float(up.opacities[k]) - float(dn.opacities[k]))
        fd = np.abs(-float(o) * dC).sum()
        assert abs(fd - base["score_l1"][k]) <= 1e-6 * base["score_l1"][k]


# ---------------------------------------------------------------- projection
def _axis_camera(W=64, H=48, f=50.0):
    return synth.Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f, W / 2, H / 2, W, H)


def _one(mean, scale, quat, opac=0.9):
    sh = np.zeros((1, 16, 3), np.float32)
    return synth.Scene(np.float32([mean]), np.float32([scale]), np.float32([quat]), np.float32([opac]), sh)


def test_isotropic_splat_on_axis():
    cam = _axis_camera()
    s = synth.RenderSettings()
    rng = np.random.default_rng(0)
    for z, sc in ((2.0, 0.05), (5.0, 0.2), (1.0, 0.01)):
        q = rng.normal(size=4)
        p = oracle.project(_one([0, 0, z], [sc] * 3, q / np.linalg.norm(q)), cam, s)
        e = (50.0 * float(np.float32(sc)) / z) ** 2 + float(np.float32(0.3))
        np.testing.assert_allclose(p["cov2d"][0], [e, 0.0, e], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(p["mean2d"][0], [32.0, 24.0], rtol=0, atol=1e-12)


def test_rotation_about_view_axis_hand_formula():
    # q = (cos th/2, 0, 0, sin th/2) rotates the scale ellipse by +th in the image plane
    cam = _axis_camera()
    s = synth.RenderSettings()
    sx, sy, z, f = 0.2, 0.05, 4.0, 50.0
    for th in (0.3, 1.1, -0.7):
        q = [math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)]
        sc = _one([0, 0, z], [sx, sy, 0.01], q)
        p = oracle.project(sc, cam, s)
        a2, b2 = (f / z * float(np.float32(sx))) ** 2, (f / z * float(np.float32(sy))) ** 2
        qn = np.float32(q).astype(float)
        qn /= np.linalg.norm(qn)
        c, sn = qn[0] ** 2 - qn[3] ** 2, 2 * qn[0] * qn[3]
        exp = [c * c * a2 + sn * sn * b2 + float(np.float32(0.3)), c * sn * (a2 - b2),
               sn * sn * a2 + c * c * b2 + float(np.float32(0.3))]
        np.testing.assert_allclose(p["cov2d"][0], exp, rtol=1e-12, atol=1e-12)


def test_off_axis_jacobian_and_clamp():
    cam = _axis_camera(W=64, H=48, f=50.0)
    s = synth.RenderSettings()
    sc, z = 0.05, 3.0
    lim = float(np.float32(1.3)) * 32.0 / 50.0
    for x in (0.5, -0.9, 1.9, -2.5):       # the last two clamp x/z
        p = oracle.project(_one([x, 0.0, z], [sc] * 3, [1, 0, 0, 0]), cam, s)
        t = min(lim, max(-lim, float(np.float32(x)) / z))
        s2 = float(np.float32(sc)) ** 2
        exx = (50.0 / z) ** 2 * s2 * (1 + t * t) + float(np.float32(0.3))
        eyy = (50.0 / z) ** 2 * s2 + float(np.float32(0.3))
        np.testing.assert_allclose(p["cov2d"][0], [exx, 0.0, eyy], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(p["mean2d"][0, 0], 50.0 * float(np.float32(x)) / z + 32.0, rtol=1e-14)


def test_culling_rules():
    cam = _axis_camera()
    s = synth.RenderSettings()
    cases = [([0, 0, 0.1], [0.1] * 3, [1, 0, 0, 0], 0.9),     # behind the near plane
             ([0, 0, 3.0], [0.1] * 3, [1, 0, 0, 0], 0.003),   # opacity below alpha_min
             ([0, 0, 3.0], [0.1] * 3, [0, 0, 0, 0], 0.9),     # zero quaternion
             ([40, 0, 3.0], [0.1] * 3, [1, 0, 0, 0], 0.9)]    # far off screen
    for m, sc, q, o in cases:
        p = oracle.project(_one(m, sc, q, o), cam, s)
        assert p["tiles_touched"][0] == 0
    p = oracle.project(_one([0, 0, 3.0], [0.1] * 3, [1, 0, 0, 0], 0.9), cam, s)
    assert p["tiles_touched"][0] > 0


def test_rect_is_conservative_brute_force():
    scene, cams = synth.workload_small()
    s = synth.RenderSettings(tile_w=8, tile_h=8)
    cam = cams[3]
    p = oracle.project(scene, cam, s)
    W, H = cam.width, cam.height
    ys, xs = np.mgrid[0:H, 0:W] + 0.5
    for i in range(0, scene.n, 7):
        dx, dy = xs - p["mean2d"][i, 0], ys - p["mean2d"][i, 1]
        A, B, Cc = p["conic"][i]
        q = A * dx * dx + 2 * B * dx * dy + Cc * dy * dy
        vis = (q <= 9.0) & (float(scene.opacities[i]) * np.exp(-0.5 * q) >= float(np.float32(1 / 255)))
        x0, y0, x1, y1 = p["rect"][i]
        assert p["tiles_touched"][i] == max(0, x1 - x0) * max(0, y1 - y0)
        if vis.any():
            tx, ty = (xs[vis] // 8).astype(int), (ys[vis] // 8).astype(int)
            assert tx.min() >= x0 and tx.max() < x1 and ty.min() >= y0 and ty.max() < y1


def _round_f32(fr: Fraction) -> float:
    """Round an exact rational to the nearest float32, ties to even."""
    if fr == 0:
        return 0.0
    sign = -1 if fr < 0 else 1
    a = abs(fr)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    ulp = Fraction(2) ** (e - 23)
    m = a / ulp
    fl = math.floor(m)
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * float(fl * ulp)


def test_depth_key_is_correctly_rounded_fma_chain():
    scene, cams = synth.workload_small()
    s = synth.RenderSettings()
    for cam in cams[:2]:
        p = oracle.project(scene, cam, s)
        for i in range(0, scene.n, 97):
            acc = Fraction(float(cam.t[2]))
            for j in range(3):
                acc = Fraction(_round_f32(Fraction(float(cam.R[2, j])) * Fraction(float(scene.means[i, j])) + acc))
            key = np.float32(float(acc)).view(np.uint32)
            assert p["depth_key"][i] == key


# ---------------------------------------------------------------- spherical harmonics
def _real_sh_scipy(l, m, d):
    from scipy import special
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    Y = special.sph_harm_y(l, abs(m), theta, phi)       # complex, Condon-Shortley phase included
    if m > 0:
        return math.sqrt(2.0) * Y.real
    if m < 0:
        return math.sqrt(2.0) * Y.imag
    return Y.real


def test_sh_matches_scipy():
    rng = np.random.default_rng(3)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        out = oracle.sh_basis(3, d)
        for l in range(4):
            for m in range(-l, l + 1):
                assert abs(out[l * (l + 1) + m] - _real_sh_scipy(l, m, d)) < 1e-13


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for the degree-6 products
    xs, ws = np.polynomial.legendre.leggauss(8)
    nphi = 16
    G = np.zeros((16, 16))
    for x, w in zip(xs, ws):
        for j in range(nphi):
            phi = 2 * math.pi * j / nphi
            st = math.sqrt(1 - x * x)
            Y = oracle.sh_basis(3, [st * math.cos(phi), st * math.sin(phi), x])
            G += w * (2 * math.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-13)


def test_sh_sign_and_dc():
    Y = oracle.sh_basis(1, [1.0, 0.0, 0.0])
    assert abs(Y[3] - (-math.sqrt(3 / (4 * math.pi)))) < 1e-15      # Y_{1,1}(+x), Condon-Shortley
    Y = oracle.sh_basis(1, [0.0, 1.0, 0.0])
    assert abs(Y[1] - (-math.sqrt(3 / (4 * math.pi)))) < 1e-15      # Y_{1,-1}(+y)
    # degree 0 only: view-independent colour 0.5 + L0 / (2 sqrt(pi))
    scene, cams = synth.workload_small()
    s = synth.RenderSettings(sh_degree=0)
    cols = [oracle.project(scene, c, s)["rgb"][:20] for c in cams]
    for c in cols[1:]:
        np.testing.assert_array_equal(c, cols[0])
    exp = np.maximum(0.0, 0.5 + scene.sh[:20, 0, :].astype(float) / (2 * math.sqrt(math.pi)))
    np.testing.assert_allclose(cols[0], exp, rtol=1e-14, atol=1e-15)


# ---------------------------------------------------------------- bin and sort
def test_bin_sort_brute_force_with_ties():
    rng = np.random.default_rng(11)
    n, tx, ty = 300, 7, 5
    x0 = rng.integers(0, tx, n); y0 = rng.integers(0, ty, n)
    x1 = np.minimum(tx, x0 + rng.integers(0, 4, n)); y1 = np.minimum(ty, y0 + rng.integers(1, 3, n))
    rect = np.stack([x0, y0, x1, y1], 1).astype(np.int32)
    key = rng.integers(1000, 1040, n).astype(np.uint32)          # many equal keys
    tile, ids, ranges = oracle.bin_sort(rect, key, tx, ty)
    for t in range(tx * ty):
        cx, cy = t % tx, t // tx
        members = [i for i in range(n) if x0[i] <= cx < x1[i] and y0[i] <= cy < y1[i]]
        exp = sorted(members, key=lambda i: (int(key[i]), i))
        b, e = ranges[t]
        assert list(ids[b:e]) == exp
        assert np.all(tile[b:e] == t)
    assert len(ids) == sum(max(0, a) * max(0, b) for a, b in zip(x1 - x0, y1 - y0))


# ---------------------------------------------------------------- early stop and alpha clamp (hand-worked)
@pytest.mark.parametrize("method", [0, 1])
def test_early_stop_pixel(method):
    """Where the stop falls (strictly below t_min), what the truncated list gives,
    and the literal deletion with the stop rerun (tests/golden/early_stop_pixel.json)."""
    g = json.load(open(os.path.join(GOLDEN, "early_stop_pixel.json")))
    for case in g["cases"]:
        scene, cam, proj = _one_pixel_proj(g["alpha"], g["colour"])
        s = synth.RenderSettings(bg=tuple(case["bg"]), t_min=case["t_min"])
        r = oracle.render(scene, cam, s, proj=proj, method=method,
                          want=("image", "t_final", "n_walk", "n_blend", "score_l1", "importance"))
        assert r["n_walk"][0, 0] == case["n_walk"] and r["n_blend"][0, 0] == case["n_blend"]
        assert r["t_final"][0, 0] == case["t_final"]
        np.testing.assert_array_equal(r["image"][0, 0], case["image"])
        np.testing.assert_array_equal(r["importance"], case["weights"])
        np.testing.assert_allclose(r["score_l1"], case["pd_l1"], rtol=0, atol=1e-15)
        for k in range(3):
            lit = oracle.render_without(scene, cam, s, k, proj=proj)
            np.testing.assert_array_equal(lit[0, 0], case["literal"][k])


@pytest.mark.parametrize("method", [0, 1])
def test_alpha_clamp_pixel(method):
    """alpha = alpha_max where o G exceeds it (tests/golden/alpha_clamp_pixel.json)."""
    g = json.load(open(os.path.join(GOLDEN, "alpha_clamp_pixel.json")))
    for case in g["cases"]:
        scene, cam, proj = _one_pixel_proj(case["opacity"], case["colour"])
        s = synth.RenderSettings(bg=tuple(case["bg"]), alpha_max=g["alpha_max"], t_min=0.0)
        r = oracle.render(scene, cam, s, proj=proj, method=method,
                          want=("image", "t_final", "score_l1", "importance"))
        np.testing.assert_array_equal(r["image"][0, 0], case["image"])
        assert r["t_final"][0, 0] == case["t_final"]
        np.testing.assert_array_equal(r["importance"], case["weights"])
        np.testing.assert_allclose(r["score_l1"], case["pd_l1"], rtol=0, atol=1e-15)


def test_default_alpha_clamp_and_visibility_floor():
    """Default settings: o = 0.995 blends with alpha = alpha_max = 0.99 (FP32 value of
    the setting), PD = alpha (bg - c); o below alpha_min = 1/255 is not blended."""
    s = synth.RenderSettings(bg=(1.0, 1.0, 1.0), t_min=0.0)
    a_max = float(np.float32(s.alpha_max))
    scene, cam, proj = _one_pixel_proj([0.995], [[0.25, 0.5, 0.75]])
    r = oracle.render(scene, cam, s, proj=proj, want=("image", "score_l1", "importance"))
    assert r["importance"][0] == a_max
    expect = a_max * (0.75 + 0.5 + 0.25)
    assert abs(r["score_l1"][0] - expect) <= 1e-15
    below = float(np.float32(1.0 / 255.0)) * 0.999
    scene, cam, proj = _one_pixel_proj([below], [[0.25, 0.5, 0.75]])
    r = oracle.render(scene, cam, s, proj=proj, want=("image", "score_l1", "n_blend"))
    assert r["n_blend"][0, 0] == 0 and r["score_l1"][0] == 0.0
    np.testing.assert_array_equal(r["image"][0, 0], [1.0, 1.0, 1.0])


# ---------------------------------------------------------------- SH direction (Sec. 3)
@pytest.mark.parametrize("index,axis,sign", [(3, 0, -1.0), (1, 1, -1.0), (2, 2, 1.0)])
def test_sh_degree1_direction_from_camera_to_splat(index, axis, sign):
    """Real SH of degree 1 with the Condon-Shortley phase are Y_{1,1} = -k x,
    Y_{1,-1} = -k y, Y_{1,0} = k z with k = sqrt(3 / (4 pi)), at index l(l+1)+m
    (0-based). The colour is evaluated along d = unit vector from the camera
    centre to the splat (Sec. 3): a splat at the origin holding only that
    coefficient L has colour 0.5 + L Y(d), with d = -axis seen from a camera on
    the +axis and d = +axis from the -axis, so the two sides see the degree-1
    term with opposite signs (a flipped direction or phase swaps them)."""
    k = math.sqrt(3.0 / (4.0 * math.pi))
    L = np.array([0.2, -0.1, 0.3])
    scene = synth.Scene(np.zeros((1, 3), np.float32), np.full((1, 3), 0.05, np.float32),
                        np.float32([[1, 0, 0, 0]]), np.float32([0.9]), np.zeros((1, 16, 3), np.float32))
    scene.sh[0, index, :] = L
    s = synth.RenderSettings(sh_degree=1)
    up = (0.0, 0.0, 1.0) if axis == 1 else (0.0, 1.0, 0.0)
    for side in (1.0, -1.0):
        eye = [0.0, 0.0, 0.0]
        eye[axis] = 3.0 * side
        cam = synth.look_at(eye, up=up, width=64, height=64)
        o = oracle.project(scene, cam, s)
        d = -np.array(eye) / 3.0                     # camera -> splat at the origin
        expect = 0.5 + L.astype(np.float32).astype(float) * sign * k * d[axis]
        np.testing.assert_allclose(o["rgb"][0], expect, rtol=0, atol=1e-6)
        # the +axis camera sees 0.5 - sign k L, the -axis camera 0.5 + sign k L
        np.testing.assert_allclose(o["rgb"][0] - 0.5, -side * sign * k * L, rtol=0, atol=2e-7)
