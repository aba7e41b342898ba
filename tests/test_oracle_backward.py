"""Pins of the oracle's analytic FP64 backward against central finite differences
of its own forward (FP64, steps below FP32 resolution), on the 64-splat 32x32
case and on screen-space records. A parameter whose +-h renders take different
decisions (blended set or stop position) is skipped and counted."""
import numpy as np
import pytest

import oracle
from paper_2601_14821_amd import synth


def _scene64():
    return synth.workload_fd_case()


def _f64_scene(scene):
    return synth.Scene(*(np.array(a, np.float64) for a in
                         (scene.means, scene.scales, scene.quats, scene.opacities, scene.sh)))


def _loss(scene, cam, s, w):
    r = oracle.render(scene, cam, s, threads=1, want=("image", "n_blend", "n_walk"))
    return float((r["image"] * w).sum()), r["n_blend"], r["n_walk"]


@pytest.mark.parametrize("t_min", [0.0, 1e-4])
def test_parameter_gradients_match_finite_differences(t_min):
    scene, cams = _scene64()
    cam = cams[0]
    s = synth.RenderSettings(t_min=t_min, bg=(0.1, 0.2, 0.3))
    sc = _f64_scene(scene)
    rng = np.random.default_rng(5)
    w = rng.normal(size=(cam.height, cam.width, 3))
    g = oracle.backward(sc, cam, s, w, threads=1)
    base, nb0, nw0 = _loss(sc, cam, s, w)
    fields = [("means", "d_means"), ("scales", "d_scales"), ("quats", "d_quats"), ("opacities", "d_opac"),
              ("sh", "d_sh")]
    checked = skipped = 0
    worst = 0.0
    for f, gk in fields:
        arr = getattr(sc, f)
        ga = g[gk].reshape(arr.shape)
        scale = np.abs(ga).max()
        flat_idx = list(np.ndindex(arr.shape))
        # every parameter of 12 splats (all SH coefficients included)
        for idx in [ix for ix in flat_idx if ix[0] % 5 == 0][:12 * int(np.prod(arr.shape[1:]))]:
            th = arr[idx]
            h = 1e-6 * max(1.0, abs(th))
            arr[idx] = th + h
            lp, nbp, nwp = _loss(sc, cam, s, w)
            arr[idx] = th - h
            lm, nbm, nwm = _loss(sc, cam, s, w)
            arr[idx] = th
            if not (np.array_equal(nbp, nb0) and np.array_equal(nbm, nb0) and np.array_equal(nwp, nw0)
                    and np.array_equal(nwm, nw0)):
                skipped += 1
                continue
            fd = (lp - lm) / (2 * h)
            err = abs(fd - ga[idx])
            worst = max(worst, err / (abs(ga[idx]) + 1e-6 * scale))
            assert err <= 1e-5 * abs(ga[idx]) + 1e-7 * scale + 1e-9, (f, idx, fd, ga[idx])
            checked += 1
    assert checked > 500 and skipped <= checked // 20, (checked, skipped)


def test_screen_space_gradients_match_finite_differences():
    """The compositing part alone: perturb the projected records."""
    scene, cams = synth.workload_small()
    cam = cams[1]
    s = synth.RenderSettings(t_min=0.0)
    sc = _f64_scene(scene)
    proj = oracle.project(sc, cam, s)
    tx, ty = s.tiles(cam)
    bins = oracle.bin_sort(proj["rect"], proj["depth_key"], tx, ty)
    rng = np.random.default_rng(9)
    w = rng.normal(size=(cam.height, cam.width, 3))
    g = oracle.backward(sc, cam, s, w, proj=proj, bins=bins)

    def L(p, o=None):
        scn = sc if o is None else synth.Scene(sc.means, sc.scales, sc.quats, o, sc.sh)
        r = oracle.render(scn, cam, s, proj=p, bins=bins, threads=4, want=("image", "n_blend"))
        return float((r["image"] * w).sum()), r["n_blend"]

    _, nb0 = L(proj)
    ks = [k for k in np.argsort(-np.abs(g["d_mean2d"]).sum(1))[:15]]
    checked = 0
    for k in ks:
        for key, gk, n in (("mean2d", "d_mean2d", 2), ("conic", "d_conic", 3), ("rgb", "d_rgb", 3)):
            for j in range(n):
                p = {kk: vv.copy() if isinstance(vv, np.ndarray) else vv for kk, vv in proj.items()}
                th = proj[key][k, j]
                h = 1e-7 * max(1.0, abs(th))
                p[key][k, j] = th + h
                lp, nbp = L(p)
                p[key][k, j] = th - h
                lm, nbm = L(p)
                if not (np.array_equal(nbp, nb0) and np.array_equal(nbm, nb0)):
                    continue
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[gk][k, j]) <= 1e-6 * abs(g[gk][k, j]) + 1e-8, (key, k, j, fd, g[gk][k, j])
                checked += 1
        o = sc.opacities.copy()
        th = o[k]
        h = 1e-7
        o[k] = th + h
        lp, _ = L(proj, o)
        o[k] = th - h
        lm, _ = L(proj, o)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g["d_opac"][k]) <= 1e-6 * abs(g["d_opac"][k]) + 1e-8
    assert checked > 100


def test_removal_effect_equals_minus_alpha_times_gradient():
    """With the pixel loss L = sum_x w(x).C(x), an unclamped splat's opacity gradient
    satisfies -o dL/do = sum_x w(x).PD_k(x) (Sec. 4.2's removal is affine in alpha);
    the squared-error mode with a shifted target recovers sum_x w.PD."""
    scene, cams = synth.workload_small()
    cam = cams[2]
    s = synth.RenderSettings(t_min=0.0)
    sc = _f64_scene(scene)
    rng = np.random.default_rng(21)
    # w = unit shift per channel: dSE(target = c - e) - dSE(target = c) = 2 PD . e
    r0 = oracle.render(sc, cam, s, want=("image",))
    img = (np.round(r0["image"] * 1024) / 1024).astype(np.float32)   # so that img - 1 is exact
    base = oracle.render(sc, cam, s, target=img, want=("score_se",))["score_se"]
    for ch in range(3):
        t2 = img.copy()
        t2[..., ch] -= 1.0
        se = oracle.render(sc, cam, s, target=t2, want=("score_se",))["score_se"]
        sum_pd = (se - base) / 2.0                     # sum_x PD_k,ch(x)
        w = np.zeros((cam.height, cam.width, 3))
        w[..., ch] = 1.0
        g = oracle.backward(sc, cam, s, w)
        ok = (sc.opacities < 0.98)
        lhs = -sc.opacities * g["d_opac"]
        np.testing.assert_allclose(lhs[ok], sum_pd[ok], rtol=1e-9, atol=1e-9)
    del rng
