"""The normalised per-splat reductions (through the C ABI): the per-camera
importance I_k(s) [V, N] and its camera average I_k (Sec. 4.1), and dMSE_k, the
dSE sums averaged over cameras, pixels and channels (Sec. 4.2), on the plain
fused path and through the persistent batch, against the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_2601_14821_amd import batch, raster, synth
from score_tolerance import compare_scores, oracle_views

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")


def _target(cams, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (len(cams), cams[0].height, cams[0].width, 3)).astype(np.float32)


def _check_importance(got, ref, tot_mag, flag, scale):
    """Importance within 1e-4 relative of the oracle's (its flag allowance, scaled)."""
    compare_scores(got, ref * scale, tot_mag * scale, flag * scale, rtol=1e-4, mfloor=0.0)


def _check_dmse(got, ref_se, mag, flag, l1, scale):
    # dSE = PD^2 + 2 PD (c - c_t): bounded by |PD| (|PD| + 2 |c - c_t|) <= 3 |PD|_1 for values in [0, 1]
    compare_scores(got, ref_se * scale, 3 * mag * scale, (3 * flag + 3e-3 * l1) * scale)


@pytest.mark.parametrize("settings", [synth.RenderSettings(), synth.RenderSettings(t_min=0.0, bg=(0.2, 0.3, 0.4))],
                         ids=["production", "exact-bg"])
def test_per_view_importance_and_dmse_plain(settings):
    _need_gpu()
    scene, cams = synth.workload_small()
    N, V, P = scene.n, len(cams), cams[0].width * cams[0].height
    target = _target(cams, 31)
    ds = raster.to_device(scene)
    rz = raster.Rasterizer(settings)
    dmse, imp, per_view = rz.removal_statistics(ds, cams, torch.from_numpy(target).cuda(), per_view_importance=True,
                                                views_per_batch=3)
    torch.cuda.synchronize()
    tot, views = oracle_views(scene, cams, settings, target=target)
    assert per_view.shape == (V, N)
    pv = per_view.cpu().numpy()
    for v in range(V):
        r = views[v]
        _check_importance(pv[v], r["importance"], r["magnitude"], r["flag_mass"], 1.0 / P)
    _check_importance(imp.cpu().numpy(), tot["importance"], tot["magnitude"], tot["flag_mass"], 1.0 / (V * P))
    # the camera average of I_k(s) is I_k
    np.testing.assert_allclose(pv.mean(axis=0), imp.cpu().numpy(), rtol=1e-5, atol=1e-12)
    _check_dmse(dmse.cpu().numpy(), tot["score_se"], tot["magnitude"], tot["flag_mass"], tot["score_l1"],
                1.0 / (3 * V * P))
    assert (np.abs(tot["score_se"]) > 0).sum() > 500


def test_batched_outputs_equal_plain():
    """Per-view importance, dSE (against targets) and L1 sums through the
    persistent batch equal the plain fused path, scene by scene."""
    _need_gpu()
    s = synth.RenderSettings()
    items, plain = [], []
    for k, (n, v, wh) in enumerate(((3000, 3, (160, 120)), (20000, 5, (320, 180)))):
        scene = synth.random_scene(n, 900 + k, clustered=True)
        cams = synth.hemisphere_cameras(v, wh[0], wh[1], seed=950 + k)
        ds = raster.to_device(scene)
        P = wh[0] * wh[1]
        tg = torch.from_numpy(_target(cams, 40 + k)).cuda()

        def outputs():
            return raster.Outputs(scores=torch.zeros(n, device="cuda"),
                                  scores_se=torch.zeros(n, device="cuda"), se_weight=1.0 / (3 * v * P),
                                  importance=torch.zeros(v, n, device="cuda"), importance_stride=n,
                                  importance_weight=1.0 / P)
        o_b, o_p = outputs(), outputs()
        items.append((ds, cams, o_b, tg))
        raster.Rasterizer(s).score_views_fused(ds, cams, views_per_batch=2, out=o_p, targets=tg)
        plain.append(o_p)
    bs = batch.BatchScorer(items, s, views_per_job=2)
    bs.run()
    torch.cuda.synchronize()
    assert bs.overflowed() == 0
    for (_, _, ob, _), op in zip(items, plain):
        for name in ("scores", "scores_se", "importance"):
            a = getattr(ob, name).cpu().numpy().astype(np.float64)
            b = getattr(op, name).cpu().numpy().astype(np.float64)
            assert np.abs(a - b).max() <= 2e-5 * np.abs(b).max() + 1e-12, name
            assert np.abs(a - b).sum() <= 2e-5 * np.abs(b).sum() + 1e-12, name
    bs.close()
