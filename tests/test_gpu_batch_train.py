"""The fine-tuning step inside the batch (Sec. 4.6, through the C ABI): per job
in its lane, composite, L1 loss gradient and the hand-written backward, in the
same run and HIP graph as the removal scores. Gradients equal the plain
autograd path's (whose own tests pin it to the FP64 oracle), for scenes whose
views are split over several jobs, with and without score outputs, eager and
replayed."""
import numpy as np
import pytest
import torch

from paper_2601_14821_amd import autograd, batch, raster, synth

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")


def _scenes():
    out = []
    for k, (n, v, wh) in enumerate(((4000, 3, (160, 120)), (20000, 5, (256, 144)))):
        scene = synth.random_scene(n, 1200 + k, clustered=True)
        cams = synth.hemisphere_cameras(v, wh[0], wh[1], seed=1300 + k)
        out.append((scene, cams))
    return out


def _targets(s, scene, cams, seed):
    """Render of a perturbed copy of the scene: the fine-tuning target."""
    rz = raster.Rasterizer(s)
    return rz.render_views(raster.to_device(synth.perturbed(scene, seed)), cams).image.clone()


def _autograd_grads(s, scene, cams, tgt):
    ds = raster.to_device(scene)
    params = [t.clone().requires_grad_(True) for t in (ds.means, ds.scales, ds.quats, ds.opacities, ds.sh)]
    img = autograd.render(*params, cams, raster.Rasterizer(s))
    (img - tgt).abs().mean().backward()
    return [p.grad.detach() for p in params]


def _zero_grads(ds):
    return raster.DeviceScene(*(torch.zeros_like(t) for t in (ds.means, ds.scales, ds.quats, ds.opacities, ds.sh)))


def _close(name, got, ref, rel=2e-5):
    g = got.double().cpu().numpy().ravel()
    r = ref.double().cpu().numpy().ravel()
    nr = np.linalg.norm(r)
    assert nr > 0, name
    e = np.linalg.norm(g - r) / nr
    worst = np.abs(g - r).max() / np.abs(r).max()
    print(f"{name}: rel L2 {e:.2e}, worst {worst:.2e}", flush=True)
    assert e <= rel and worst <= 10 * rel, (name, e, worst)


@pytest.mark.parametrize("with_scores", [True, False])
def test_batched_step_equals_autograd(with_scores):
    _need_gpu()
    s = synth.RenderSettings()
    items, refs, plain_scores = [], [], []
    for k, (scene, cams) in enumerate(_scenes()):
        ds = raster.to_device(scene)
        tgt = _targets(s, scene, cams, 1400 + k)
        V, H, W = len(cams), cams[0].height, cams[0].width
        grads = _zero_grads(ds)
        out = raster.Outputs(scores=torch.zeros(scene.n, device="cuda")) if with_scores else raster.Outputs()
        items.append((ds, cams, out, None, batch.FineTune(tgt, grads, 1.0 / (V * H * W * 3))))
        refs.append(_autograd_grads(s, scene, cams, tgt))
        if with_scores:
            sc = torch.zeros(scene.n, device="cuda")
            raster.Rasterizer(s).score_views_fused(ds, cams, scores=sc)
            plain_scores.append(sc)
    bs = batch.BatchScorer(items, s, views_per_job=2)      # every scene's views over several jobs
    bs.run()
    torch.cuda.synchronize()
    assert bs.overflowed() == 0
    for k, (item, ref) in enumerate(zip(items, refs)):
        g = item[4].grads
        for name, got, r in zip(("means", "scales", "quats", "opacities", "sh"),
                                (g.means, g.scales, g.quats, g.opacities, g.sh), ref):
            _close(f"scene {k} d_{name}", got, r)
        if with_scores:
            a = item[2].scores.double().cpu().numpy()
            b = plain_scores[k].double().cpu().numpy()
            assert np.abs(a - b).max() <= 2e-5 * np.abs(b).max() + 1e-7
    bs.close()


def test_batched_step_graph_replays():
    """The captured graph replays the step: with the gradients cleared between
    replays (eager work in between), every replay gives the eager run's."""
    _need_gpu()
    s = synth.RenderSettings()
    scene, cams = _scenes()[1]
    ds = raster.to_device(scene)
    tgt = _targets(s, scene, cams, 1500)
    grads = _zero_grads(ds)
    V, H, W = len(cams), cams[0].height, cams[0].width
    scores = torch.zeros(scene.n, device="cuda")
    bs = batch.BatchScorer([(ds, cams, raster.Outputs(scores=scores), None,
                             batch.FineTune(tgt, grads, 1.0 / (V * H * W * 3)))], s, views_per_job=3)
    bs.run()
    torch.cuda.synchronize()
    names = ("d_means", "d_scales", "d_quats", "d_opacities", "d_sh", "scores")
    live = (grads.means, grads.scales, grads.quats, grads.opacities, grads.sh, scores)
    eager = [t.clone() for t in live]
    bs.capture()
    for rep in range(3):
        for t in live:
            t.zero_()
        torch.cuda.synchronize()
        bs.replay()
        torch.cuda.synchronize()
        # the same sums up to the order of their float atomic additions
        for name, got, ref in zip(names, live, eager):
            _close(f"replay {rep} {name}", got, ref)
    bs.close()


def test_one_scene_over_many_jobs():
    """Eight one-view jobs of one scene add into the same gradient arrays: they
    share a lane (the projection backward adds without atomics), and the sums
    equal the autograd path's."""
    _need_gpu()
    s = synth.RenderSettings()
    scene = synth.random_scene(50000, 1600, clustered=True)
    cams = synth.hemisphere_cameras(8, 320, 180, seed=1601)
    ds = raster.to_device(scene)
    tgt = _targets(s, scene, cams, 1602)
    V, H, W = len(cams), cams[0].height, cams[0].width
    grads = _zero_grads(ds)
    bs = batch.BatchScorer([(ds, cams, raster.Outputs(), None, batch.FineTune(tgt, grads, 1.0 / (V * H * W * 3)))],
                           s, views_per_job=1)
    assert bs.n_jobs == 8
    bs.run()
    torch.cuda.synchronize()
    ref = _autograd_grads(s, scene, cams, tgt)
    for name, got, r in zip(("means", "scales", "quats", "opacities", "sh"),
                            (grads.means, grads.scales, grads.quats, grads.opacities, grads.sh), ref):
        _close(f"d_{name}", got, r)
    bs.close()
