"""The pruning controller on the GPU (Sec. 4.3, through the C ABI) against the
oracle: the selection bit-exact on the same inputs (random arrays with ties,
negative dMSE, non-candidates; a hand-worked case; up to 3M splats), the
survivor compaction exact, and whole controller runs on the small and the
500k-splat scenes, where every iteration's statistics match the oracle's on the
same survivors and every iteration's choice matches the oracle's choice on the
GPU statistics bit for bit."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import prune as oprune
from paper_2601_14821_amd import prune, raster, synth
from score_tolerance import compare_scores, oracle_views

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")


def _gpu_select(dm, im, dmax, R, a=10.0):
    rm, n = prune.select(torch.from_numpy(dm).cuda(), torch.from_numpy(im).cuda(), dmax, R, a)
    torch.cuda.synchronize()
    return rm.cpu().numpy().astype(bool), int(n.item())


def test_select_hand_worked_case():
    _need_gpu()
    g = json.load(open(os.path.join(HERE, "golden", "prune_select.json")))
    dm = np.array(g["dmse"], np.float32)
    im = np.array(g["importance"], np.float32)
    for case in g["cases"]:
        got, n = _gpu_select(dm, im, g["dmse_max"], case["remaining"], g["a"])
        assert sorted(np.nonzero(got)[0].tolist()) == case["removed"], case
        assert n == len(case["removed"])


def _random_inputs(n, seed):
    rng = np.random.default_rng(seed)
    # a few repeated values (ties in m), a continuous part, exact zeros and non-candidates
    pool = np.float32([-3e-6, -2e-7, 0.0, 1e-9, 5e-8, 2.5e-7, 9.9e-7, 1e-6, 3e-5])
    dm = np.where(rng.random(n) < 0.4, rng.choice(pool, n),
                  rng.normal(2e-7, 6e-7, n)).astype(np.float32)
    dm[rng.random(n) < 0.01] = -0.0
    im = (rng.exponential(1.0, n) * (rng.random(n) < 0.9)).astype(np.float64)
    im = (im / im.sum() * 0.8).astype(np.float32)     # an image fraction
    im[rng.random(n) < 0.02] = np.float32(im.max())   # repeated importances
    im = (im / im.astype(np.float64).sum() * 0.8).astype(np.float32)
    return dm, im


@pytest.mark.parametrize("n,seed", [(1, 1), (7, 2), (1000, 3), (65_537, 4), (400_000, 5), (3_000_000, 6)])
def test_select_matches_oracle_bit_exact(n, seed):
    _need_gpu()
    dm, im = _random_inputs(n, seed)
    for R in (48, 7, 2, 1):
        want = oprune.select(dm, im, 1e-6, R)
        got, k = _gpu_select(dm, im, 1e-6, R)
        print(f"n {n} remaining {R}: removed {want.sum()}", flush=True)
        np.testing.assert_array_equal(got, want)
        assert k == int(want.sum())


def test_select_edge_cases():
    _need_gpu()
    # nothing to remove: no candidate importance, no candidates, empty input
    got, k = _gpu_select(np.float32([0.5, 2.0, -1.0]), np.float32([0, 0.5, 0]), 1.0, 3)
    assert k == 0 and not got.any()
    got, k = _gpu_select(np.float32([1.0, 3.0]), np.float32([0.5, 0.5]), 1.0, 1)
    assert k == 0 and not got.any()
    got, k = _gpu_select(np.zeros(0, np.float32), np.zeros(0, np.float32), 1.0, 1)
    assert k == 0 and got.size == 0
    # importance outside [0, 1], NaN, or summing above 2: reported, nothing removed
    for im in (np.float32([0.5, 1.5, 0.0]), np.float32([0.9, 0.9, 0.9]), np.float32([0.2, np.nan, 0.1])):
        got, k = _gpu_select(np.zeros(3, np.float32), im, 1.0, 2)
        assert k == -1 and not got.any()
    # NaN dMSE is never a candidate; +-0 tie with each other by index
    dm = np.float32([np.nan, -0.0, 0.0, 0.5])
    im = np.float32([0.25, 0.25, 0.25, 0.25])
    for R in (1, 2, 3):
        got, _ = _gpu_select(dm, im, 1.0, R)
        np.testing.assert_array_equal(got, oprune.select(dm, im, 1.0, R))


def test_compact_keeps_survivors_in_order():
    _need_gpu()
    scene = synth.random_scene(50_003, 77)
    ds = raster.to_device(scene)
    rng = np.random.default_rng(3)
    rm = (rng.random(scene.n) < 0.37).astype(np.uint8)
    ids = torch.from_numpy((np.arange(scene.n) * 3 + 11).astype(np.int32)).cuda()
    kept, kid, k = prune.compact(ds, torch.from_numpy(rm).cuda(), ids)
    keep = rm == 0
    assert k == keep.sum()
    np.testing.assert_array_equal(kid.cpu().numpy(), (np.arange(scene.n) * 3 + 11)[keep])
    sub = scene.subset(np.nonzero(keep)[0])
    for a, b in ((kept.means, sub.means), (kept.scales, sub.scales), (kept.quats, sub.quats),
                 (kept.opacities, sub.opacities), (kept.sh, sub.sh)):
        np.testing.assert_array_equal(a.cpu().numpy(), b)
    # without ids: the original indices
    _, kid2, _ = prune.compact(ds, torch.from_numpy(rm).cuda())
    np.testing.assert_array_equal(kid2.cpu().numpy(), np.nonzero(keep)[0])


def _controller_run(scene, cams, s, n_iter, dmax, iterations):
    """GPU controller; per iteration: its statistics against the oracle's on the
    same survivors (and the same targets), its choice against the oracle's choice
    on the GPU statistics."""
    ds = raster.to_device(scene)
    pc = prune.PruneController(ds, cams, s, n_iter=n_iter, dmse_max=dmax)
    targets = pc.targets.cpu().numpy()
    V, P = len(cams), cams[0].width * cams[0].height
    alive = np.arange(scene.n)
    sizes = []
    for it in range(iterations):
        removed = pc.step()
        dm = pc.last["dmse"].cpu().numpy()
        im = pc.last["importance"].cpu().numpy()
        rm = pc.last["remove"].cpu().numpy().astype(bool)
        np.testing.assert_array_equal(rm, oprune.select(dm, im, dmax, n_iter - it))
        assert removed == rm.sum()
        # the statistics of this iteration's survivors, from the oracle
        tot, _ = oracle_views(scene.subset(alive), cams, s, target=targets)
        ref_dm = tot["score_se"] / (3 * V * P)
        ref_im = tot["importance"] / (V * P)
        compare_scores(im, ref_im, tot["magnitude"] / (V * P), tot["flag_mass"] / (V * P), rtol=1e-4, mfloor=0.0)
        compare_scores(dm, ref_dm, 3 * tot["magnitude"] / (3 * V * P),
                       (3 * tot["flag_mass"] + 3e-3 * tot["score_l1"]) / (3 * V * P))
        alive = alive[~rm]
        np.testing.assert_array_equal(pc.ids.cpu().numpy(), alive)
        sizes.append(len(alive))
        print(f"iteration {it}: removed {removed}, {len(alive)} left", flush=True)
    return sizes


def test_controller_small_scene_all_iterations():
    _need_gpu()
    scene, cams = synth.workload_small()
    sizes = _controller_run(scene, cams, synth.RenderSettings(), n_iter=6, dmax=1e-6, iterations=6)
    assert sizes[-1] < scene.n - 300      # the candidates' importance was spent over the iterations


def test_controller_single_view_scene():
    _need_gpu()
    scene, cams = synth.workload_single_view()
    sizes = _controller_run(scene, cams, synth.RenderSettings(), n_iter=48, dmax=1e-9, iterations=2)
    assert sizes[0] < scene.n
