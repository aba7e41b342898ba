"""The codec's encoder (Sec. 4.5) on the GPU against the oracle: the bitstream
byte for byte and the leaf order at sizes the oracle finishes in seconds; at the
full scene (3M splats, 200 training cameras), what the oracle can check splat
by splat on a sample."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import codec as oc
from paper_2601_14821_amd import _lib as L
from paper_2601_14821_amd import codec, raster, synth

pytestmark = pytest.mark.gpu


def _scene(n, seed, dup=0):
    s = synth.random_scene(n, seed)
    if dup:
        s.means[-dup:] = s.means[:dup]
    return s


def _prm(q, D, **kw):
    p = oc.params(q, D)
    p.update(kw)
    return p, codec.params(q, D, **{k: v for k, v in kw.items()})


CASES = [  # n, seed, q, D, dup, cameras, extra
    (1, 0, 0.5, 21, 0, 3, {}),
    (2, 1, 0.5, 21, 1, 3, {}),              # two splats at one position: a cap leaf of two
    (3, 2, 0.5, 3, 0, 2, {}),
    (700, 3, 0.5, 21, 4, 6, {}),
    (2500, 4, 0.1, 8, 6, 4, {}),            # a shallow cap: many shared cap leaves
    (4000, 5, 1.0, 21, 0, 12, {}),
    (3000, 6, 0.5, 21, 0, 5, {"beta": 0.0}),
    (3000, 7, 0.5, 21, 0, 5, {"gamma": 0.0, "beta": 3e-3}),
    (20000, 8, 0.5, 21, 10, 8, {}),
]


@pytest.mark.parametrize("n,seed,q,D,dup,nc,extra", CASES)
def test_bitstream_matches_oracle(n, seed, q, D, dup, nc, extra):
    print(f"codec case n={n} seed={seed} q={q} D={D} dup={dup}", flush=True)
    s = _scene(n, seed, dup)
    cams = synth.hemisphere_cameras(nc, 64, 48, seed)
    po, pg = _prm(q, D, **extra)
    want, info = oc.encode_raw(s, cams, po)
    got, order = codec.encode(raster.to_device(s), cams, pg, want_order=True)
    got = got.tobytes()
    torch.cuda.synchronize()
    assert np.array_equal(order.cpu().numpy(), info["order"])
    assert len(got) == len(want)
    if got != want:
        a, b = np.frombuffer(got, np.uint8), np.frombuffer(want, np.uint8)
        first = int(np.nonzero(a != b)[0][0])
        pytest.fail(f"bitstreams differ first at byte {first} of {len(want)}")
    dec = codec.decode(codec.decompress(codec.compress(got)))
    ref = oc.decode_raw(want)
    for k in ("means", "scales", "quats", "opacities"):
        np.testing.assert_array_equal(dec[k], ref[k], err_msg=k)


def test_empty_model():
    cams = synth.ring_cameras(2, 32, 32)
    s = _scene(1, 0)
    ds = raster.to_device(s)
    empty = raster.DeviceScene(ds.means[:0], ds.scales[:0], ds.quats[:0], ds.opacities[:0], ds.sh[:0])
    raw = codec.encode(empty, cams, codec.params(0.5))
    assert raw.nbytes == oc.HEADER.size
    dec = codec.decode(raw)
    assert dec["means"].shape == (0, 3)


def test_out_of_range_values_are_rejected():
    s = _scene(100, 9)
    s.scales[17, 1] = 1e9        # 1e9 * SF_scale leaves int32
    with pytest.raises(L.PotrError) as e:
        codec.encode(raster.to_device(s), synth.ring_cameras(2, 32, 32), codec.params(0.5))
    assert e.value.status == L.POTR_EINVAL
    s = _scene(100, 9)
    s.means[3, 0] = np.inf
    with pytest.raises(L.PotrError):
        codec.encode(raster.to_device(s), synth.ring_cameras(2, 32, 32), codec.params(0.5))


def test_full_scene_sampled():
    """3M clustered splats with the full scene's 200 training cameras: the stream
    parses, every sampled splat's decoded position passes the precision test
    against the oracle's bound (or sits in a cap cell), and its decoded
    attributes are the oracle's dequantised values."""
    scene, cams = synth.workload_full_scene()
    print("codec full scene", scene.n, len(cams), flush=True)
    po, pg = _prm(0.5, 21)
    raw, order = codec.encode(raster.to_device(scene), cams, pg, want_order=True)
    order = order.cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(scene.n))
    comp = codec.compress(raw)
    dec = codec.decode(codec.decompress(comp))
    head = oc.HEADER.unpack_from(raw[: oc.HEADER.size].tobytes(), 0)
    lo, size = np.array(head[5:8]), head[8]
    _, size_o, _ = oc.grid(scene.means, 21)
    assert size == size_o and np.array_equal(lo, scene.means.min(0).astype(np.float64))
    rng = np.random.default_rng(0)
    k = rng.choice(scene.n, 20000, replace=False)
    i = order[k]
    thr2 = np.maximum(po["gamma"] ** 2, po["beta"] ** 2 * oc.nearest_eye_d2(scene.means[i], oc.camera_eyes(cams)))
    d2 = ((dec["means"][k].astype(np.float64) - scene.means[i]) ** 2).sum(1)
    cap = 0.75 * (size * 2.0 ** -21) ** 2
    assert np.all((d2 < thr2 * (1 + 1e-5)) | (d2 <= cap * (1 + 1e-5)))
    np.testing.assert_array_equal(dec["opacities"][k], oc.dequantise(oc.quantise(scene.opacities[i], po["sf_opac"]),
                                                                      po["sf_opac"], 0.25).astype(np.float32))
    np.testing.assert_array_equal(dec["scales"][k], oc.dequantise(oc.quantise(scene.scales[i], po["sf_scale"]),
                                                                  po["sf_scale"]).astype(np.float32))
    np.testing.assert_array_equal(dec["sh"][k, 1:], oc.dequantise(oc.quantise(scene.sh[i, 1:], po["sf_sh"]),
                                                                  po["sf_sh"]).astype(np.float32))
    np.testing.assert_array_equal(dec["sh"][k, 0], oc.dequantise(oc.quantise(scene.sh[i, 0], po["sf_sh"]),
                                                                 po["sf_sh"]).astype(np.float32))
    u = oc.unit_quat(scene.quats[i])
    np.testing.assert_array_equal(dec["quats"][k, 1:], oc.dequantise(np.floor(0.5 + u[:, 1:] * po["sf_rot"]),
                                                                     po["sf_rot"]).astype(np.float32))
    print(f"codec full scene: raw {raw.nbytes} B, zstd {len(comp)} B, {scene.n * 236 / len(comp):.1f}x vs 236 B/splat")
