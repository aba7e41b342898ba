"""Pins of the oracle's codec (Sec. 4.5: uniform quantisation, the octree with
its precision test, depth-first occupancy bytes, zstd), on the CPU."""
import json
import os

import numpy as np

from oracle import codec
from paper_2601_14821_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _centre_expr(expr, lo, size):
    # "lo + a size/b" or "lo + size/b"
    rest = expr.split("+", 1)[1].strip()
    num, den = rest.split("/")
    a = float(num.replace("size", "").strip() or 1.0)
    return lo + a * size / float(den)


def test_hand_worked_octree():
    g = json.load(open(os.path.join(HERE, "golden", "codec_octree.json")))
    m = np.array(g["means"], np.float32)
    for case in g["cases"]:
        thr2 = np.full(len(m), case["gamma"] ** 2)
        nodes, caps, order, depth, _, lo, size = codec.build_octree(m, thr2, g["D"])
        assert list(nodes) == case["nodes"], case["note"]
        assert caps == case["caps"] and order.tolist() == case["order"] and depth.tolist() == case["depths"]
        assert abs(size - 0.8 * (1 + 2 ** -20)) < 1e-7
        pos, d = codec.parse_octree(nodes, caps, g["D"], lo, size)
        want = np.array([[_centre_expr(e, lo[a], size) for a, e in enumerate(row)] for row in case["centres"]])
        np.testing.assert_allclose(pos, want, rtol=0, atol=1e-15)
        assert d.tolist() == case["depths"]


def _one_splat(mu, gamma, beta=0.0, eye=None, D=21):
    class S:
        pass
    s = S()
    s.n = 1
    s.means = np.array([mu], np.float32)
    s.scales = np.full((1, 3), 0.01, np.float32)
    s.quats = np.array([[1, 0, 0, 0]], np.float32)
    s.opacities = np.array([0.5], np.float32)
    s.sh = np.zeros((1, 1, 3), np.float32)
    eye = np.asarray(eye if eye is not None else [1e3, 0, 0], np.float32)
    cam = synth.look_at(eye, target=tuple(float(x) for x in mu))
    prm = dict(codec.params(0.5, D), gamma=gamma, beta=beta)
    return s, [cam], prm


def test_single_splat_depth_closed_form():
    # one splat: lo = mu, size = 1, the node at depth L is [mu, mu + 2^-L)^3, whose
    # centre lies 2^-(L+1) away per axis: d^2 = 0.75 4^-L. With gamma = 0.01 the
    # first L with 0.75 4^-L < 1e-4 is 7 (4^6 = 4096 < 7500 < 16384 = 4^7).
    mu = (0.25, -1.5, 2.0)
    s, cams, prm = _one_splat(mu, gamma=0.01)
    raw, info = codec.encode_raw(s, cams, prm)
    assert info["nodes"] == bytes([1] * 7 + [0]) and info["caps"] == []
    dec = codec.decode_raw(raw)
    want = (np.array(mu, np.float64) + 2.0 ** -8).astype(np.float32)
    np.testing.assert_array_equal(dec["means"][0], want)
    # a loose gamma keeps the root as the leaf (0.75 < gamma^2)
    s, cams, prm = _one_splat(mu, gamma=0.9)
    _, info = codec.encode_raw(s, cams, prm)
    assert info["nodes"] == bytes([0])
    # a tight one runs to the cap: 21 one-child nodes and a cap leaf
    s, cams, prm = _one_splat(mu, gamma=1e-9)
    _, info = codec.encode_raw(s, cams, prm)
    assert info["nodes"] == bytes([1] * 21 + [0]) and info["caps"] == [1]


def test_beta_term_uses_the_nearest_eye():
    # the camera eye 10 away: beta = 0.001 gives beta^2 d^2 = 1e-4, the same bound
    # as gamma = 0.01 above, whatever the (tiny) gamma
    mu = (0.0, 0.0, 0.0)
    s, cams, prm = _one_splat(mu, gamma=1e-6, beta=1e-3, eye=[0.0, 0.0, 10.0])
    eyes = codec.camera_eyes(cams)
    np.testing.assert_allclose(eyes[0], [0, 0, 10], atol=1e-5)
    raw, info = codec.encode_raw(s, cams, prm)
    assert abs(info["thr2"][0] - 1e-4) < 1e-9
    assert info["nodes"] == bytes([1] * 7 + [0])
    # a second, nearer camera (5 away) takes over: 0.25e-4 needs 4^L > 30000, L = 8
    cams2 = cams + [synth.look_at(np.array([5.0, 0.0, 0.0], np.float32), target=mu)]
    _, info = codec.encode_raw(s, cams2, prm)
    assert info["nodes"] == bytes([1] * 8 + [0])


def test_quantise_closed_forms():
    sf = 101.0
    x = np.array([0.123, -0.05, 0.0, 1.0, -1.0, 0.2], np.float32)
    # floor(1/2 + x SF): 12.92 -> 12 ... computed by hand from the FP32 values
    want = [int(np.floor(0.5 + float(v) * sf)) for v in x]
    assert want == [12, -5, 0, 101, -101, 20]
    assert codec.quantise(x, sf).tolist() == want
    # opacity is reconstructed a quarter step above the level
    assert codec.dequantise([12], sf, 0.25)[0] == 12.25 / 101.0
    assert codec.dequantise([-5], sf)[0] == -5.0 / 101.0
    # the hyperparameter table at q = 0.5
    p = codec.params(0.5)
    assert (p["sf_sh"], p["sf_opac"], p["sf_rot"], p["sf_scale"]) == (51.0, 101.0, 201.0, 2001.0)
    assert abs(p["gamma"] - 5.0 * 10 ** -5.5) < 1e-18 and abs(p["beta"] - 0.7e-4) < 1e-18


def _scene(n, seed, dup=0):
    s = synth.random_scene(n, seed)
    if dup:
        s.means[-dup:] = s.means[:dup]     # identical positions share a cap leaf
    return s


def test_round_trip_error_bounds():
    s = _scene(1500, 3, dup=4)
    cams = synth.ring_cameras(6, 64, 64)
    prm = codec.params(0.5)
    raw, info = codec.encode_raw(s, cams, prm)
    dec = codec.decode_raw(codec.zstd_decompress(codec.zstd_compress(raw)))
    order = info["order"]
    assert sorted(order.tolist()) == list(range(s.n))
    # uniform quantisation: |x~ - x| <= 1 / (2 SF) (+ the FP32 rounding of the output)
    d = np.abs(dec["scales"].astype(np.float64) - s.scales[order])
    assert d.max() <= 0.5 / prm["sf_scale"] + 1e-6
    d = np.abs(dec["sh"].astype(np.float64) - s.sh[order])
    assert d.max() <= 0.5 / prm["sf_sh"] + 1e-6
    # opacity: levels shifted a quarter step up, so x~ - x lies in [-1/4, 3/4] / SF
    d = dec["opacities"].astype(np.float64) - s.opacities[order]
    assert d.min() >= -0.25 / prm["sf_opac"] - 1e-6 and d.max() <= 0.75 / prm["sf_opac"] + 1e-6
    # rotations: the same rotation (|<q~, q>| ~ 1) with w >= 0, unit norm up to the steps
    u = codec.unit_quat(s.quats)[order]
    q = dec["quats"].astype(np.float64)
    assert np.all(q[:, 0] >= 0)
    # each kept component moves at most half a step; w follows from unit norm
    assert np.abs(q[:, 1:] - u[:, 1:]).max() <= 0.5 / prm["sf_rot"] + 1e-6
    assert np.abs(np.abs((q * u).sum(1)) - 1).max() < 2 * np.sqrt(3) / prm["sf_rot"]
    # positions: within the precision bound below the cap; at the cap within half a cell diagonal
    mu = s.means[order].astype(np.float64)
    d2 = ((dec["means"].astype(np.float64) - mu) ** 2).sum(1)
    dep = info["depth"][order]
    below = dep < prm["max_depth"]
    assert np.all(d2[below] < info["thr2"][order][below] * (1 + 1e-6) + 1e-12)
    cell = info["size"] * 2.0 ** -prm["max_depth"]
    assert np.all(d2[~below] <= 0.75 * cell * cell * (1 + 1e-6) + 1e-12)
    assert info["caps"] and max(info["caps"]) >= 2        # the duplicates share leaves


def test_octree_is_minimal_by_brute_force():
    # every leaf cell holds exactly its splats, passes the test (below the cap),
    # and its parent held another splat or failed the test for its one splat
    for seed, n, q, D in ((1, 200, 0.5, 21), (2, 300, 0.1, 8), (4, 60, 1.0, 5)):
        s = _scene(n, seed, dup=2)
        cams = synth.ring_cameras(4, 32, 32)
        prm = codec.params(q, D)
        _, info = codec.encode_raw(s, cams, prm)
        lo, size, X = codec.grid(s.means, D)
        m = s.means.astype(np.float64)
        thr2 = info["thr2"]
        for i in range(n):
            d = int(info["depth"][i])
            cell_i = X[i] >> (D - d)
            same = np.all((X >> (D - d)) == cell_i, axis=1)
            assert np.array_equal(info["cell"][i], cell_i)
            if d < D:
                assert same.sum() == 1
                c = lo + (cell_i + 0.5) * (size * 2.0 ** -d)
                assert ((m[i] - c) ** 2).sum() < thr2[i] * (1 + 1e-12)
            if d > 0:
                par = X[i] >> (D - d + 1)
                share = np.all((X >> (D - d + 1)) == par, axis=1).sum()
                cp = lo + (par + 0.5) * (size * 2.0 ** -(d - 1))
                assert share > 1 or ((m[i] - cp) ** 2).sum() >= thr2[i] * (1 - 1e-12)


def test_dc_coefficients_are_differential():
    s = _scene(400, 7)
    cams = synth.ring_cameras(3, 32, 32)
    prm = codec.params(0.5)
    raw, info = codec.encode_raw(s, cams, prm)
    head = codec.HEADER.unpack_from(raw, 0)
    n_nodes, n_caps = head[-2], head[-1]
    p = codec.HEADER.size + n_nodes + 4 * n_caps
    st = np.frombuffer(raw, "<i4", (7 + 3 * 16) * s.n, p).reshape(-1, s.n)
    direct = codec.quantise(s.sh[info["order"], 0, 0], prm["sf_sh"])
    assert st[7][0] == direct[0] and np.array_equal(np.cumsum(st[7].astype(np.int64)), direct)
    assert np.array_equal(st[10], codec.quantise(s.sh[info["order"], 1, 0], prm["sf_sh"]))   # AC as is


def test_zstd_round_trip():
    rng = np.random.default_rng(0)
    raw = rng.integers(0, 4, 100000, dtype=np.uint8).tobytes() + bytes(50000)
    comp = codec.zstd_compress(raw, 3)
    assert len(comp) < len(raw) // 2
    assert codec.zstd_decompress(comp) == raw
