"""The codec's host side in libpotr.so (Sec. 4.5 decoder: zstd, the depth-first
parse of the octree bytes, dequantisation) against the oracle, on the CPU: the
library decodes bitstreams the oracle wrote, bit for bit."""
import ctypes as C

import numpy as np
import pytest

from oracle import codec as oc
from paper_2601_14821_amd import _lib as L
from paper_2601_14821_amd import codec, synth


def _scene(n, seed, dup=0):
    s = synth.random_scene(n, seed)
    if dup:
        s.means[-dup:] = s.means[:dup]
    return s


@pytest.mark.parametrize("n,seed,q,D,dup", [(1, 0, 0.5, 21, 0), (3, 1, 0.5, 3, 0), (500, 2, 0.5, 21, 3),
                                            (800, 3, 0.1, 6, 5), (300, 4, 1.0, 21, 0)])
def test_library_decodes_oracle_streams(n, seed, q, D, dup):
    s = _scene(n, seed, dup)
    cams = synth.ring_cameras(5, 64, 64)
    raw, _ = oc.encode_raw(s, cams, oc.params(q, D))
    got = codec.decode(raw)
    want = oc.decode_raw(raw)
    for k in ("means", "scales", "quats", "opacities"):
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)
    np.testing.assert_array_equal(got["sh"], want["sh"])
    assert got["sh_degree"] == 3


def test_library_zstd_matches_the_format():
    s = _scene(400, 5)
    raw, _ = oc.encode_raw(s, synth.ring_cameras(3, 32, 32), oc.params(0.5))
    comp = codec.compress(raw, 3)
    assert len(comp) < len(raw)
    assert codec.decompress(comp) == raw
    assert oc.zstd_decompress(comp) == raw          # a standard zstd frame
    assert codec.decompress(oc.zstd_compress(raw, 9)) == raw


def test_bad_streams_are_rejected():
    s = _scene(50, 6)
    raw, _ = oc.encode_raw(s, synth.ring_cameras(2, 32, 32), oc.params(0.5))
    with pytest.raises(L.PotrError) as e:
        codec.decode(raw[:-4])                       # truncated
    assert e.value.status == L.POTR_EINVAL
    bad = bytearray(raw)
    bad[0] ^= 0xFF                                   # magic
    with pytest.raises(L.PotrError):
        codec.decode(bytes(bad))
    bad = bytearray(raw)
    bad[oc.HEADER.size] = 0                          # the root turns into a leaf: bytes left over
    with pytest.raises(L.PotrError):
        codec.decode(bytes(bad))
    with pytest.raises(L.PotrError):
        codec.decompress(b"not a zstd frame")


def test_size_queries():
    b = C.c_size_t(0)
    L.call("potr_codec_max_bytes", 1000, 3, 21, C.byref(b))
    s = _scene(1000, 7, dup=2)
    raw, _ = oc.encode_raw(s, synth.ring_cameras(3, 32, 32), oc.params(0.5))
    assert len(raw) <= b.value
    with pytest.raises(L.PotrError):
        L.call("potr_codec_max_bytes", 10, 3, 22, C.byref(b))
    L.call("potr_codec_workspace_size", 1000, 3, 4, C.byref(b))
    assert b.value > 1000 * (8 + 8 + 8 + 4 + 4 + 2 + 4 * 55)
