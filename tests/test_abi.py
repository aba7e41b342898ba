"""Host-side checks of libpotr.so: it loads, exports every entry point that
include/potr.h declares, and rejects bad arguments before launching anything."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2601_14821_amd import _lib as L
from paper_2601_14821_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "potr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(potr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2601_14821_amd import build
        build.build()
    return L.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 9
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert n in L.SIGNATURES, f"{n} has no ctypes signature"
    # nothing but the C ABI is exported from the library's own code
    own = [s for s in exported if s.startswith("_ZN4potr")]
    assert not own, own[:5]


def test_abi_version(lib):
    assert lib.potr_abi_version() == 3


def test_struct_layouts():
    assert C.sizeof(L.potr_camera) == 72
    assert C.sizeof(L.potr_config) == 56
    assert L.PROJ_DTYPE.itemsize == 48
    # three (pointer, int64 stride, float weight) triples, each padded to 24 bytes
    assert C.sizeof(L.potr_outputs) == 72
    assert L.potr_outputs.importance_weight.offset == 64
    assert L.potr_outputs.fixed_point.offset == 68
    assert C.sizeof(L.potr_job) == 8 * 6 + 8 + 8 + 72 + 8 + 8 + 8 + 5 * 8


def _cfg(**kw):
    return L.make_config(synth.RenderSettings(**kw))


def _cams(n=1, w=64, h=48):
    return L.make_cameras(synth.ring_cameras(n, w, h))


def _status(name, *args):
    return getattr(L.lib(), name)(*args)


@pytest.mark.parametrize("kw, msg", [
    (dict(tile_w=12, tile_h=12), "tile"),
    (dict(lds_batch=100), "lds_batch"),
    (dict(lds_batch=1024), "lds_batch"),
    (dict(sh_degree=4), "sh_degree"),
    (dict(alpha_max=1.0), "alpha"),
    (dict(t_min=-1.0), "t_min"),
])
def test_project_rejects_bad_config(lib, kw, msg):
    st = _status("potr_project", 10, 1, _cams(), C.byref(_cfg(**kw)), 16, 16, 16, 16, 16, 16, 16, None)
    assert st == L.POTR_EINVAL
    assert msg in lib.potr_last_error().decode()


def test_rejects_bad_views_and_buffers(lib):
    cfg = _cfg()
    assert _status("potr_project", 10, 0, _cams(), C.byref(cfg), 16, 16, 16, 16, 16, 16, 16, None) == L.POTR_EINVAL
    cams = _cams(2)
    cams[1].width = 80
    assert _status("potr_project", 10, 2, cams, C.byref(cfg), 16, 16, 16, 16, 16, 16, 16, None) == L.POTR_EINVAL
    assert "same size" in lib.potr_last_error().decode()
    assert _status("potr_project", 10, 1, _cams(), C.byref(cfg), None, 16, 16, 16, 16, 16, 16, None) == L.POTR_EINVAL
    # misaligned record buffer
    assert _status("potr_project", 10, 1, _cams(), C.byref(cfg), 16, 16, 16, 16, 16, 20, 16, None) == L.POTR_EINVAL
    assert _status("potr_score", 10, 1, _cams(), C.byref(cfg), 16, 16, 16, 16, 16, 16, None, None, None, None,
                   None) == L.POTR_EINVAL


def test_workspace_too_small_is_capacity_error(lib):
    cfg = _cfg()
    need = L.bin_workspace_size(1000, 2, _cams(2), cfg)
    assert need > 0
    st = _status("potr_bin", 1000, 2, _cams(2), C.byref(cfg), 16, 16, need - 1, 16, 16, None)
    assert st == L.POTR_ECAPACITY
    sneed = L.sort_workspace_size(5000)
    assert sneed >= 8 * 5000   # the row lists: at most one 8-byte entry per pair
    st = _status("potr_sort", 1000, 2, _cams(2), C.byref(cfg), 16, 16, 16, need - 1, 16, 5000, 16, sneed, 16, 16,
                 None)
    assert st == L.POTR_ECAPACITY
    st = _status("potr_sort", 1000, 2, _cams(2), C.byref(cfg), 16, 16, 16, need, 16, 5000, 16, sneed - 1, 16, 16,
                 None)
    assert st == L.POTR_ECAPACITY
    st = _status("potr_sort", 1000, 2, _cams(2), C.byref(cfg), 16, 16, 16, need, 16, -1, 16, sneed, 16, 16, None)
    assert st == L.POTR_EINVAL


def test_workspace_sizes_grow(lib):
    cfg = _cfg()
    ws = lambda n, v, w=64, h=48: L.bin_workspace_size(n, v, L.make_cameras(synth.ring_cameras(v, w, h)), cfg)
    assert ws(10_000, 1) < ws(100_000, 1) < ws(100_000, 4)
    # the chunk table grows with the tile count
    assert ws(100_000, 1) < ws(100_000, 1, 1280, 720)


def test_new_entry_points_validate(lib):
    cfg = _cfg()
    out = C.c_void_p()
    # no jobs
    assert _status("potr_batch_create", None, 0, C.byref(cfg), 0.05, C.byref(out), None) == L.POTR_EINVAL
    # a job with a NULL buffer
    j = L.potr_job()
    j.N, j.V = 100, 1
    cams = _cams(1)
    j.cams = C.cast(cams, C.POINTER(L.potr_camera))
    arr = (L.potr_job * 1)(j)
    assert _status("potr_batch_create", arr, 1, C.byref(cfg), 0.05, C.byref(out), None) == L.POTR_EINVAL
    assert "NULL" in lib.potr_last_error().decode()
    # autotune without jobs
    assert _status("potr_autotune", None, 0, C.byref(cfg), 1, None, None, None, None, None) == L.POTR_EINVAL
    # operations on a batch that does not exist
    assert _status("potr_batch_run", None, None) == L.POTR_EINVAL
    assert _status("potr_batch_replay", None, None) == L.POTR_EINVAL
    assert _status("potr_batch_destroy", None) == L.POTR_OK
    # fused call without any output
    assert _status("potr_render_score", 10, 1, _cams(), C.byref(cfg), 16, 16, 16, None, None, None, None, None,
                   None) == L.POTR_EINVAL
    # squared error without a target
    assert _status("potr_render_score", 10, 1, _cams(), C.byref(cfg), 16, 16, 16, None, None, None, 16, None,
                   None) == L.POTR_EINVAL
    # backward with a workspace that is too small
    b = C.c_size_t(0)
    assert _status("potr_backward_workspace_size", 1000, 2, C.byref(b)) == L.POTR_OK
    assert b.value == 1000 * 2 * 9 * 4
    args = [1000, 2, _cams(2), C.byref(cfg)] + [16] * 12 + [16, b.value - 4] + [16] * 5 + [None]
    assert _status("potr_backward", *args) == L.POTR_ECAPACITY


def _render_score_out(out, target=None, N=100, V=2):
    return _status("potr_render_score_out", N, V, _cams(V), C.byref(_cfg()), 16, 16, 16, None, target,
                   C.byref(out), None)


@pytest.mark.parametrize("field, value, msg", [
    ("scores_weight", 0.0, "weight"), ("scores_weight", -1.0, "weight"), ("scores_weight", float("inf"), "weight"),
    ("scores_stride", -1, "stride"), ("scores_stride", 50, "stride")])
def test_outputs_are_validated(lib, field, value, msg):
    o = L.potr_outputs()
    o.scores, o.scores_weight = 16, 1.0
    setattr(o, field, value)
    assert _render_score_out(o) == L.POTR_EINVAL
    assert msg in lib.potr_last_error().decode()


def test_outputs_se_needs_target_and_some_output(lib):
    o = L.potr_outputs()
    assert _render_score_out(o) == L.POTR_EINVAL                       # nothing requested
    o.scores_se, o.se_weight = 16, 1.0
    assert _render_score_out(o) == L.POTR_EINVAL
    assert "target" in lib.potr_last_error().decode()
    # a job's outputs are checked by the batch the same way
    j = L.potr_job()
    j.N, j.V = 100, 1
    cams = _cams(1)
    j.cams = C.cast(cams, C.POINTER(L.potr_camera))
    j.means = j.scales = j.quats = j.opac = j.sh = 16
    j.out.importance, j.out.importance_weight, j.out.importance_stride = 16, 1.0, 7
    out = C.c_void_p()
    arr = (L.potr_job * 1)(j)
    assert _status("potr_batch_create", arr, 1, C.byref(_cfg()), 0.05, C.byref(out), None) == L.POTR_EINVAL
    assert "job 0" in lib.potr_last_error().decode() and "stride" in lib.potr_last_error().decode()


def test_fixed_point_mode_is_validated(lib):
    o = L.potr_outputs()
    o.scores, o.scores_weight = 16, 1.0
    o.fixed_point = 2
    assert _render_score_out(o) == L.POTR_EINVAL
    assert "fixed_point" in lib.potr_last_error().decode()
    # the jobs of one batch are all fixed point or none
    cams = _cams(1)
    jobs = []
    for k in range(3):
        j = L.potr_job()
        j.N, j.V = 100, 1
        j.cams = C.cast(cams, C.POINTER(L.potr_camera))
        j.means = j.scales = j.quats = j.opac = j.sh = 16
        j.out.scores, j.out.scores_weight = 16, 1.0
        j.out.fixed_point = 1 if k == 2 else 0
        jobs.append(j)
    arr = (L.potr_job * 3)(*jobs)
    out = C.c_void_p()
    assert _status("potr_batch_create", arr, 3, C.byref(_cfg()), 0.05, C.byref(out), None) == L.POTR_EINVAL
    assert "job 2" in lib.potr_last_error().decode() and "fixed point" in lib.potr_last_error().decode()
    assert _status("potr_fixed_to_float", None, 5, None, None) == L.POTR_EINVAL
    assert _status("potr_fixed_to_float", None, 0, None, None) == L.POTR_OK
