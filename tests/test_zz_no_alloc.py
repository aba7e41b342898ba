"""The no-allocation pruning select (potr_prune_select_noalloc, through the C
ABI) against the workspace entry point potr_prune_select: the same removal
mask and count, bit for bit, on two calls in a row, the second with fewer
splats (the shared scratch keeps the first call's contents)."""
import numpy as np
import pytest
import torch

from paper_2601_14821_amd import _lib as L
from paper_2601_14821_amd import prune

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    pool = np.float32([-3e-6, -2e-7, 0.0, 1e-9, 5e-8, 2.5e-7, 9.9e-7, 1e-6, 3e-5])
    dm = np.where(rng.random(n) < 0.4, rng.choice(pool, n), rng.normal(2e-7, 6e-7, n)).astype(np.float32)
    im = (rng.exponential(1.0, n) * (rng.random(n) < 0.9)).astype(np.float64)
    im = (im / im.sum() * 0.8).astype(np.float32)
    return torch.from_numpy(dm).cuda(), torch.from_numpy(im).cuda()


def _noalloc(dm, im, dmax, R, a=10.0):
    N = dm.numel()
    remove = torch.full((max(N, 1),), 7, dtype=torch.uint8, device="cuda")[:N]
    n = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    L.call("potr_prune_select_noalloc", N, L.ptr(dm), L.ptr(im), float(dmax), int(R), float(a), L.ptr(remove),
           L.ptr(n), L.stream_handle())
    return remove, n


def test_noalloc_select_equals_workspace_select():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    for n, seed in ((400_000, 21), (3_001, 22)):        # the second call is smaller
        dm, im = _inputs(n, seed)
        for R in (48, 5, 1):
            want, kw = prune.select(dm, im, 1e-6, R)
            got, kg = _noalloc(dm, im, 1e-6, R)
            torch.cuda.synchronize()
            print(f"n {n} remaining {R}: removed {int(kw.item())}", flush=True)
            assert int(kg.item()) == int(kw.item()) > 0
            np.testing.assert_array_equal(got.cpu().numpy(), want.cpu().numpy())


def test_noalloc_rejects_too_many_splats():
    st = L.lib().potr_prune_select_noalloc(1 << 31, 16, 16, 1e-6, 1, 10.0, 16, 16, None)
    assert st == L.POTR_EINVAL
    assert "2^31" in L.lib().potr_last_error().decode()
