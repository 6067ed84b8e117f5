"""The batched entry point that allocates nothing, against the plan-based
batched entry point and the oracle: two calls in a row on one stream, the
second with fewer and smaller images (the static job table keeps the first
call's records, which the second must overwrite correctly)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_19926_amd import workloads as wl
from paper_2507_19926_amd.ops import median_filter_batched, median_filter_batched_noalloc

pytestmark = pytest.mark.gpu


def _mixed(n, seed, lo, hi, kmax):
    g = wl.rng(seed)
    out = []
    for i in range(n):
        H = int(np.exp(g.uniform(np.log(lo), np.log(hi))))
        W = int(np.exp(g.uniform(np.log(lo), np.log(hi))))
        k = int(g.choice(np.arange(3, kmax + 1, 2)))
        dt = [np.uint8, np.uint16, np.uint32, np.float32][i % 4]
        img = wl.float_specials_plane(H, W, seed + i) if dt == np.float32 else wl.uniform_plane(H, W, dt, seed + i)
        out.append((img, k))
    return out


def _run(imgs):
    xs = [torch.from_numpy(a).cuda() for a, _ in imgs]
    ks = [k for _, k in imgs]
    got = [torch.full_like(x, 7) for x in xs]
    median_filter_batched_noalloc(xs, ks, got)
    want_plan = median_filter_batched(xs, ks)
    torch.cuda.synchronize()
    for i, ((a, k), g, w) in enumerate(zip(imgs, got, want_plan)):
        gb = g.cpu().numpy().tobytes()
        assert gb == w.cpu().numpy().tobytes(), ("plan", i, k, a.dtype, a.shape)
        assert gb == oracle.median_filter(a, k).tobytes(), ("oracle", i, k, a.dtype, a.shape)


def test_noalloc_matches_plan_twice_second_smaller():
    big = _mixed(150, seed=811, lo=9, hi=420, kmax=31)
    small = _mixed(37, seed=977, lo=3, hi=90, kmax=21)
    _run(big)
    _run(small)


def test_noalloc_back_to_back_without_sync():
    """Two calls queued on one stream without a host wait between them: the
    second call's records overwrite the first call's only after the first
    call's kernels have read them (stream order)."""
    a = _mixed(24, seed=1201, lo=20, hi=300, kmax=25)
    b = _mixed(9, seed=1301, lo=5, hi=120, kmax=15)
    xa = [torch.from_numpy(x).cuda() for x, _ in a]
    xb = [torch.from_numpy(x).cuda() for x, _ in b]
    oa = [torch.empty_like(x) for x in xa]
    ob = [torch.empty_like(x) for x in xb]
    median_filter_batched_noalloc(xa, [k for _, k in a], oa)
    median_filter_batched_noalloc(xb, [k for _, k in b], ob)
    torch.cuda.synchronize()
    for (img, k), o in list(zip(a, oa)) + list(zip(b, ob)):
        assert o.cpu().numpy().tobytes() == oracle.median_filter(img, k).tobytes(), (k, img.dtype, img.shape)
