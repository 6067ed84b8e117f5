"""Batched form on the GPU: one graph launch over mixed sizes, k and dtypes,
bit-exact against the oracle and against plain launches; plan reuse with
updated pointers (replayed several times, eager work in between)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_19926_amd import workloads as wl
from paper_2507_19926_amd.ops import BatchedPlan, median_filter, median_filter_batched

pytestmark = pytest.mark.gpu


def _mixed(n, seed, lo=17, hi=300, kmax=25):
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


def test_plan_matches_oracle_and_replays():
    imgs = _mixed(40, seed=7)
    xs = [torch.from_numpy(a).cuda() for a, _ in imgs]
    ks = [k for _, k in imgs]
    outs = [torch.empty_like(x) for x in xs]
    plan = BatchedPlan(xs, outs, ks)
    nb, blocks = plan.info()
    assert 1 <= nb <= 40 and blocks > 0
    wants = [oracle.median_filter(a, k) for a, k in imgs]
    for rep in range(3):
        for o in outs:
            o.zero_()
        plan.launch()
        torch.cuda.synchronize()
        for i, (o, w) in enumerate(zip(outs, wants)):
            assert o.cpu().numpy().tobytes() == w.tobytes(), (rep, i, ks[i], o.dtype, tuple(o.shape))
        # eager work between replays
        median_filter(xs[0], 3)
        torch.cuda.synchronize()
    # new pointers, same shapes
    xs2 = [torch.flip(x, dims=[1]).contiguous() for x in xs]
    outs2 = [torch.empty_like(x) for x in xs2]
    plan.update(xs2, outs2, ks)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for i, o in enumerate(outs2):
            want = oracle.median_filter(xs2[i].cpu().numpy(), ks[i])
            assert o.cpu().numpy().tobytes() == want.tobytes(), (rep, i)
    plan.close()


def test_one_shot_equals_plain_launches():
    imgs = _mixed(24, seed=3, kmax=75)
    xs = [torch.from_numpy(a).cuda() for a, _ in imgs]
    ks = [k for _, k in imgs]
    outs = median_filter_batched(xs, ks)
    torch.cuda.synchronize()
    for x, k, o in zip(xs, ks, outs):
        assert o.cpu().numpy().tobytes() == median_filter(x, k).cpu().numpy().tobytes(), (k, x.dtype)


def test_mixed_batch_workload_sampled():
    """The mixed-batch workload (256 images, sides 64..2048, k 3..25, u8/u16):
    one plan launch, sampled pixels of every image against the oracle."""
    batch = wl.mixed_batch()
    xs = [torch.from_numpy(a).cuda() for a, _ in batch]
    ks = [k for _, k in batch]
    outs = [torch.empty_like(x) for x in xs]
    plan = BatchedPlan(xs, outs, ks)
    plan.launch()
    torch.cuda.synchronize()
    g = wl.rng(99)
    for i, ((a, k), o) in enumerate(zip(batch, outs)):
        H, W = a.shape
        ys = np.concatenate([[0, H - 1], g.integers(0, H, 30)])
        xs_ = np.concatenate([[0, W - 1], g.integers(0, W, 30)])
        got = o.cpu().numpy()[ys, xs_]
        assert np.array_equal(got, oracle.median_points(a, k, ys, xs_)), (i, k, a.dtype, a.shape)
    plan.close()


def test_batched_data_aware_8_and_16_bit_apart():
    """Data-aware images of one k, tile and 16-bit element size but different
    dtypes run different kernels (16-bit data can equal the merge sentinel,
    8-bit data cannot): a batch mixing them, the 16-bit images full of the
    largest value, matches the oracle image by image."""
    from paper_2507_19926_amd import _lib
    k = 25
    assert _lib.query_config(_lib.MF_U16, k)[0] == _lib.MF_VARIANT_DATA_AWARE
    imgs = []
    for i in range(6):
        t = wl.tie_heavy_plane(40 + 3 * i, 57 + 5 * i, np.uint8, levels=3, seed=i)
        if i % 2:
            imgs.append(np.where(t == 0, 0, np.where(t == 1, 0xFFFE, 0xFFFF)).astype(np.uint16))
        else:
            imgs.append((t * 100).astype(np.uint8))
    xs = [torch.from_numpy(a).cuda() for a in imgs]
    outs = median_filter_batched(xs, [k] * len(xs))
    torch.cuda.synchronize()
    for i, (a, o) in enumerate(zip(imgs, outs)):
        assert o.cpu().numpy().tobytes() == oracle.median_filter(a, k).tobytes(), i
