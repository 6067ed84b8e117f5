"""Differentiable form on the GPU: argmedian and gradient bit-exact against
the oracle, central finite differences, and the torch.autograd.Function."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_19926_amd import workloads as wl
from paper_2507_19926_amd.ops import (MedianFilterFn, median_filter_argmedian,
                                      median_filter_backward)

pytestmark = pytest.mark.gpu


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


@pytest.mark.parametrize("k", [3, 7, 15, 31])
@pytest.mark.parametrize("kind", ["jitter", "ties"])
def test_forward_and_backward_match_oracle(k, kind):
    if kind == "jitter":
        x = wl.autograd_tensor(shape=(2, 3, 45, 77))
    else:
        x = wl.tie_heavy_plane(6 * 45, 77, np.float32, levels=3, seed=k).reshape(2, 3, 45, 77)
    g = wl.grad_out_like(x.shape, seed=k)
    xd = torch.from_numpy(x).cuda()
    y, idx = median_filter_argmedian(xd, k)
    gi = median_filter_backward(torch.from_numpy(g).cuda(), idx, k)
    torch.cuda.synchronize()
    y, idx, gi = y.cpu().numpy(), idx.cpu().numpy(), gi.cpu().numpy()
    for n in range(2):
        for c in range(3):
            v, i = oracle.argmedian_f32(x[n, c], k)
            assert np.array_equal(_bits(y[n, c]), _bits(v)), (n, c)
            assert np.array_equal(idx[n, c], i), (n, c)
            want = oracle.grad_f32(g[n, c], i)
            assert np.array_equal(_bits(gi[n, c]), _bits(want)), (n, c)


@pytest.mark.parametrize("k", [7, 15])
def test_autograd_function_and_conservation(k):
    x = torch.from_numpy(wl.autograd_tensor(shape=(1, 2, 64, 80))).cuda().requires_grad_(True)
    g = torch.from_numpy(wl.grad_out_like((1, 2, 64, 80), seed=3)).cuda()
    y = MedianFilterFn.apply(x, k)
    y.backward(g)
    torch.cuda.synchronize()
    xs = x.detach().cpu().numpy()
    for c in range(2):
        v, i = oracle.argmedian_f32(xs[0, c], k)
        assert np.array_equal(_bits(y.detach().cpu().numpy()[0, c]), _bits(v))
        want = oracle.grad_f32(g.cpu().numpy()[0, c], i)
        assert np.array_equal(_bits(x.grad.cpu().numpy()[0, c]), _bits(want))
    assert abs(float(x.grad.double().sum()) - float(g.double().sum())) < 1e-3


@pytest.mark.parametrize("k", [7, 15])
def test_central_finite_differences(k):
    """FD on the 2x1x32x32 slice of the autograd workload, filtered as its own
    image: perturb x[q] by +-1e-3, divide by the actual perturbation, compare
    with the gather gradient at coordinates where no other value of the
    (4r+1)^2 neighbourhood lies within 2*eps of x[q]."""
    full = wl.autograd_tensor(shape=(2, 3, 64, 64))
    xs = np.ascontiguousarray(full[:2, :1, :32, :32])
    g = wl.grad_out_like(xs.shape, seed=11).astype(np.float32)
    xd = torch.from_numpy(xs).cuda()
    _, idx = median_filter_argmedian(xd, k)
    grad = median_filter_backward(torch.from_numpy(g).cuda(), idx, k).cpu().numpy().astype(np.float64)
    eps = np.float32(1e-3)
    r = (k - 1) // 2
    H, W = 32, 32
    compared = 0
    rng = wl.rng(k)
    cand = [(n, qy, qx) for n in range(2) for qy in range(H) for qx in range(W)]
    rng.shuffle(cand)
    for (n, qy, qx) in cand:
        if compared >= 50:
            break
        v = xs[n, 0, qy, qx]
        y0, y1 = max(0, qy - 2 * r), min(H, qy + 2 * r + 1)
        x0, x1 = max(0, qx - 2 * r), min(W, qx + 2 * r + 1)
        nb = xs[n, 0, y0:y1, x0:x1].astype(np.float64)
        close = np.abs(nb - float(v)) < 2 * float(eps)
        if close.sum() > 1:
            continue
        xp = xs.copy(); xm = xs.copy()
        xp[n, 0, qy, qx] = v + eps
        xm[n, 0, qy, qx] = v - eps
        yp, _ = median_filter_argmedian(torch.from_numpy(xp).cuda(), k)
        ym, _ = median_filter_argmedian(torch.from_numpy(xm).cuda(), k)
        dy = (yp.cpu().numpy().astype(np.float64) - ym.cpu().numpy().astype(np.float64))
        fd = float((g.astype(np.float64) * dy).sum()) / (float(xp[n, 0, qy, qx]) - float(xm[n, 0, qy, qx]))
        assert abs(fd - grad[n, 0, qy, qx]) < 1e-3 * (1 + abs(fd)), (n, qy, qx, fd, grad[n, 0, qy, qx])
        compared += 1
    assert compared >= 50


def test_autograd_workload_first_plane():
    """The differentiable workload's shape (32x3x512x512 float32 with jitter):
    every output of plane 0 and sampled outputs of the last plane."""
    x = wl.autograd_tensor()
    g = wl.grad_out_like(x.shape)
    xd = torch.from_numpy(x).cuda()
    for k in (7, 15):
        y, idx = median_filter_argmedian(xd, k)
        gi = median_filter_backward(torch.from_numpy(g).cuda(), idx, k)
        torch.cuda.synchronize()
        v, i = oracle.argmedian_f32(x[0, 0], k)
        assert np.array_equal(_bits(y[0, 0].cpu().numpy()), _bits(v))
        assert np.array_equal(idx[0, 0].cpu().numpy(), i)
        assert np.array_equal(_bits(gi[0, 0].cpu().numpy()), _bits(oracle.grad_f32(g[0, 0], i)))
        last = x[31, 2]
        ys = wl.rng(k).integers(0, 512, 300); xs_ = wl.rng(k + 1).integers(0, 512, 300)
        assert np.array_equal(_bits(y[31, 2].cpu().numpy()[ys, xs_]),
                              _bits(oracle.median_points(last, k, ys, xs_)))
