"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws numbers: it holds none of the filter's arithmetic and
imports nothing from the library or from the oracle. Every generator uses
NumPy's PCG64 with an explicit seed, so the oracle and the GPU consume the same
bits.

The paper measures on 30-megapixel photographs whose 8-bit R, G and B planes
are filtered separately (Section 6). Those photographs are not available; the
generators below stand in for them with images of the same shape, bit depth and
planar layout (smooth gradients plus impulse noise), and add the dtype sweep,
the mixed batch and the differentiable workload that the library also serves.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 250719926

#: 30 MP frame of the paper's teaser, three planar channels
RGB30_H, RGB30_W = 4480, 6720
#: odd kernel diameters of the uint8 sweep
RGB30_KS = (3, 5, 7, 9, 11, 15, 17, 25, 35, 51, 75)
#: rectangular windows (kw columns, kh rows) timed on the same frame
RGB30_RECT = ((5, 3), (9, 5), (15, 5), (5, 15), (17, 9), (31, 3), (31, 9), (9, 31), (31, 1), (1, 31),
              (21, 13), (31, 29))
#: dtype sweep at 4096 x 4096
SWEEP_SIDE = 4096
SWEEP_KS = (3, 7, 17, 35, 75)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_plane(H: int, W: int, dtype, seed: int) -> np.ndarray:
    """Values uniform over the dtype's full range (float32: U[0, 1))."""
    g = rng(seed)
    dt = np.dtype(dtype)
    if dt == np.float32:
        return g.random((H, W), dtype=np.float32)
    hi = int(np.iinfo(dt).max) + 1
    return g.integers(0, hi, size=(H, W), dtype=np.uint64).astype(dt)


def small_512_u8() -> np.ndarray:
    """512 x 512 uint8, uniform 0..255 (the small parity/smoke case)."""
    return uniform_plane(512, 512, np.uint8, BASE_SEED + 0)


def rgb30_planes(H: int = RGB30_H, W: int = RGB30_W, noise: float = 0.05,
                 seed: int = BASE_SEED + 1) -> np.ndarray:
    """(3, H, W) uint8: smooth gradients R(x), G(y), B(x+y) with salt-and-pepper.

    Each plane gets an independent Bernoulli(noise) mask; masked samples become
    0 or 255 with probability 1/2 each.
    """
    g = rng(seed)
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    planes = np.empty((3, H, W), dtype=np.uint8)
    planes[0] = np.rint(255.0 * x / max(W - 1, 1)).astype(np.uint8)
    planes[1] = np.rint(255.0 * y / max(H - 1, 1)).astype(np.uint8)
    planes[2] = np.rint(255.0 * (x + y) / max(W + H - 2, 1)).astype(np.uint8)
    for c in range(3):
        mask = g.random((H, W)) < noise
        salt = g.random((H, W)) < 0.5
        planes[c][mask & salt] = 255
        planes[c][mask & ~salt] = 0
    return planes


def sweep_plane(dtype, side: int = SWEEP_SIDE, seed: int = BASE_SEED + 2) -> np.ndarray:
    """Single plane of the dtype sweep.

    uint16: uniform 0..65535; uint32: uniform over 32 bits; float32: normal
    (mean 0.5, std 0.2) with 2 % of the samples replaced by +10 or -10.
    """
    dt = np.dtype(dtype)
    g = rng(seed + {np.dtype(np.uint16): 0, np.dtype(np.uint32): 100,
                    np.dtype(np.float32): 200, np.dtype(np.uint8): 300}[dt])
    if dt == np.float32:
        v = g.normal(0.5, 0.2, size=(side, side)).astype(np.float32)
        out = g.random((side, side)) < 0.02
        sign = np.where(g.random((side, side)) < 0.5, np.float32(10.0), np.float32(-10.0))
        v[out] = sign[out]
        return v
    hi = int(np.iinfo(dt).max) + 1
    return g.integers(0, hi, size=(side, side), dtype=np.uint64).astype(dt)


def mixed_batch(n: int = 256, lo: int = 64, hi: int = 2048, kmax: int = 25,
                seed: int = BASE_SEED + 3):
    """n images with log-uniform sides in [lo, hi], odd k in 3..kmax, u8/u16.

    Returns a list of (image, k) pairs.
    """
    g = rng(seed)
    out = []
    ks = np.arange(3, kmax + 1, 2)
    for _ in range(n):
        H = int(round(float(np.exp(g.uniform(np.log(lo), np.log(hi))))))
        W = int(round(float(np.exp(g.uniform(np.log(lo), np.log(hi))))))
        k = int(ks[g.integers(0, len(ks))])
        dt = np.uint8 if g.random() < 0.5 else np.uint16
        hi_v = int(np.iinfo(dt).max) + 1
        img = g.integers(0, hi_v, size=(H, W), dtype=np.uint64).astype(dt)
        out.append((img, k))
    return out


def autograd_tensor(shape=(32, 3, 512, 512), seed: int = BASE_SEED + 4) -> np.ndarray:
    """float32 U[0, 1) plus 1e-7 * flat index, which makes most values distinct."""
    g = rng(seed)
    n = int(np.prod(shape))
    v = g.random(n, dtype=np.float32) + (np.float32(1e-7) * np.arange(n, dtype=np.float32))
    return v.astype(np.float32).reshape(shape)


def grad_out_like(shape, seed: int = BASE_SEED + 5) -> np.ndarray:
    """Gaussian std 1 upstream gradient."""
    return rng(seed).standard_normal(size=shape).astype(np.float32)


def tie_heavy_plane(H: int, W: int, dtype, levels: int, seed: int) -> np.ndarray:
    """Few distinct values, so windows hold many equal keys."""
    g = rng(seed)
    v = g.integers(0, levels, size=(H, W))
    dt = np.dtype(dtype)
    if dt == np.float32:
        return (v.astype(np.float32) * np.float32(0.25)).astype(np.float32)
    return v.astype(dt)


def float_specials_plane(H: int, W: int, seed: int) -> np.ndarray:
    """float32 mixing normal values with +-0, +-inf, NaNs with payloads and
    denormals, as raw bit patterns."""
    g = rng(seed)
    bits = g.integers(0, 2 ** 32, size=(H, W), dtype=np.uint64).astype(np.uint32)
    specials = np.array([0x00000000, 0x80000000, 0x7F800000, 0xFF800000,
                         0x7FC00000, 0xFFC00000, 0x7F800001, 0xFFBFFFFF,
                         0x00000001, 0x80000001, 0x007FFFFF, 0x807FFFFF,
                         0x3F800000, 0xBF800000], dtype=np.uint32)
    pick = g.random((H, W)) < 0.3
    bits[pick] = specials[g.integers(0, len(specials), size=int(pick.sum()))]
    return bits.view(np.float32)


def volume_u8(side: int = 256, seed: int = BASE_SEED + 5) -> np.ndarray:
    """(side, side, side) uint8 volume, uniform 0..255 (3-D box filter input)."""
    return rng(seed).integers(0, 256, size=(side, side, side), dtype=np.uint8)
