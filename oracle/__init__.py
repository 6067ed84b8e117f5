"""Plain CPU oracle for the exact k x k median filter (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark load
this package. It shares nothing with the HIP library: the C source next to this
file (``medfilt_oracle.c``) is compiled with gcc into ``_build/liboracle.so``
and called through ctypes on host numpy arrays.

What it computes is the definition of the median filter (Sugy 2025, Section 1):
every output pixel is the rank-(k*k-1)/2 element of the k x k window around it,
with replicate borders and IEEE totalOrder for float32; the ``*_rect``
functions take a kw x kh window (odd sides) instead, and ``median_filter_3d``
a kx x ky x kz box over a volume. ``argmedian_f32`` and
``grad_f32`` add the index of the selected input pixel (lowest plane-flat index
among window pixels bit-equal to the median) and the gradient scatter in
ascending output order. Each function is pinned by the CPU oracle tests.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "medfilt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")

DTYPE_CODE = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1,
              np.dtype(np.uint32): 2, np.dtype(np.float32): 3}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP). Returns the library path."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.oracle_median_filter.argtypes = [vp, vp, i64, i64, i64, i32, i32, i64, i64, i32]
    lib.oracle_median_filter.restype = i32
    lib.oracle_median_points.argtypes = [vp, i64, i64, i64, i32, i32, vp, vp, i64, vp, i32]
    lib.oracle_median_points.restype = i32
    lib.oracle_median_filter_rect.argtypes = [vp, vp, i64, i64, i64, i32, i32, i32, i64, i64, i32]
    lib.oracle_median_filter_rect.restype = i32
    lib.oracle_median_points_rect.argtypes = [vp, i64, i64, i64, i32, i32, i32, vp, vp, i64, vp,
                                              i32]
    lib.oracle_median_points_rect.restype = i32
    lib.oracle_argmedian_f32.argtypes = [vp, vp, vp, i64, i64, i32, i64, i64, i32]
    lib.oracle_argmedian_f32.restype = i32
    lib.oracle_median_filter_3d.argtypes = [vp, vp, i64, i64, i64, i64, i64, i32, i32, i32, i32, i64, i64,
                                            i32]
    lib.oracle_median_filter_3d.restype = i32
    lib.oracle_grad_f32.argtypes = [vp, vp, vp, i64]
    lib.oracle_grad_f32.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _plane(img: np.ndarray) -> np.ndarray:
    if img.ndim != 2:
        raise ValueError("oracle works on one 2-D plane")
    if np.dtype(img.dtype) not in DTYPE_CODE:
        raise TypeError("unsupported dtype %s" % img.dtype)
    return np.ascontiguousarray(img)


def median_filter(img: np.ndarray, k: int, rows: tuple[int, int] | None = None,
                  nthreads: int = 0) -> np.ndarray:
    """k x k median of every pixel (replicate border). With ``rows=(a, b)``
    only rows a..b-1 are computed and returned (shape (b-a, W))."""
    img = _plane(img)
    H, W = img.shape
    a, b = (0, H) if rows is None else rows
    out = np.zeros_like(img)
    rc = _load().oracle_median_filter(_ptr(img), _ptr(out), H, W, img.strides[0],
                                      DTYPE_CODE[img.dtype], int(k), a, b, nthreads)
    if rc:
        raise ValueError("oracle_median_filter: bad argument (code %d)" % rc)
    return out[a:b].copy() if rows is not None else out


def median_points(img: np.ndarray, k: int, ys, xs, nthreads: int = 0) -> np.ndarray:
    """k x k median at the listed pixels."""
    img = _plane(img)
    H, W = img.shape
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    if ys.shape != xs.shape or ys.ndim != 1:
        raise ValueError("ys and xs must be 1-D of equal length")
    if len(ys) and (ys.min() < 0 or ys.max() >= H or xs.min() < 0 or xs.max() >= W):
        raise ValueError("point outside the image")
    out = np.zeros(len(ys), dtype=img.dtype)
    rc = _load().oracle_median_points(_ptr(img), H, W, img.strides[0],
                                      DTYPE_CODE[img.dtype], int(k), _ptr(ys), _ptr(xs),
                                      len(ys), _ptr(out), nthreads)
    if rc:
        raise ValueError("oracle_median_points: bad argument (code %d)" % rc)
    return out


def median_filter_rect(img: np.ndarray, kw: int, kh: int, rows: tuple[int, int] | None = None,
                       nthreads: int = 0) -> np.ndarray:
    """Median of the kw x kh window (kw columns, kh rows, both odd) of every
    pixel, replicate border; ``rows`` as in ``median_filter``."""
    img = _plane(img)
    H, W = img.shape
    a, b = (0, H) if rows is None else rows
    out = np.zeros_like(img)
    rc = _load().oracle_median_filter_rect(_ptr(img), _ptr(out), H, W, img.strides[0],
                                           DTYPE_CODE[img.dtype], int(kw), int(kh), a, b,
                                           nthreads)
    if rc:
        raise ValueError("oracle_median_filter_rect: bad argument (code %d)" % rc)
    return out[a:b].copy() if rows is not None else out


def median_filter_3d(vol: np.ndarray, kx: int, ky: int | None = None, kz: int | None = None,
                     slices: tuple[int, int] | None = None, nthreads: int = 0) -> np.ndarray:
    """Median of the kx x ky x kz box (odd sides; ky, kz default to kx) around
    every voxel of a (D, H, W) volume, each axis clamped (replicate border).
    With ``slices=(a, b)`` only slices a..b-1 are computed and returned."""
    ky = kx if ky is None else ky
    kz = kx if kz is None else kz
    if vol.ndim != 3:
        raise ValueError("median_filter_3d needs a (D, H, W) volume")
    if np.dtype(vol.dtype) not in DTYPE_CODE:
        raise TypeError("unsupported dtype %s" % vol.dtype)
    vol = np.ascontiguousarray(vol)
    D, H, W = vol.shape
    a, b = (0, D) if slices is None else slices
    out = np.zeros_like(vol)
    es = vol.dtype.itemsize       # contiguous: rows W*es apart, slices H*W*es apart
    rc = _load().oracle_median_filter_3d(_ptr(vol), _ptr(out), D, H, W, W * es, H * W * es,
                                         DTYPE_CODE[vol.dtype], int(kx), int(ky), int(kz), a, b, nthreads)
    if rc:
        raise ValueError("oracle_median_filter_3d: bad argument (code %d)" % rc)
    return out[a:b].copy() if slices is not None else out


def median_points_rect(img: np.ndarray, kw: int, kh: int, ys, xs,
                       nthreads: int = 0) -> np.ndarray:
    """kw x kh median at the listed pixels."""
    img = _plane(img)
    H, W = img.shape
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    if ys.shape != xs.shape or ys.ndim != 1:
        raise ValueError("ys and xs must be 1-D of equal length")
    if len(ys) and (ys.min() < 0 or ys.max() >= H or xs.min() < 0 or xs.max() >= W):
        raise ValueError("point outside the image")
    out = np.zeros(len(ys), dtype=img.dtype)
    rc = _load().oracle_median_points_rect(_ptr(img), H, W, img.strides[0],
                                           DTYPE_CODE[img.dtype], int(kw), int(kh), _ptr(ys),
                                           _ptr(xs), len(ys), _ptr(out), nthreads)
    if rc:
        raise ValueError("oracle_median_points_rect: bad argument (code %d)" % rc)
    return out


def argmedian_f32(img: np.ndarray, k: int, rows: tuple[int, int] | None = None,
                  nthreads: int = 0):
    """(median, idx) of a float32 plane; idx is int32 plane-flat."""
    img = _plane(img)
    if img.dtype != np.float32:
        raise TypeError("argmedian_f32 needs float32")
    H, W = img.shape
    a, b = (0, H) if rows is None else rows
    val = np.zeros_like(img)
    idx = np.full(img.shape, -1, dtype=np.int32)
    rc = _load().oracle_argmedian_f32(_ptr(img), _ptr(val), _ptr(idx), H, W, int(k),
                                      a, b, nthreads)
    if rc:
        raise ValueError("oracle_argmedian_f32: bad argument (code %d)" % rc)
    if rows is not None:
        return val[a:b].copy(), idx[a:b].copy()
    return val, idx


def grad_f32(grad_out: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Gradient of one plane: grad_in[idx[p]] += grad_out[p], p ascending."""
    g = np.ascontiguousarray(grad_out, dtype=np.float32)
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    if g.shape != ix.shape:
        raise ValueError("grad_out and idx differ in shape")
    out = np.zeros_like(g)
    rc = _load().oracle_grad_f32(_ptr(g), _ptr(ix), _ptr(out), g.size)
    if rc:
        raise ValueError("oracle_grad_f32: bad argument (code %d)" % rc)
    return out
