"""Torch-facing entry points. Torch supplies device memory and the stream;
every step of the filter runs in the HIP kernels of libmedfilt.so."""
from __future__ import annotations

import ctypes

import torch

from . import _lib

_DT = {torch.uint8: _lib.MF_U8, torch.uint16: _lib.MF_U16, torch.uint32: _lib.MF_U32,
       torch.float32: _lib.MF_F32}


def dtype_code(t: torch.dtype) -> int:
    try:
        return _DT[t]
    except KeyError:
        raise TypeError("median_filter supports uint8, uint16, uint32 and float32, not %s" % t)


def _stream_handle(dev: torch.device):
    return torch.cuda.current_stream(dev).cuda_stream


def median_filter(x: torch.Tensor, k: int, out: torch.Tensor | None = None,
                  variant: int = _lib.MF_VARIANT_AUTO, tile=None) -> torch.Tensor:
    """Exact k x k median (replicate border) of every (H, W) plane of x.

    x: a device tensor of shape (..., H, W) whose last dimension is contiguous;
    rows may be pitched (x.stride(-2) >= W). Leading dimensions are filtered
    plane by plane on the current stream.
    """
    if not x.is_cuda:
        raise ValueError("median_filter needs a GPU tensor")
    if x.dim() < 2:
        raise ValueError("median_filter needs (..., H, W)")
    code = dtype_code(x.dtype)
    if x.stride(-1) != 1:
        x = x.contiguous()
    H, W = x.shape[-2], x.shape[-1]
    if out is None:
        out = torch.empty(x.shape, dtype=x.dtype, device=x.device)
    if out.shape != x.shape or out.dtype != x.dtype or out.stride() != x.stride():
        raise ValueError("out must match x in shape, dtype and strides")
    es = x.element_size()
    pitch = x.stride(-2) * es
    stream = _stream_handle(x.device)
    opt = _lib.options(variant, tile)
    L = _lib.lib()
    planes_x = x.reshape(-1, H, W) if x.dim() > 2 else x.unsqueeze(0)
    planes_o = out.reshape(-1, H, W) if out.dim() > 2 else out.unsqueeze(0)
    if planes_x.data_ptr() != x.data_ptr() or planes_o.data_ptr() != out.data_ptr():
        raise ValueError("leading dimensions must be collapsible")
    for i in range(planes_x.shape[0]):
        _lib.check(L.median_filter_ex(planes_x[i].data_ptr(), planes_o[i].data_ptr(), H, W, pitch,
                                      code, int(k), _lib.MF_BORDER_REPLICATE, ctypes.byref(opt), stream))
    return out
