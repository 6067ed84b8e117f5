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
                  variant: int = _lib.MF_VARIANT_AUTO, tile=None, group: int = 0,
                  form: int = 0, rows: int = 0) -> torch.Tensor:
    """Exact k x k median (replicate border) of every (H, W) plane of x.

    x: a device tensor of shape (..., H, W) whose last dimension is contiguous;
    rows may be pitched (x.stride(-2) >= W). Leading dimensions are planes,
    each filtered on its own; equally spaced planes go to the library in one
    call (median_filter_planes), on the current stream.
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
    opt = _lib.options(variant, tile, group, form, rows)
    L = _lib.lib()
    planes_x = x.reshape(-1, H, W) if x.dim() > 2 else x.unsqueeze(0)
    planes_o = out.reshape(-1, H, W) if out.dim() > 2 else out.unsqueeze(0)
    if planes_x.data_ptr() != x.data_ptr() or planes_o.data_ptr() != out.data_ptr():
        raise ValueError("leading dimensions must be collapsible")
    n = planes_x.shape[0]
    if n == 0:
        return out
    # equally spaced planes (the usual case after collapsing) go in one call
    stride = planes_x.stride(0) * es if n > 1 else 0
    if n == 1 or stride >= (H - 1) * pitch + W * es:
        _lib.check(L.median_filter_planes(x.data_ptr(), out.data_ptr(), n, stride, H, W, pitch, code, int(k),
                                          _lib.MF_BORDER_REPLICATE, ctypes.byref(opt), stream))
        return out
    for i in range(n):
        _lib.check(L.median_filter_ex(planes_x[i].data_ptr(), planes_o[i].data_ptr(), H, W, pitch,
                                      code, int(k), _lib.MF_BORDER_REPLICATE, ctypes.byref(opt), stream))
    return out


def median_filter_global(x: torch.Tensor, k: int, out: torch.Tensor | None = None, tile=None,
                         budget_bytes: int | None = None) -> torch.Tensor:
    """The global-memory multi-pass form (median_filter_global) over the
    equally spaced (H, W) planes of x: the workspace is a torch allocation of
    min(budget_bytes, every tile at once) bytes, at least one tile's slot;
    the library runs the tiles in slices that fit it."""
    if not x.is_cuda:
        raise ValueError("median_filter_global needs a GPU tensor")
    code = dtype_code(x.dtype)
    if x.stride(-1) != 1:
        x = x.contiguous()
    H, W = x.shape[-2], x.shape[-1]
    if out is None:
        out = torch.empty(x.shape, dtype=x.dtype, device=x.device)
    if out.shape != x.shape or out.dtype != x.dtype or out.stride() != x.stride():
        raise ValueError("out must match x in shape, dtype and strides")
    es = x.element_size()
    px = x.reshape(-1, H, W) if x.dim() > 2 else x.unsqueeze(0)
    n = px.shape[0]
    stride = px.stride(0) * es if n > 1 else 0
    slot, allb, _, _, _ = _lib.global_workspace(code, int(k), n, H, W, tile)
    nbytes = allb if budget_bytes is None else max(slot, min(allb, int(budget_bytes)))
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=x.device)
    wp = (ws.data_ptr() + 255) // 256 * 256
    tw, th = (0, 0) if tile is None else (int(tile[0]), int(tile[1]))
    _lib.check(_lib.lib().median_filter_global(x.data_ptr(), out.data_ptr(), n, stride, H, W, x.stride(-2) * es,
                                               code, int(k), _lib.MF_BORDER_REPLICATE, tw, th, wp, nbytes,
                                               _stream_handle(x.device)))
    # ws goes back to torch's caching allocator on the stream the kernels
    # were enqueued on, so no later allocation can reuse it before they finish
    return out


def median_filter_3d(x: torch.Tensor, k: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Exact k x k x k box median (each axis clamped) of a (D, H, W) device
    volume, through median_filter_3d; rows may be pitched, slices equally
    spaced."""
    if not x.is_cuda:
        raise ValueError("median_filter_3d needs a GPU tensor")
    if x.dim() != 3:
        raise ValueError("median_filter_3d needs a (D, H, W) volume")
    code = dtype_code(x.dtype)
    if x.stride(-1) != 1:
        x = x.contiguous()
    if out is None:
        out = torch.empty(x.shape, dtype=x.dtype, device=x.device)
    if out.shape != x.shape or out.dtype != x.dtype or out.stride() != x.stride():
        raise ValueError("out must match x in shape, dtype and strides")
    D, H, W = x.shape
    es = x.element_size()
    _lib.check(_lib.lib().median_filter_3d(x.data_ptr(), out.data_ptr(), D, H, W, x.stride(1) * es,
                                           x.stride(0) * es, code, int(k), _lib.MF_BORDER_REPLICATE,
                                           _stream_handle(x.device)))
    return out


def median_filter_rect(x: torch.Tensor, kw: int, kh: int, out: torch.Tensor | None = None,
                       variant: int = _lib.MF_VARIANT_AUTO) -> torch.Tensor:
    """Exact median of the kw x kh window (kw columns, kh rows, both odd;
    replicate border) of every (H, W) plane of x, through
    median_filter_rect. Layout rules as in ``median_filter``; the planes must
    be equally spaced (one call)."""
    if not x.is_cuda:
        raise ValueError("median_filter_rect needs a GPU tensor")
    if x.dim() < 2:
        raise ValueError("median_filter_rect needs (..., H, W)")
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
    planes_x = x.reshape(-1, H, W) if x.dim() > 2 else x.unsqueeze(0)
    if planes_x.data_ptr() != x.data_ptr():
        raise ValueError("leading dimensions must be collapsible")
    n = planes_x.shape[0]
    if n == 0:
        return out
    stride = planes_x.stride(0) * es if n > 1 else 0
    opt = _lib.options(variant)
    _lib.check(_lib.lib().median_filter_rect(x.data_ptr(), out.data_ptr(), n, stride, H, W, pitch, code,
                                             int(kw), int(kh), _lib.MF_BORDER_REPLICATE, ctypes.byref(opt),
                                             _stream_handle(x.device)))
    return out


def median_filter_argmedian(x: torch.Tensor, k: int):
    """(y, idx) for a float32 tensor (..., H, W): the median and, per output
    pixel, the plane-local flat index of the input pixel it was taken from
    (lowest index among window pixels equal to the median)."""
    if not x.is_cuda or x.dtype != torch.float32 or x.dim() < 2:
        raise ValueError("median_filter_argmedian needs a float32 GPU tensor (..., H, W)")
    x = x.contiguous()
    H, W = x.shape[-2], x.shape[-1]
    planes = x.numel() // (H * W)
    y = torch.empty_like(x)
    idx = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    if planes:
        _lib.check(_lib.lib().median_filter_fwd_argmedian(
            x.data_ptr(), y.data_ptr(), idx.data_ptr(), planes, H, W, int(k),
            _lib.MF_BORDER_REPLICATE, _stream_handle(x.device)))
    return y, idx


def median_filter_backward(grad_out: torch.Tensor, idx: torch.Tensor, k: int) -> torch.Tensor:
    """Gradient of the median filter w.r.t. its input (deterministic gather)."""
    g = grad_out.contiguous()
    if g.dtype != torch.float32 or idx.dtype != torch.int32 or g.shape != idx.shape:
        raise ValueError("grad_out must be float32 and match idx (int32) in shape")
    H, W = g.shape[-2], g.shape[-1]
    planes = g.numel() // (H * W)
    gi = torch.empty_like(g)
    if planes:
        _lib.check(_lib.lib().median_filter_bwd_gather(
            g.data_ptr(), idx.contiguous().data_ptr(), gi.data_ptr(), planes, H, W, int(k),
            _lib.MF_BORDER_REPLICATE, _stream_handle(g.device)))
    return gi


class MedianFilterFn(torch.autograd.Function):
    """y = median_filter(x, k) with the gradient routed to the argmedian.

    forward saves the int32 argmedian; backward is the deterministic gather,
    bit-identical to a scatter of grad_out in ascending output order."""

    @staticmethod
    def forward(ctx, x, k):
        y, idx = median_filter_argmedian(x, k)
        ctx.save_for_backward(idx)
        ctx.k = int(k)
        return y

    @staticmethod
    def backward(ctx, grad_out):
        (idx,) = ctx.saved_tensors
        return median_filter_backward(grad_out, idx, ctx.k), None


def median_filter_ad(x: torch.Tensor, k: int) -> torch.Tensor:
    return MedianFilterFn.apply(x, k)


def _images(xs, outs, ks):
    if not (len(xs) == len(outs) == len(ks)):
        raise ValueError("xs, outs and ks differ in length")
    arr = (_lib.mf_image * len(xs))()
    for i, (x, o, k) in enumerate(zip(xs, outs, ks)):
        if x.dim() != 2 or x.stride(-1) != 1 or o.shape != x.shape or o.stride() != x.stride():
            raise ValueError("image %d: need 2-D row-major tensors with matching out" % i)
        arr[i].src, arr[i].dst = x.data_ptr(), o.data_ptr()
        arr[i].H, arr[i].W = x.shape
        arr[i].pitch_bytes = x.stride(0) * x.element_size()
        arr[i].dtype = dtype_code(x.dtype)
        arr[i].k = int(k)
        arr[i].border = _lib.MF_BORDER_REPLICATE
    return arr


class BatchedPlan:
    """A plan filtering many (H, W) images of mixed sizes, k and dtypes with
    one hipGraph launch (mf_plan_*). The tensors must stay alive while the
    plan is used; update() swaps in new tensors of the same shapes."""

    def __init__(self, xs, outs, ks):
        self._arr = _images(xs, outs, ks)
        self._keep = (list(xs), list(outs))
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().mf_plan_create(self._arr, len(self._arr), ctypes.byref(h)))
        self._h = h

    def info(self):
        b, n = ctypes.c_int32(), ctypes.c_int64()
        _lib.check(_lib.lib().mf_plan_info(self._h, ctypes.byref(b), ctypes.byref(n)))
        return b.value, n.value

    def launch(self, stream=None):
        dev = self._keep[0][0].device
        s = stream.cuda_stream if stream is not None else _stream_handle(dev)
        _lib.check(_lib.lib().mf_plan_launch(self._h, s))

    def update(self, xs, outs, ks):
        arr = _images(xs, outs, ks)
        _lib.check(_lib.lib().mf_plan_update(self._h, arr, len(arr)))
        self._arr, self._keep = arr, (list(xs), list(outs))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().mf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def median_filter_batched(xs, ks, outs=None):
    """One-shot batched filter (creates, launches and destroys a plan)."""
    if outs is None:
        outs = [torch.empty_like(x) for x in xs]
    arr = _images(xs, outs, ks)
    dev = xs[0].device
    _lib.check(_lib.lib().median_filter_batched(arr, len(arr), _stream_handle(dev)))
    return outs


def median_filter_batched_noalloc(xs, ks, outs):
    """Batched filter through the entry point that allocates nothing on the
    device (job records in the library's static per-GPU table); enqueued on
    the current stream, not waited for. `outs` must be given: this wrapper
    allocates nothing either."""
    arr = _images(xs, outs, ks)
    dev = xs[0].device
    _lib.check(_lib.lib().median_filter_batched_noalloc(arr, len(arr), _stream_handle(dev)))
    return outs
