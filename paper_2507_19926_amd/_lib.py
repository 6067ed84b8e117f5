"""ctypes binding of libmedfilt.so (include/medfilt.h): argument marshalling only.

The library must have been built (``__graft_entry__.build()`` or
``python -m paper_2507_19926_amd.build``); loading fails loudly otherwise.
There is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmedfilt.so")

MF_U8, MF_U16, MF_U32, MF_F32 = 0, 1, 2, 3
MF_BORDER_REPLICATE = 0
MF_VARIANT_AUTO, MF_VARIANT_OBLIVIOUS, MF_VARIANT_DATA_AWARE, MF_VARIANT_GLOBAL = 0, 1, 2, 3
MF_NOALLOC_MAX_IMAGES = 4096

STATUS = {
    0: "MF_OK", -1: "MF_ERR_NULL", -2: "MF_ERR_DIMS", -3: "MF_ERR_PITCH", -4: "MF_ERR_DTYPE",
    -5: "MF_ERR_K", -6: "MF_ERR_BORDER", -7: "MF_ERR_ALIAS", -8: "MF_ERR_NOMEM",
    -9: "MF_ERR_PLAN", -10: "MF_ERR_CONFIG", -11: "MF_ERR_WORKSPACE", -100: "MF_ERR_HIP",
}


class MfError(RuntimeError):
    def __init__(self, code: int, detail: str):
        self.code = code
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, detail))


class mf_options(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("group", ctypes.c_int32), ("form", ctypes.c_int32), ("rows", ctypes.c_int32)]


class mf_image(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("H", ctypes.c_int64),
                ("W", ctypes.c_int64), ("pitch_bytes", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("k", ctypes.c_int32), ("border", ctypes.c_int32)]


_lib = None


def lib():
    """Load libmedfilt.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmedfilt.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.median_filter.argtypes = [vp, vp, i64, i64, i64, i32, i32, i32, vp]
    L.median_filter.restype = i32
    L.median_filter_ex.argtypes = [vp, vp, i64, i64, i64, i32, i32, i32, ctypes.POINTER(mf_options), vp]
    L.median_filter_ex.restype = i32
    L.median_filter_planes.argtypes = [vp, vp, i64, i64, i64, i64, i64, i32, i32, i32, ctypes.POINTER(mf_options), vp]
    L.median_filter_planes.restype = i32
    L.median_filter_rect.argtypes = [vp, vp, i64, i64, i64, i64, i64, i32, i32, i32, i32,
                                     ctypes.POINTER(mf_options), vp]
    L.median_filter_rect.restype = i32
    L.mf_max_rect_side.argtypes = []
    L.mf_max_rect_side.restype = i32
    L.mf_query_rect_config.argtypes = [i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32)]
    L.mf_query_rect_config.restype = i32
    L.mf_peak_minmax.argtypes = [vp, i32, i32, vp]
    L.mf_peak_minmax.restype = i32
    L.mf_query_config.argtypes = [i32, i32, ctypes.POINTER(mf_options), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.mf_query_config.restype = i32
    L.mf_query_options.argtypes = [i32, i32, ctypes.POINTER(mf_options), ctypes.POINTER(mf_options)]
    L.mf_query_options.restype = i32
    L.median_filter_fwd_argmedian.argtypes = [vp, vp, vp, i64, i64, i64, i32, i32, vp]
    L.median_filter_fwd_argmedian.restype = i32
    L.median_filter_bwd_gather.argtypes = [vp, vp, vp, i64, i64, i64, i32, i32, vp]
    L.median_filter_bwd_gather.restype = i32
    pim = ctypes.POINTER(mf_image)
    L.mf_plan_create.argtypes = [pim, i32, ctypes.POINTER(vp)]
    L.mf_plan_create.restype = i32
    L.mf_plan_update.argtypes = [vp, pim, i32]
    L.mf_plan_update.restype = i32
    L.mf_plan_launch.argtypes = [vp, vp]
    L.mf_plan_launch.restype = i32
    L.mf_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.mf_plan_info.restype = i32
    L.mf_plan_destroy.argtypes = [vp]
    L.mf_plan_destroy.restype = None
    L.median_filter_batched.argtypes = [pim, i32, vp]
    L.median_filter_batched.restype = i32
    L.mf_global_workspace.argtypes = [i32, i32, i32, i32, i64, i64, i64, ctypes.POINTER(i64),
                                      ctypes.POINTER(i64), ctypes.POINTER(mf_options)]
    L.mf_global_workspace.restype = i32
    L.median_filter_global.argtypes = [vp, vp, i64, i64, i64, i64, i64, i32, i32, i32, i32, i32, vp, i64, vp]
    L.median_filter_global.restype = i32
    L.median_filter_3d.argtypes = [vp, vp, i64, i64, i64, i64, i64, i32, i32, i32, vp]
    L.median_filter_3d.restype = i32
    L.mf_max_k_3d.argtypes = []
    L.mf_max_k_3d.restype = i32
    L.median_filter_batched_noalloc.argtypes = [pim, i32, vp]
    L.median_filter_batched_noalloc.restype = i32
    L.mf_list_configs.argtypes = [i32, i32, ctypes.POINTER(mf_options), i32]
    L.mf_list_configs.restype = i32
    L.mf_max_k.argtypes = []
    L.mf_max_k.restype = i32
    L.mf_status_string.argtypes = [i32]
    L.mf_status_string.restype = ctypes.c_char_p
    L.mf_last_error.argtypes = []
    L.mf_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(code: int) -> None:
    if code != 0:
        raise MfError(code, lib().mf_last_error().decode())


def options(variant: int = MF_VARIANT_AUTO, tile=None, group: int = 0, form: int = 0,
            rows: int = 0) -> mf_options:
    o = mf_options()
    o.variant = variant
    if tile is not None:
        o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
    o.group = int(group)
    o.form = int(form)
    o.rows = int(rows)
    return o


def list_configs(dtype_code: int, k: int):
    """Every compiled (variant, tile_w, tile_h, group, form, rows) for dtype and k, default first."""
    L = lib()
    n = L.mf_list_configs(dtype_code, k, None, 0)
    if n < 0:
        check(n)
    arr = (mf_options * max(n, 1))()
    m = L.mf_list_configs(dtype_code, k, arr, n)
    if m < 0:
        check(m)
    return [(o.variant, o.tile_w, o.tile_h, o.group, o.form, o.rows) for o in arr[:n]]


def query_config(dtype_code: int, k: int, variant: int = MF_VARIANT_AUTO, tile=None):
    """(variant, tile_w, tile_h) the library runs for this dtype, k and request."""
    v, tw, th = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    o = options(variant, tile)
    check(lib().mf_query_config(dtype_code, k, ctypes.byref(o), ctypes.byref(v), ctypes.byref(tw),
                                ctypes.byref(th)))
    return v.value, tw.value, th.value


def global_workspace(dtype_code: int, k: int, planes: int, H: int, W: int, tile=None):
    """(slot_bytes, all_bytes, tile_w, tile_h, passes) of the global-memory
    form for planes of H x W."""
    slot, allb = ctypes.c_int64(), ctypes.c_int64()
    r = mf_options()
    tw, th = (0, 0) if tile is None else (int(tile[0]), int(tile[1]))
    check(lib().mf_global_workspace(dtype_code, k, tw, th, planes, H, W, ctypes.byref(slot),
                                    ctypes.byref(allb), ctypes.byref(r)))
    return slot.value, allb.value, r.tile_w, r.tile_h, r.rows


def query_options(dtype_code: int, k: int, variant: int = MF_VARIANT_AUTO, tile=None):
    """Resolved (variant, tile_w, tile_h, group, form, rows) the library runs."""
    o = options(variant, tile)
    r = mf_options()
    check(lib().mf_query_options(dtype_code, k, ctypes.byref(o), ctypes.byref(r)))
    return r.variant, r.tile_w, r.tile_h, r.group, r.form, r.rows


def query_rect_config(dtype_code: int, kw: int, kh: int):
    """(variant, tile_w, tile_h) median_filter_rect runs for this window."""
    v, tw, th = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().mf_query_rect_config(dtype_code, kw, kh, ctypes.byref(v), ctypes.byref(tw), ctypes.byref(th)))
    return v.value, tw.value, th.value
