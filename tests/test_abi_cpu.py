"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/*.h, and rejects bad arguments on the host before any GPU
work (every error code of the header)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2507_19926_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "sizeof")))


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = _declared_functions()
    assert "median_filter" in names and "mf_last_error" in names
    for n in names:
        assert hasattr(L, n), "missing export %s" % n


FAKE_SRC = 0x10000000
FAKE_DST = 0x20000000


def _call(src=FAKE_SRC, dst=FAKE_DST, H=16, W=16, pitch=16, dtype=0, k=3, border=0, opt=None):
    L = _lib.lib()
    o = ctypes.byref(opt) if opt is not None else None
    return L.median_filter_ex(src, dst, H, W, pitch, dtype, k, border, o, None)


@pytest.mark.parametrize("kw,code", [
    (dict(src=None), -1), (dict(dst=None), -1),
    (dict(H=0), -2), (dict(W=0), -2), (dict(H=-3), -2), (dict(W=2 ** 31), -2),
    (dict(pitch=15), -3), (dict(dtype=1, pitch=31), -3), (dict(dtype=2, pitch=62), -3),
    (dict(dtype=7), -4), (dict(dtype=-1), -4),
    (dict(dtype=1, src=FAKE_SRC + 1, pitch=32), -3), (dict(dtype=3, dst=FAKE_DST + 2, pitch=64), -3),
    (dict(k=4), -5), (dict(k=0), -5), (dict(k=-3), -5), (dict(k=77), -5),
    (dict(border=1), -6),
    (dict(dst=FAKE_SRC + 100), -7), (dict(dst=FAKE_SRC - 255 + 16), -7), (dict(dst=FAKE_SRC), -7),
    (dict(opt=_lib.options(variant=9)), -10),
    (dict(opt=_lib.options(tile=(3, 1))), -10),
    (dict(opt=_lib.options(tile=(4, 4)), k=3), -10),
])
def test_validation_codes(kw, code):
    assert _call(**kw) == code
    assert _lib.lib().mf_last_error().decode() != ""
    assert _lib.lib().mf_status_string(code).decode() not in ("", "unknown status")


def test_adjacent_buffers_are_not_aliases():
    # dst starts right after the last byte of src: no overlap, so validation
    # passes and the call reaches the launch (which fails without a GPU, or
    # is never reached when the oblivious table lacks the config).
    code = _call(dst=FAKE_SRC + 15 * 16 + 16, opt=_lib.options(variant=1, tile=(8, 8)), k=3)
    assert code == -10  # rejected on the config, after the alias check passed


def test_query_config():
    for dtype in range(4):
        v, tw, th = _lib.query_config(dtype, 1)
        assert (tw, th) == (1, 1)
    v, tw, th = _lib.query_config(0, 9)
    assert v == _lib.MF_VARIANT_OBLIVIOUS and tw >= 1 and th >= 1
    with pytest.raises(_lib.MfError):
        _lib.query_config(0, 8)
    with pytest.raises(_lib.MfError):
        _lib.query_config(5, 9)
    assert _lib.lib().mf_max_k() >= 75


def test_planes_entry_validation():
    """median_filter_planes validates on the host: plane count, plane stride
    (planes may not overlap or misalign) and the src/dst ranges over all
    planes; a plain image's checks still apply."""
    L = _lib.lib()

    def call(planes=3, stride=16 * 16, src=FAKE_SRC, dst=FAKE_DST, H=16, W=16, pitch=16, dtype=0, k=3):
        return L.median_filter_planes(src, dst, planes, stride, H, W, pitch, dtype, k, 0, None, None)

    assert call(planes=0) == -2
    assert call(planes=-1) == -2
    assert call(stride=16 * 16 - 1) == -3          # planes would overlap
    assert call(dtype=1, W=8, stride=16 * 16 + 1) == -3   # stride not a multiple of 2 bytes
    assert call(dst=FAKE_SRC + 2 * 256 + 100) == -7  # dst inside the src planes
    assert call(H=0) == -2 and call(k=4) == -5 and call(src=None) == -1
    # planes = 1 ignores the stride: the call passes validation and fails
    # later (no GPU) or not at all, but never with a stride error
    assert call(planes=1, stride=1) != -3


def test_rect_entry_validation():
    """median_filter_rect: both sides odd in [1, mf_max_rect_side()] for a
    rectangular window, the plain image and plane checks as in
    median_filter_planes."""
    L = _lib.lib()
    side = L.mf_max_rect_side()
    assert side >= 31

    def call(kw=5, kh=3, planes=1, stride=0, src=FAKE_SRC, dst=FAKE_DST, H=16, W=16, pitch=16, dtype=0,
             border=0, opt=None):
        o = ctypes.byref(opt) if opt is not None else None
        return L.median_filter_rect(src, dst, planes, stride, H, W, pitch, dtype, kw, kh, border, o, None)

    for kw, kh in ((4, 3), (3, 4), (0, 3), (3, -1), (side + 2, 3), (3, side + 2)):
        assert call(kw=kw, kh=kh) == -5, (kw, kh)
    assert call(kw=4, kh=4) == -5                    # square: the k x k rules
    assert call(kw=77, kh=77) == -5
    assert call(src=None) == -1 and call(H=0) == -2 and call(pitch=15) == -3
    assert call(dtype=9) == -4 and call(border=2) == -6 and call(dst=FAKE_SRC + 8) == -7
    assert call(planes=0) == -2 and call(planes=2, stride=255) == -3
    assert call(planes=3, stride=256, dst=FAKE_SRC + 600) == -7
    assert L.mf_last_error().decode() != ""
    # options: only the variant applies to a rectangular window
    assert call(opt=_lib.options(variant=9)) == -10
    assert call(opt=_lib.options(tile=(2, 2))) == -10
    assert call(opt=_lib.options(group=4)) == -10
    assert call(kw=25, kh=11, opt=_lib.options(variant=_lib.MF_VARIANT_OBLIVIOUS)) == -10   # no network


def test_rect_config_query():
    from paper_2507_19926_amd import build as mfbuild, emit_da
    for dtype in range(4):
        compiled = {tuple(c[:2]) for c in mfbuild.RECT_OBL_CONFIGS}
        for kw, kh in [w for w in ((29, 9), (3, 13), (23, 3), (27, 31)) if w not in compiled]:
            v, tw, th = _lib.query_rect_config(dtype, kw, kh)
            assert v == _lib.MF_VARIANT_DATA_AWARE and 1 <= tw <= kw and 1 <= th <= kh
            assert (tw, th) == emit_da.candidates(kw, 4, {}, kh, emit_da.LDS_BUDGETS[:1])[0][:2]
        # shapes with a compiled network run it
        for cfg in mfbuild.RECT_OBL_CONFIGS:
            assert _lib.query_rect_config(dtype, cfg[0], cfg[1]) == (_lib.MF_VARIANT_OBLIVIOUS, cfg[2], cfg[3])
    assert _lib.query_rect_config(0, 9, 9) == _lib.query_config(0, 9)
    for kw, kh in ((2, 3), (33, 1)):
        with pytest.raises(_lib.MfError):
            _lib.query_rect_config(0, kw, kh)
    with pytest.raises(_lib.MfError):
        _lib.query_rect_config(7, 3, 5)


def test_peak_diagnostic_validation():
    L = _lib.lib()
    assert L.mf_peak_minmax(None, 1, 1, None) == -2
    assert L.mf_peak_minmax(FAKE_DST, 0, 1, None) == -2
    assert L.mf_peak_minmax(FAKE_DST, 1, 0, None) == -2


def test_strip_form_listed_and_resolved():
    """The column-strip form exists for k = 3 only, is the last oblivious
    entry (never the default), and a request for it resolves to root tile
    1x1."""
    for dtype in range(4):
        cfgs = _lib.list_configs(dtype, 3)
        obl = [c for c in cfgs if c[0] == _lib.MF_VARIANT_OBLIVIOUS]
        assert obl[-1] == (_lib.MF_VARIANT_OBLIVIOUS, 1, 1, 4, 3, 16)
        assert cfgs[0][4] != 3
        assert all(c[4] != 3 for c in _lib.list_configs(dtype, 5))
    L = _lib.lib()
    v, tw, th = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    o = _lib.options(_lib.MF_VARIANT_OBLIVIOUS, (1, 1), 4, 3, 16)
    assert L.mf_query_config(0, 3, ctypes.byref(o), ctypes.byref(v), ctypes.byref(tw), ctypes.byref(th)) == 0
    assert (v.value, tw.value, th.value) == (_lib.MF_VARIANT_OBLIVIOUS, 1, 1)
    o = _lib.options(_lib.MF_VARIANT_OBLIVIOUS, None, 0, 3, 0)
    assert L.mf_query_config(0, 5, ctypes.byref(o), ctypes.byref(v), ctypes.byref(tw), ctypes.byref(th)) == -10
    o = _lib.options(_lib.MF_VARIANT_OBLIVIOUS, None, 0, 4, 0)
    assert L.mf_query_config(0, 3, ctypes.byref(o), ctypes.byref(v), ctypes.byref(tw), ctypes.byref(th)) == -10


def test_autograd_entry_validation():
    L = _lib.lib()
    A, B, C = 0x10000000, 0x20000000, 0x30000000
    assert L.median_filter_fwd_argmedian(None, B, C, 1, 8, 8, 3, 0, None) == -1
    assert L.median_filter_fwd_argmedian(A, B, C, 0, 8, 8, 3, 0, None) == -2
    assert L.median_filter_fwd_argmedian(A, B, C, 1, 1 << 16, 1 << 16, 3, 0, None) == -2
    assert L.median_filter_fwd_argmedian(A, B, C, 1, 8, 8, 2, 0, None) == -5
    assert L.median_filter_fwd_argmedian(A, B, C, 1, 8, 8, 3, 4, None) == -6
    assert L.median_filter_fwd_argmedian(A, A + 64, C, 1, 8, 8, 3, 0, None) == -7
    assert L.median_filter_bwd_gather(A, B, A + 4, 1, 8, 8, 3, 0, None) == -7
    assert L.median_filter_bwd_gather(A, None, C, 1, 8, 8, 3, 0, None) == -1


def test_plan_validation():
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.mf_plan_create(None, 1, ctypes.byref(h)) == -1
    arr = (_lib.mf_image * 2)()
    for i in range(2):
        arr[i].src, arr[i].dst = 0x10000000 + i * 0x100000, 0x20000000 + i * 0x100000
        arr[i].H, arr[i].W, arr[i].pitch_bytes, arr[i].dtype, arr[i].k, arr[i].border = 16, 16, 16, 0, 3, 0
    assert L.mf_plan_create(arr, 0, ctypes.byref(h)) == -2
    assert L.mf_plan_create(arr, 2, None) == -1
    arr[1].k = 1
    assert L.mf_plan_create(arr, 2, ctypes.byref(h)) == -5
    arr[1].k = 4
    assert L.mf_plan_create(arr, 2, ctypes.byref(h)) == -5
    arr[1].k = 3
    arr[1].dst = arr[0].src + 8       # overlaps another image's source
    assert L.mf_plan_create(arr, 2, ctypes.byref(h)) == -7
    assert not h.value
    assert L.mf_plan_launch(None, None) == -9
    assert L.mf_plan_update(None, arr, 2) == -9
    L.mf_plan_destroy(None)


def test_noalloc_batched_validation():
    """The no-allocation batched entry rejects bad lists on the host, before
    any GPU work: NULL list, empty list, more images than its static table,
    bad images and overlapping destinations."""
    L = _lib.lib()
    arr = (_lib.mf_image * 2)()
    for i in range(2):
        arr[i].src, arr[i].dst = 0x10000000 + i * 0x100000, 0x20000000 + i * 0x100000
        arr[i].H, arr[i].W, arr[i].pitch_bytes, arr[i].dtype, arr[i].k, arr[i].border = 16, 16, 16, 0, 3, 0
    assert L.median_filter_batched_noalloc(None, 1, None) == -1
    assert L.median_filter_batched_noalloc(arr, 0, None) == -2
    assert L.median_filter_batched_noalloc(arr, 4097, None) == -2
    assert "4096" in L.mf_last_error().decode()
    arr[1].k = 1
    assert L.median_filter_batched_noalloc(arr, 2, None) == -5
    arr[1].k = 3
    arr[1].dtype = 9
    assert L.median_filter_batched_noalloc(arr, 2, None) == -4
    arr[1].dtype = 0
    arr[1].dst = arr[0].src + 8
    assert L.median_filter_batched_noalloc(arr, 2, None) == -7


def test_global_form_validation():
    """Workspace query and the global-memory entry's host checks (no GPU
    work): sizes consistent with the tiles, every error before a launch."""
    L = _lib.lib()
    slot, allb, tw, th, passes = _lib.global_workspace(_lib.MF_U8, 75, 3, 4480, 6720)
    assert slot > 0 and slot % 256 == 0 and passes >= 2
    assert allb == slot * 3 * (-(-4480 // th)) * (-(-6720 // tw))
    s2, a2, tw2, th2, _ = _lib.global_workspace(_lib.MF_F32, 25, 1, 100, 100, tile=(16, 8))
    assert (tw2, th2) == (16, 8) and a2 == s2 * 13 * 7
    o = _lib.options()
    o.variant = _lib.MF_VARIANT_GLOBAL
    r = _lib.mf_options()
    assert L.mf_query_options(0, 51, ctypes.byref(o), ctypes.byref(r)) == 0 and r.variant == 3 and r.rows >= 2
    for args, code in (((0, 4, 0, 0), -5), ((0, 1, 0, 0), -5), ((9, 25, 0, 0), -4), ((0, 25, 3, 3), -10),
                       ((0, 25, 16, 0), -10), ((0, 25, 32, 32), -10)):
        sl, al = ctypes.c_int64(), ctypes.c_int64()
        assert L.mf_global_workspace(*args, 1, 64, 64, ctypes.byref(sl), ctypes.byref(al), None) == code, args
    A, B, WS = 0x10000000, 0x20000000, 0x30000000

    def g(ws=WS, nbytes=slot, k=75, src=A, dst=B):
        return L.median_filter_global(src, dst, 1, 0, 64, 64, 64, 0, k, 0, 0, 0, ws, nbytes, None)

    assert g(ws=None) == -1
    assert g(ws=WS + 16) == -11
    assert g(nbytes=100) == -11
    assert g(ws=A + 256) == -7
    assert g(k=1) == -5 and g(k=76) == -5
    assert g(src=None) == -1
    assert L.mf_status_string(-11).decode() != "unknown status"


def test_3d_entry_validation():
    """3-D box entry: host checks before any GPU work."""
    L = _lib.lib()
    A, B = 0x10000000, 0x20000000

    def c(src=A, dst=B, D=4, H=8, W=8, pitch=8, slice_=64, dtype=0, k=3, border=0):
        return L.median_filter_3d(src, dst, D, H, W, pitch, slice_, dtype, k, border, None)

    assert L.mf_max_k_3d() >= 15
    assert c(src=None) == -1
    assert c(D=0) == -2 and c(H=0) == -2
    assert c(pitch=7) == -3 and c(slice_=63) == -3 and c(dtype=1, pitch=16, slice_=129) == -3
    assert c(dtype=5) == -4
    assert c(k=4) == -5 and c(k=L.mf_max_k_3d() + 2) == -5
    assert c(border=2) == -6
    assert c(dst=A + 100) == -7
