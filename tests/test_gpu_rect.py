"""GPU parity of the rectangular-window filter (median_filter_rect, kw
columns by kh rows, data-aware variant) against the CPU oracle, bit-exact."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_19926_amd import _lib, build as mfbuild, workloads as wl
from paper_2507_19926_amd.ops import median_filter, median_filter_rect

pytestmark = pytest.mark.gpu

DTYPES = [np.uint8, np.uint16, np.uint32, np.float32]
SHAPES = [(3, 1), (1, 3), (5, 3), (3, 5), (9, 3), (3, 9), (15, 5), (5, 15), (31, 1), (1, 31),
          (31, 29), (29, 31), (11, 21), (21, 11), (31, 3), (7, 27)]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _img(dtype, H, W, seed):
    if np.dtype(dtype) == np.float32:
        return wl.float_specials_plane(H, W, seed)
    return wl.uniform_plane(H, W, dtype, seed)


def _rect(a, kw, kh, variant=_lib.MF_VARIANT_AUTO):
    out = median_filter_rect(_dev(a), kw, kh, variant=variant)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _eq(a, b):
    return a.tobytes() == b.tobytes()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kw,kh", SHAPES)
def test_rect_matches_oracle(kw, kh, dtype):
    # several root tiles in each direction plus ragged partial tiles
    H, W = 41 + 3 * kh, 150 + 5 * kw
    img = _img(dtype, H, W, seed=kw * 100 + kh)
    got = _rect(img, kw, kh)
    want = oracle.median_filter_rect(img, kw, kh)
    if not _eq(got, want):
        bad = np.argwhere(got.view(np.uint8).reshape(H, -1) != want.view(np.uint8).reshape(H, -1))
        pytest.fail("%dx%d %s: %d mismatching bytes, first at %s"
                    % (kw, kh, np.dtype(dtype).name, len(bad), bad[:5].tolist()))


@pytest.mark.parametrize("kw", list(range(1, 32, 2)))
def test_every_rect_window(kw):
    """Each generated rectangular schedule once (the two element sizes share
    it), data-aware variant forced, dtype rotating over the shapes."""
    for i, kh in enumerate(range(1, 32, 2)):
        if kh == kw:
            continue
        dtype = DTYPES[(kw + i) % 4]
        img = _img(dtype, 37, 53, seed=kw * 1000 + kh)
        got = _rect(img, kw, kh, variant=_lib.MF_VARIANT_DATA_AWARE)
        assert _eq(got, oracle.median_filter_rect(img, kw, kh)), (kw, kh, dtype)


RECT_OBL = [tuple(c[:2]) for c in mfbuild.RECT_OBL_CONFIGS]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kw,kh", RECT_OBL)
def test_rect_oblivious_networks(kw, kh, dtype):
    """Every compiled rectangular network: several work-groups in each
    direction with ragged edges, against the oracle and the data-aware
    variant."""
    H, W = 61 + 5 * kh, 1100 + 3 * kw
    img = _img(dtype, H, W, seed=kw * 31 + kh)
    got = _rect(img, kw, kh, variant=_lib.MF_VARIANT_OBLIVIOUS)
    want = oracle.median_filter_rect(img, kw, kh)
    if not _eq(got, want):
        bad = np.argwhere(got.view(np.uint8).reshape(H, -1) != want.view(np.uint8).reshape(H, -1))
        pytest.fail("%dx%d %s: %d mismatching bytes, first at %s"
                    % (kw, kh, np.dtype(dtype).name, len(bad), bad[:5].tolist()))
    assert _eq(got, _rect(img, kw, kh, variant=_lib.MF_VARIANT_DATA_AWARE))


@pytest.mark.parametrize("kw,kh", [(5, 3), (3, 9), (15, 5), (5, 15)])
def test_rect_oblivious_large_image(kw, kh):
    """Enough blocks for the persistent form (rows in ranges across planes),
    uint8 and float32, three planes, sampled rows and points."""
    for dtype in (np.uint8, np.float32):
        planes = np.stack([_img(dtype, 2000, 3000, seed=s + kw) for s in range(3)])
        got = _rect(planes, kw, kh, variant=_lib.MF_VARIANT_OBLIVIOUS)
        for c in range(3):
            H, W = planes[c].shape
            for a, b in ((0, 16), (H // 2 - 8, H // 2 + 8), (H - 16, H)):
                assert _eq(got[c][a:b], oracle.median_filter_rect(planes[c], kw, kh, rows=(a, b))), (c, a)
            g = wl.rng(kw * 5 + kh + c)
            ys, xs = g.integers(0, H, 1500), g.integers(0, W, 1500)
            assert _eq(got[c][ys, xs], oracle.median_points_rect(planes[c], kw, kh, ys, xs)), c


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kw,kh", [(31, 1), (1, 31), (15, 5), (5, 15), (3, 1), (9, 31)])
def test_rect_lane_groups_across_workgroups(kw, kh, dtype):
    """Small tiles run many to a work-group (lane groups): images several
    work-groups wide and tall, with a partial last work-group and tile."""
    H, W = 75 + kh, 1500 + 3 * kw
    img = _img(dtype, H, W, seed=kw * 7 + kh)
    assert _eq(_rect(img, kw, kh), oracle.median_filter_rect(img, kw, kh)), (kw, kh)


@pytest.mark.parametrize("dtype", [np.uint8, np.float32])
@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (2, 3), (5, 700), (129, 65)])
def test_rect_small_and_degenerate_images(dtype, shape):
    for kw, kh in ((3, 1), (1, 5), (9, 3), (3, 31), (31, 5)):
        img = _img(dtype, *shape, seed=sum(shape) + kw + kh)
        assert _eq(_rect(img, kw, kh), oracle.median_filter_rect(img, kw, kh)), (shape, kw, kh)


def test_square_window_is_the_k_by_k_filter():
    img = wl.uniform_plane(90, 200, np.uint16, seed=5)
    for k in (1, 3, 9, 17, 25):
        a = _rect(img, k, k)
        b = median_filter(_dev(img), k)
        torch.cuda.synchronize()
        assert _eq(a, b.cpu().numpy()) and _eq(a, oracle.median_filter(img, k)), k


def test_rect_planes_and_pitch():
    """Three planes in one launch from a pitched, strided view; bytes outside
    the views stay untouched."""
    H, W, kw, kh = 77, 203, 11, 5
    planes = np.stack([wl.uniform_plane(H, W, np.uint8, seed=s) for s in range(3)])
    big = torch.zeros((3, H + 3, 256), dtype=torch.uint8, device="cuda")
    big[:, :H, :W] = _dev(planes)
    out_big = torch.full((3, H + 3, 256), 7, dtype=torch.uint8, device="cuda")
    median_filter_rect(big[:, :H, :W], kw, kh, out=out_big[:, :H, :W])
    torch.cuda.synchronize()
    ob = out_big.cpu().numpy()
    for c in range(3):
        assert _eq(ob[c, :H, :W], oracle.median_filter_rect(planes[c], kw, kh)), c
    assert (ob[:, H:, :] == 7).all() and (ob[:, :, W:] == 7).all()


def test_rect_tie_heavy():
    for dtype in (np.uint8, np.uint16, np.float32):
        img = wl.tie_heavy_plane(70, 90, dtype, levels=3, seed=4)
        for kw, kh in ((7, 3), (3, 13), (21, 9)):
            assert _eq(_rect(img, kw, kh), oracle.median_filter_rect(img, kw, kh)), (dtype, kw, kh)


@pytest.mark.parametrize("kw,kh", [(31, 9), (9, 31), (1, 31), (31, 1), (29, 9)])
def test_rect_full_size_rgb30_sampled(kw, kh):
    """30 MP RGB uint8, three planes in one launch, checked at corners,
    edges and random interior points against the oracle one by one."""
    frame = wl.rgb30_planes()
    H, W = frame.shape[1:]
    got = _rect(frame, kw, kh)
    g = wl.rng(kw * 64 + kh)
    ys = np.concatenate([[0, 0, H - 1, H - 1], g.integers(0, H, 400), np.zeros(50, int) + H - 1,
                         g.integers(0, H, 50)])
    xs = np.concatenate([[0, W - 1, 0, W - 1], g.integers(0, W, 400), g.integers(0, W, 50),
                         np.zeros(50, int) + W - 1])
    for c in range(3):
        assert np.array_equal(got[c][ys, xs], oracle.median_points_rect(frame[c], kw, kh, ys, xs)), c


def test_rect_rejects_bad_windows():
    x = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    side = _lib.lib().mf_max_rect_side()
    for kw, kh in ((2, 3), (3, 0), (side + 2, 1)):
        with pytest.raises(_lib.MfError):
            median_filter_rect(x, kw, kh)
    with pytest.raises(_lib.MfError):
        median_filter_rect(x, 25, 11, variant=_lib.MF_VARIANT_OBLIVIOUS)   # no network for 25x11


TORCH_DT = {np.dtype(np.uint8): torch.uint8, np.dtype(np.uint16): torch.uint16,
            np.dtype(np.uint32): torch.uint32, np.dtype(np.float32): torch.float32}


def _placed(img, placement):
    """(x, out) device views of img: a plain tensor, or views into bigger
    buffers starting 16 or 4 bytes in, or with a pitch that is not a
    multiple of 16 bytes."""
    H, W = img.shape
    es = img.dtype.itemsize
    tdt = TORCH_DT[img.dtype]
    if placement == "aligned":
        x = _dev(img)
        return x, torch.empty_like(x)
    lead = {"offset16": 16, "offset4": 4, "pitch_odd": 0}[placement] // es
    pitch = W + 16 // es + (1 if placement == "pitch_odd" else 0)
    n = H * pitch + lead + W
    xb = torch.zeros(n * es, dtype=torch.uint8, device="cuda").view(tdt)
    x = xb[lead:lead + H * pitch].view(H, pitch)[:, :W]
    x.copy_(_dev(img))
    ob = torch.zeros(n * es, dtype=torch.uint8, device="cuda").view(tdt)
    return x, ob[lead:lead + H * pitch].view(H, pitch)[:, :W]


@pytest.mark.parametrize("placement", ["aligned", "offset16", "offset4", "pitch_odd"])
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kw,kh", [(5, 3), (3, 9), (15, 5), (31, 9), (1, 31), (7, 21), (9, 21), (7, 31)])
def test_rect_oblivious_placements(kw, kh, dtype, placement):
    """Rectangular networks on a plane large enough for the persistent form,
    with rows 16-byte aligned (LDS-direct staging) or not (element loads)."""
    img = _img(dtype, 4000, 3000, seed=kw * 3 + kh)
    x, out = _placed(img, placement)
    median_filter_rect(x, kw, kh, out=out, variant=_lib.MF_VARIANT_OBLIVIOUS)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    H, W = img.shape
    for a, b in ((0, 12), (H // 2 - 6, H // 2 + 6), (H - 12, H)):
        assert _eq(got[a:b], oracle.median_filter_rect(img, kw, kh, rows=(a, b))), (a, b)
    g = wl.rng(kw + kh)
    ys, xs = g.integers(0, H, 2000), g.integers(0, W, 2000)
    assert _eq(got[ys, xs], oracle.median_points_rect(img, kw, kh, ys, xs))
