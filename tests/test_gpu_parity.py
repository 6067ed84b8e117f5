"""GPU parity: the HIP kernels against the CPU oracle, bit-exact (selection
does no rounding, so every dtype must match exactly)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_19926_amd import _lib, build as mfbuild, workloads as wl
from paper_2507_19926_amd.ops import median_filter

pytestmark = pytest.mark.gpu

DTYPES = [np.uint8, np.uint16, np.uint32, np.float32]
TORCH_DT = {np.dtype(np.uint8): torch.uint8, np.dtype(np.uint16): torch.uint16,
            np.dtype(np.uint32): torch.uint32, np.dtype(np.float32): torch.float32}


def _dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _gpu(a: np.ndarray, k: int, **kw) -> np.ndarray:
    out = median_filter(_dev(a), k, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _img(dtype, H, W, seed):
    if np.dtype(dtype) == np.float32:
        return wl.float_specials_plane(H, W, seed)
    return wl.uniform_plane(H, W, dtype, seed)


def _eq(a, b):
    return a.tobytes() == b.tobytes()


def test_gpu_present():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    name = torch.cuda.get_device_properties(0).gcnArchName
    assert name.startswith("gfx950"), name


OBL = [(c[0], c[1], c[2], c[4], 2 if (len(c) > 5 and c[5]) else 1, c[3]) for c in mfbuild.OBL_CONFIGS]


@pytest.mark.parametrize("k,tw,th,nw,form,rows", OBL)
@pytest.mark.parametrize("dtype", DTYPES)
def test_oblivious_configs_match_oracle(k, tw, th, nw, form, rows, dtype):
    # ragged: several work-groups in each direction plus partial tiles
    H, W = 45 + 7 * k, 1100 + k
    img = _img(dtype, H, W, seed=k * 10 + tw)
    got = _gpu(img, k, variant=_lib.MF_VARIANT_OBLIVIOUS, tile=(tw, th), group=nw, form=form, rows=rows)
    want = oracle.median_filter(img, k)
    if not _eq(got, want):
        bad = np.argwhere(got.view(np.uint8).reshape(H, -1) != want.view(np.uint8).reshape(H, -1))
        pytest.fail("k=%d tile %dx%d waves %d %s: %d mismatching bytes, first at %s"
                    % (k, tw, th, nw, np.dtype(dtype).name, len(bad), bad[:5].tolist()))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (2, 3), (5, 700), (129, 65)])
def test_small_and_degenerate_shapes(dtype, shape):
    for k in (3, 5, 9, 15):
        img = _img(dtype, *shape, seed=sum(shape) + k)
        assert _eq(_gpu(img, k), oracle.median_filter(img, k)), (shape, k)


@pytest.mark.parametrize("dtype", DTYPES)
def test_k1_identity(dtype):
    img = _img(dtype, 33, 47, seed=1)
    assert _eq(_gpu(img, 1), img)


def test_pitched_rows():
    img = wl.uniform_plane(70, 301, np.uint8, seed=3)
    big = torch.zeros((70, 384), dtype=torch.uint8, device="cuda")
    big[:, :301] = _dev(img)
    view = big[:, :301]
    out_big = torch.full((70, 384), 7, dtype=torch.uint8, device="cuda")
    out = out_big[:, :301]
    median_filter(view, 5, out=out)
    torch.cuda.synchronize()
    assert _eq(out.cpu().numpy(), oracle.median_filter(img, 5))
    # padding bytes beyond W are untouched
    assert torch.all(out_big[:, 301:] == 7)


@pytest.mark.parametrize("dtype", DTYPES)
def test_tie_heavy(dtype):
    img = wl.tie_heavy_plane(101, 517, dtype, levels=3, seed=9)
    for k in (3, 7, 11):
        assert _eq(_gpu(img, k), oracle.median_filter(img, k))


def test_deterministic():
    img = wl.uniform_plane(257, 1031, np.uint16, seed=4)
    a = _gpu(img, 9)
    b = _gpu(img, 9)
    assert _eq(a, b)


def test_batch_of_planes():
    x = wl.rgb30_planes(H=97, W=613, seed=2)
    got = _gpu(x, 7)
    for c in range(3):
        assert _eq(got[c], oracle.median_filter(x[c], 7))


ALL_K = list(range(3, 76, 2))


@pytest.mark.parametrize("k", ALL_K)
def test_data_aware_every_k(k):
    H, W = 23 + k // 3, 41 + k
    for dtype in DTYPES:
        img = _img(dtype, H, W, seed=1000 + k)
        got = _gpu(img, k, variant=_lib.MF_VARIANT_DATA_AWARE)
        want = oracle.median_filter(img, k)
        assert _eq(got, want), (k, np.dtype(dtype).name, int((got != want).sum()))


@pytest.mark.parametrize("k", [17, 25, 35, 51, 75])
def test_data_aware_multi_workgroup(k):
    img = wl.rgb30_planes(H=150, W=333, seed=k)[0]
    assert _eq(_gpu(img, k, variant=_lib.MF_VARIANT_DATA_AWARE), oracle.median_filter(img, k))
    u16 = wl.uniform_plane(97, 211, np.uint16, seed=k)
    assert _eq(_gpu(u16, k), oracle.median_filter(u16, k))


@pytest.mark.parametrize("k", [3, 9, 15, 17])
def test_variants_agree(k):
    img = wl.uniform_plane(131, 517, np.uint16, seed=k)
    a = _gpu(img, k, variant=_lib.MF_VARIANT_OBLIVIOUS)
    b = _gpu(img, k, variant=_lib.MF_VARIANT_DATA_AWARE)
    assert _eq(a, b)


@pytest.mark.parametrize("k", list(wl.RGB30_KS))
def test_full_size_rgb30_sampled(k):
    """The benchmark's workload and launch configuration (30 MP RGB uint8,
    three planes on the current stream), checked at sampled pixels (corners,
    edges and random interior points) against the oracle computed one by one."""
    frame = wl.rgb30_planes()
    H, W = frame.shape[1:]
    got = _gpu(frame, k)
    g = wl.rng(k)
    ys = np.concatenate([[0, 0, H - 1, H - 1], g.integers(0, H, 400), np.zeros(50, int) + H - 1,
                         g.integers(0, H, 50)])
    xs = np.concatenate([[0, W - 1, 0, W - 1], g.integers(0, W, 400), g.integers(0, W, 50),
                         np.zeros(50, int) + W - 1])
    for c in range(3):
        want = oracle.median_points(frame[c], k, ys, xs)
        assert np.array_equal(got[c][ys, xs], want), (k, c)


def _check_rows_and_points(img, got, k, seed):
    """Full rows at the top, bottom and across a block boundary (every column,
    so both left/right edge blocks and interior blocks), plus random points."""
    H, W = img.shape
    for a, b in ((0, 24), (H // 2 - 12, H // 2 + 12), (H - 24, H)):
        want = oracle.median_filter(img, k, rows=(a, b))
        assert _eq(got[a:b], want), (k, a, b)
    g = wl.rng(seed)
    ys, xs = g.integers(0, H, 2000), g.integers(0, W, 2000)
    assert _eq(got[ys, xs], oracle.median_points(img, k, ys, xs))   # bit patterns (NaN payloads)


def _placed(img, dtype, placement):
    """(x, out) device views of img: a plain tensor, or views into bigger
    buffers starting 16 or 4 bytes in, or with a pitch that is not a multiple
    of 16 bytes."""
    H, W = img.shape
    es = np.dtype(dtype).itemsize
    tdt = TORCH_DT[np.dtype(dtype)]
    if placement == "aligned":
        x = _dev(img)
        out = torch.empty_like(x)
    else:
        lead = {"offset16": 16, "offset4": 4, "pitch_odd": 0}[placement] // es
        pitch = W + 16 // es + (1 if placement == "pitch_odd" else 0)
        n = H * pitch + lead + W
        xb = torch.zeros(n * es, dtype=torch.uint8, device="cuda").view(tdt)
        x = xb[lead:lead + H * pitch].view(H, pitch)[:, :W]
        x.copy_(_dev(img))
        ob = torch.zeros(n * es, dtype=torch.uint8, device="cuda").view(tdt)
        out = ob[lead:lead + H * pitch].view(H, pitch)[:, :W]
    return x, out


PLACEMENTS = ["aligned", "offset16", "offset4", "pitch_odd"]


@pytest.mark.parametrize("k", [3, 9, 17, 19])
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("placement", PLACEMENTS)
def test_persistent_staging_placements(k, dtype, placement):
    """The persistent form stages footprints with LDS-direct 16-byte loads
    when the rows are 16-byte aligned and falls back to element loads
    otherwise: an aligned plane, a view starting 16 bytes into a buffer, a
    view starting 4 bytes in (unaligned) and a pitch that is not a multiple of
    16 must all give the oracle's result. The plane is big enough for several
    blocks per work-group."""
    H, W = 1500, 2600
    img = _img(dtype, H, W, seed=k * 7 + len(placement))
    x, out = _placed(img, dtype, placement)
    median_filter(x, k, out=out)
    torch.cuda.synchronize()
    _check_rows_and_points(img, out.cpu().numpy(), k, seed=k)


STRIP = dict(variant=_lib.MF_VARIANT_OBLIVIOUS, tile=(1, 1), group=4, form=3, rows=16)

PLANE_CFGS = [dict(k=3), dict(k=3, **STRIP), dict(k=5), dict(k=9), dict(k=17), dict(k=25),
              dict(k=17, variant=_lib.MF_VARIANT_DATA_AWARE)]


@pytest.mark.parametrize("cfg", PLANE_CFGS, ids=lambda c: "_".join("%s%s" % kv for kv in c.items()))
@pytest.mark.parametrize("dtype", [np.uint8, np.float32])
def test_planes_one_launch(cfg, dtype):
    """Several planes in one median_filter_planes call (contiguous stack and
    planes with gaps between them) equal the oracle plane by plane; big enough
    for the persistent form to spread blocks over plane boundaries."""
    cfg = dict(cfg)
    k = cfg.pop("k")
    P, H, W = 3, 700, 1300
    imgs = np.stack([_img(dtype, H, W, seed=40 + p) for p in range(P)])
    want = [oracle.median_filter(imgs[p], k) for p in range(P)]
    got = _gpu(imgs, k, **cfg)
    for p in range(P):
        assert _eq(got[p], want[p]), (k, p)
    # planes with a gap of 3 rows plus 32 bytes between them (padded rows)
    tdt = TORCH_DT[np.dtype(dtype)]
    es = np.dtype(dtype).itemsize
    pitch = W + 32 // es
    stride = (H + 3) * pitch
    xb = torch.zeros(P * stride * es, dtype=torch.uint8, device="cuda").view(tdt)
    ob = torch.zeros(P * stride * es, dtype=torch.uint8, device="cuda").view(tdt)
    x = torch.as_strided(xb, (P, H, W), (stride, pitch, 1))
    out = torch.as_strided(ob, (P, H, W), (stride, pitch, 1))
    x.copy_(_dev(imgs))
    median_filter(x, k, out=out, **cfg)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    for p in range(P):
        assert _eq(res[p], want[p]), (k, p, "strided")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (7, 1), (2, 3), (17, 33), (63, 1023), (64, 1024),
                                   (65, 1025), (130, 2049), (301, 4099)])
def test_strip_form_k3(dtype, shape):
    """Column-strip form (k = 3): whole images against the oracle, from one
    pixel to several strips and work-groups in each direction with ragged
    right and bottom edges (partial chunks, lanes past the image)."""
    H, W = shape
    img = _img(dtype, H, W, seed=H * 31 + W)
    assert _eq(_gpu(img, 3, **STRIP), oracle.median_filter(img, 3))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("placement", PLACEMENTS)
def test_strip_form_placements(dtype, placement):
    """Column-strip form with 16-byte chunk loads and stores on aligned rows
    and element loads and stores otherwise."""
    H, W = 1500, 2600
    img = _img(dtype, H, W, seed=5 + len(placement))
    x, out = _placed(img, dtype, placement)
    median_filter(x, 3, out=out, **STRIP)
    torch.cuda.synchronize()
    assert _eq(out.cpu().numpy(), oracle.median_filter(img, 3))


@pytest.mark.parametrize("k,tw,th,nw,form,rows", [c for c in OBL if c[0] in (3, 9, 17)])
def test_oblivious_large_image_persistent(k, tw, th, nw, form, rows):
    """A plane big enough for the persistent launch (several blocks per
    work-group), checked at sampled pixels."""
    img = wl.uniform_plane(2100, 3000, np.uint8, seed=k + nw)
    got = _gpu(img, k, variant=_lib.MF_VARIANT_OBLIVIOUS, tile=(tw, th), group=nw, form=form, rows=rows)
    g = wl.rng(k)
    ys = np.concatenate([[0, 2099, 0, 2099], g.integers(0, 2100, 3000)])
    xs = np.concatenate([[0, 0, 2999, 2999], g.integers(0, 3000, 3000)])
    assert np.array_equal(got[ys, xs], oracle.median_points(img, k, ys, xs))


def test_peak_diagnostic_runs():
    """The min/max rate diagnostic runs and is deterministic (its output is a
    function of the thread index only)."""
    import ctypes
    out = torch.zeros(4 * 256, dtype=torch.int32, device="cuda")
    L = _lib.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(L.mf_peak_minmax(out.data_ptr(), 4, 3, s))
    a = out.clone()
    _lib.check(L.mf_peak_minmax(out.data_ptr(), 4, 3, s))
    torch.cuda.synchronize()
    assert torch.equal(a, out)


@pytest.mark.parametrize("k", [19, 23, 25, 31, 35, 45, 51, 63, 75])
def test_data_aware_every_listed_schedule(k):
    """Every compiled data-aware configuration of k (each root tile and both
    round modes: rounds per recursion level, rounds over the whole schedule),
    on images several tiles wide with ragged edges: 16-bit and 8-bit data
    full of the largest value (the merge sentinel's value: 8-bit data is
    held in bytes), uniform 8-bit data and 32-bit data."""
    t = wl.tie_heavy_plane(37 + k // 3, 61 + k, np.uint8, levels=3, seed=k)
    u16 = np.where(t == 0, 0, np.where(t == 1, 0xFFFE, 0xFFFF)).astype(np.uint16)
    u8sat = np.where(t == 0, 0, np.where(t == 1, 0xFE, 0xFF)).astype(np.uint8)
    u8 = _img(np.uint8, 29 + k // 2, 47 + k, seed=k + 1)
    f32 = _img(np.float32, 31, 40 + k, seed=k + 2)
    for img in (u16, u8sat, u8, f32):
        code = {np.dtype(np.uint8): _lib.MF_U8, np.dtype(np.uint16): _lib.MF_U16,
                np.dtype(np.float32): _lib.MF_F32}[img.dtype]
        cfgs = [c for c in _lib.list_configs(code, k) if c[0] == _lib.MF_VARIANT_DATA_AWARE]
        assert {c[4] for c in cfgs} == {1, 2}, cfgs
        want = oracle.median_filter(img, k)
        for c in cfgs:
            got = _gpu(img, k, variant=c[0], tile=(c[1], c[2]), group=c[3], form=c[4])
            assert _eq(got, want), (k, img.dtype.name, c, int((got != want).sum()))
