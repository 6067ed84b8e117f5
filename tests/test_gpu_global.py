"""Global-memory multi-pass form on the GPU: the data-aware recursion with its
lists in a device workspace, run in passes of two recursion levels over slices
of tiles, bit-exact against the oracle for every dtype; workspaces from one
tile's slot (one tile per launch) to every tile at once; the library-allocated
path through the variant option; planes in one call."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_19926_amd import _lib
from paper_2507_19926_amd import workloads as wl
from paper_2507_19926_amd.ops import median_filter, median_filter_global

pytestmark = pytest.mark.gpu

DTYPES = [np.uint8, np.uint16, np.uint32, np.float32]


def _img(dt, H, W, seed):
    if dt == np.float32:
        return wl.float_specials_plane(H, W, seed)
    return wl.uniform_plane(H, W, dt, seed)


def _eq(a, b):
    return a.view(np.uint8).tobytes() == b.view(np.uint8).tobytes()


@pytest.mark.parametrize("k", [25, 51, 75])
@pytest.mark.parametrize("dtype", DTYPES)
def test_global_matches_oracle_sliced(k, dtype):
    H, W = 37 + k // 2, 53 + k
    img = _img(dtype, H, W, seed=7000 + k)
    x = torch.from_numpy(img).cuda()
    code = _lib.MF_U8 if dtype == np.uint8 else _lib.MF_U16 if dtype == np.uint16 else _lib.MF_U32 if dtype == np.uint32 else _lib.MF_F32
    slot, allb, tw, th, passes = _lib.global_workspace(code, k, 1, H, W)
    assert passes >= 2 and allb >= slot > 0
    want = oracle.median_filter(img, k)
    for budget in (slot, 3 * slot + 17, allb):
        got = median_filter_global(x, k, budget_bytes=budget)
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        assert _eq(g, want), (k, np.dtype(dtype).name, budget, int((g != want).sum()))


@pytest.mark.parametrize("k", [3, 9, 17, 33])
def test_global_small_k_and_ragged(k):
    for dtype, (H, W) in zip(DTYPES, ((5, 3), (29, 71), (64, 64), (1, 40))):
        img = _img(dtype, H, W, seed=k * 13 + H)
        got = median_filter_global(torch.from_numpy(img).cuda(), k, budget_bytes=1 << 20)
        torch.cuda.synchronize()
        assert _eq(got.cpu().numpy(), oracle.median_filter(img, k)), (k, np.dtype(dtype).name, H, W)


@pytest.mark.parametrize("k", [25, 75])
def test_global_planes_and_variant_option(k):
    """Three planes in one call (tiles numbered across planes, slices that
    straddle planes), and the variant option of median_filter, whose
    workspace the library allocates."""
    planes = np.stack([_img(np.uint8, 41, 67, seed=k + c) for c in range(3)])
    x = torch.from_numpy(planes).cuda()
    slot, _, _, _, _ = _lib.global_workspace(_lib.MF_U8, k, 3, 41, 67)
    got = median_filter_global(x, k, budget_bytes=5 * slot)
    via_opt = median_filter(x, k, variant=_lib.MF_VARIANT_GLOBAL)
    torch.cuda.synchronize()
    for c in range(3):
        want = oracle.median_filter(planes[c], k)
        assert _eq(got[c].cpu().numpy(), want), c
        assert _eq(via_opt[c].cpu().numpy(), want), c


@pytest.mark.parametrize("k", [25, 35, 75])
def test_global_with_lds_tiles(k):
    """Every root tile whose schedule also runs in LDS (the library's
    data-aware configurations for this k) gives the same result from the
    workspace."""
    img = _img(np.uint16, 50, 90, seed=k)
    want = oracle.median_filter(img, k)
    tiles = [(c[1], c[2]) for c in _lib.list_configs(_lib.MF_U16, k) if c[0] == _lib.MF_VARIANT_DATA_AWARE]
    assert tiles
    for tile in tiles:
        got = median_filter_global(torch.from_numpy(img).cuda(), k, tile=tile, budget_bytes=1 << 22)
        torch.cuda.synchronize()
        assert _eq(got.cpu().numpy(), want), tile
