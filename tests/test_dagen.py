"""CPU checks of the data-aware schedule generator: schedules run by the
numpy model (both a sort-based chunk model and the exact merge-path
procedure the kernel follows) against the oracle, and the invariants the
kernel relies on (every access inside the LDS arena)."""
import numpy as np
import pytest

import oracle
from paper_2507_19926_amd import dagen as dg, emit_da
from paper_2507_19926_amd import workloads as wl

CASES = [(3, 1, 1), (3, 2, 2), (5, 2, 2), (5, 4, 2), (7, 4, 4), (9, 4, 4), (9, 8, 4),
         (13, 8, 8), (17, 8, 8), (25, 16, 8), (35, 16, 16)]


@pytest.mark.parametrize("k,tw,th", CASES)
def test_schedule_matches_oracle(k, tw, th):
    S = dg.schedule(k, tw, th)
    for dtype, shape, seed in ((np.uint8, (19, 43), 1), (np.uint16, (23, 17), 2), (np.uint32, (7, 9), 3)):
        img = wl.uniform_plane(*shape, dtype, seed=seed + k)
        np.testing.assert_array_equal(dg.run_schedule_on_image(S, img), oracle.median_filter(img, k))
    ties = wl.tie_heavy_plane(15, 22, np.uint8, levels=3, seed=k)
    np.testing.assert_array_equal(dg.run_schedule_on_image(S, ties), oracle.median_filter(ties, k))


@pytest.mark.parametrize("k,tw,th", [(3, 2, 2), (5, 4, 2), (9, 4, 4), (11, 8, 4)])
def test_schedule_exact_merge_path(k, tw, th):
    S = dg.schedule(k, tw, th)
    img = wl.tie_heavy_plane(9, 11, np.uint16, levels=4, seed=k)
    np.testing.assert_array_equal(dg.run_schedule_on_image(S, img, exact_merge_path=True),
                                  oracle.median_filter(img, k))


def test_merge_path_chunk_all_splits():
    g = wl.rng(0)
    for _ in range(200):
        na, nb = int(g.integers(0, 9)), int(g.integers(0, 9))
        A = np.sort(g.integers(0, 4, na)); B = np.sort(g.integers(0, 4, nb))
        full = np.sort(np.concatenate([A, B]))
        for r0 in range(na + nb):
            for n in range(1, na + nb - r0 + 1):
                assert list(dg._merge_path_chunk(A, B, r0, n)) == list(full[r0:r0 + n])


def test_library_tiles_fit_lds():
    cache = {}
    for k in (3, 17, 41, 75):
        for es in (2, 4):
            key = emit_da.choose_tile(k, es, cache)
            S = cache[key]
            assert S.arena * es <= emit_da.LDS_BYTES
            assert S.chunks.shape[1] == 4 and len(S.outputs) == key[2] * key[3]
    for kw, kh in ((31, 3), (1, 29), (17, 5)):
        for es in (2, 4):
            key = emit_da.choose_tile(kw, es, cache, kh)
            S = cache[key]
            assert S.arena * es <= emit_da.LDS_BYTES and (S.kw, S.rows) == (kw, kh)
            assert key[2] <= kw and key[3] <= kh and len(S.outputs) == key[2] * key[3]


@pytest.mark.parametrize("kw,kh,tw,th", [(5, 3, 2, 2), (3, 7, 2, 4), (9, 5, 4, 4), (7, 1, 4, 1),
                                         (1, 9, 1, 8), (15, 5, 8, 4), (11, 21, 8, 16), (31, 7, 16, 4)])
def test_rect_schedule_matches_oracle(kw, kh, tw, th):
    """The generated recursion for a rectangular window (separate horizontal
    and vertical radii) reproduces the oracle's kw x kh median, merged with
    sorts and with the kernel's merge-path chunks."""
    img = wl.uniform_plane(23, 29, np.uint8, seed=kw * 64 + kh)
    S = dg.schedule(kw, tw, th, kh=kh)
    assert (S.fw, S.fh) == (kw + tw - 1, kh + th - 1)
    want = oracle.median_filter_rect(img, kw, kh)
    np.testing.assert_array_equal(dg.run_schedule_on_image(S, img), want)
    if kw * kh <= 45:
        np.testing.assert_array_equal(dg.run_schedule_on_image(S, img, exact_merge_path=True), want)


@pytest.mark.parametrize("kw,kh", [(31, 1), (1, 31), (15, 5), (5, 15), (9, 31), (31, 29)])
def test_rect_lane_groups(kw, kh):
    """Small rectangular tiles run G to a work-group: G is a power of two
    that divides the lanes, G arenas of 32-bit elements fit half the LDS, and
    the schedule cut for G lane groups still computes the oracle's median."""
    cache = {}
    tw, th, _ = emit_da.candidates(kw, 4, cache, kh, emit_da.LDS_BUDGETS[:1])[0]
    G = emit_da.lane_groups(cache[(kw, kh, tw, th)])
    assert 1 <= G <= emit_da.MAX_GROUPS and dg.LANES % G == 0 and G & (G - 1) == 0
    S = dg.schedule(kw, tw, th, kh=kh, lanes=dg.LANES // G)
    assert G * S.arena * 4 <= emit_da.LDS_BYTES // 2
    if tw * th <= 16:
        assert G >= 8            # tiny tiles must not leave the work-group idle
    img = wl.uniform_plane(19, 37, np.uint16, seed=kw + kh)
    np.testing.assert_array_equal(dg.run_schedule_on_image(S, img), oracle.median_filter_rect(img, kw, kh))


def test_rect_windows_listed():
    ws = emit_da.windows()
    assert (3, 3) in ws and (75, 75) in ws and (31, 1) in ws and (1, 31) in ws
    assert all(kw % 2 and kh % 2 for kw, kh in ws) and len(ws) == len(set(ws))

