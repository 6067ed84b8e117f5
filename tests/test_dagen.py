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
            assert S.chunks.shape[1] == 4 and len(S.outputs) == key[1] * key[2]

