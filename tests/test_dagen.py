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


@pytest.mark.parametrize("k,tw,th", [(3, 2, 2), (5, 4, 2), (9, 4, 4), (11, 8, 4), (17, 8, 8), (25, 16, 8)])
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
    tw, th, mi = emit_da.candidates(kw, 4, cache, kh, emit_da.LDS_BUDGETS[:1])[0]
    G = emit_da.lane_groups(cache[(kw, kh, tw, th, emit_da.MODES[mi])])
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



def test_blob_layout_as_the_kernel_reads_it(tmp_path):
    """The generated blob and table, decoded the way the kernel reads them
    (items, round boundaries, per-round chunk lengths and median offsets at
    the table's word offsets), equal the generator's schedules; every chunk
    length is a positive multiple of the chunk quantum and every item stays
    inside its entry."""
    import re
    info = emit_da.generate(str(tmp_path), workers=4)
    blob = np.fromfile(tmp_path / "mf_da_blob.bin", dtype="<u4")
    text = (tmp_path / "mf_da_table.h").read_text()
    assert int(re.search(r"MF_DA_BLOB_WORDS (\d+)", text).group(1)) == len(blob)
    assert int(re.search(r"MF_DA_GUARD (\d+)", text).group(1)) == dg.GUARD
    rows = [tuple(int(v) for v in m.group(1).split(","))
            for m in re.finditer(r"\{([0-9, ]+)\}", text)]
    assert len(rows) == info["entries"]
    seen = 0
    for (kw, kh, kz, es, tw, th, tz, T, G, mem, mode, c_off, nch, r_off, nr, l_off, p_off, o_off, arena) in rows:
        assert T == 1 and G >= 1 and c_off % 4 == 0 and mem in (0, 1) and mode in (0, 1)
        assert (kz, tz) == (1, 1) or (kz == kw == kh and mem == 0)
        rounds = blob[r_off:r_off + nr + 1]
        clen = blob[l_off:l_off + nr]
        phase = blob[p_off:p_off + nr]
        assert rounds[0] == 0 and rounds[-1] == nch and np.all(np.diff(rounds.astype(np.int64)) >= 0)
        assert np.all(clen >= dg.CHUNK) and np.all(clen % dg.CHUNK == 0) and np.all(clen <= 256)
        assert phase[0] == 0 and np.all(np.diff(phase.astype(np.int64)) >= 0)
        assert mem == 1 or (arena * es * G) <= emit_da.LDS_BYTES
        assert arena + 64 < dg.MAX_OFF
        if kz == 1 and (kw, kh, tw, th) in ((25, 25, 16, 16), (35, 35, 16, 8), (9, 31, 2, 8), (5, 3, 4, 2)) and seen < 6:
            S = dg.schedule(kw, tw, th, kh=kh, lanes=dg.LANES // G, rounds=emit_da.MODES[mode])
            assert np.array_equal(blob[c_off:c_off + 4 * nch].reshape(-1, 4), S.items)
            assert np.array_equal(rounds, S.rounds) and np.array_equal(clen, S.chunk_len)
            assert np.array_equal(phase, S.round_phase)
            assert np.array_equal(blob[o_off:o_off + tw * th], S.outputs) and arena == S.arena
            seen += 1
    assert seen >= 3
    # one global-memory entry per (square k, element size)
    glob = [r for r in rows if r[9] == 1]
    assert all(r[10] == 0 for r in glob)
    assert sorted(set((r[0], r[3]) for r in glob)) == sorted((k, es) for k in emit_da.KS for es in (2, 4))
    # one 3-D entry per (cubic k, element size), its schedule as schedule3 makes it
    box = [r for r in rows if r[2] > 1]
    assert sorted((r[0], r[3]) for r in box) == sorted((k, es) for k in emit_da.K3 for es in (2, 4))
    r = [r for r in box if r[0] == 7 and r[3] == 2][0]
    S = dg.schedule3(7, 7, 7, r[4], r[5], r[6], lanes=dg.LANES // r[8], rounds="asap")
    assert np.array_equal(blob[r[11]:r[11] + 4 * r[12]].reshape(-1, 4), S.items) and r[18] == S.arena
    # both round modes are offered for square windows
    sq = [r for r in rows if r[2] == 1 and r[0] == r[1] and r[9] == 0 and r[0] == 25]
    assert {r[10] for r in sq} == {0, 1}


@pytest.mark.parametrize("k,tw,th", [(5, 4, 2), (9, 4, 4), (13, 8, 8), (25, 16, 8)])
def test_sentinel_ties_exact_model(k, tw, th):
    """16-bit and 32-bit data that equals the sentinel value (the largest
    element) in most windows: the kernel's exact merge procedure (sentinel
    reads, clamped A index) still gives the oracle's median."""
    S = dg.schedule(k, tw, th)
    t = wl.tie_heavy_plane(17, 21, np.uint8, levels=3, seed=k)
    for dt, top in ((np.uint16, 0xFFFF), (np.uint32, 0xFFFFFFFF)):
        img = np.where(t == 0, 0, np.where(t == 1, top - 1, top)).astype(dt)
        np.testing.assert_array_equal(dg.run_schedule_on_image(S, img, exact_merge_path=True),
                                      oracle.median_filter(img, k))
    f = wl.float_specials_plane(13, 19, k)
    got = dg.run_schedule_on_image(S, f, exact_merge_path=True)
    assert got.view(np.uint32).tobytes() == oracle.median_filter(f, k).view(np.uint32).tobytes()


@pytest.mark.parametrize("box,tile", [((3, 3, 3), (2, 2, 2)), ((5, 5, 5), (4, 4, 2)), ((7, 7, 7), (4, 4, 4)),
                                      ((5, 3, 7), (2, 2, 4)), ((3, 5, 1), (2, 4, 1)), ((9, 9, 9), (8, 4, 4))])
def test_3d_schedule_matches_oracle(box, tile):
    """The 3-D recursion (faces, edges and corners around a box core, split
    along the longest tile side) reproduces the oracle's box median, with
    sorted chunks and with the kernel's exact merge procedure."""
    S = dg.schedule3(*box, *tile)
    assert (S.fw, S.fh, S.fd) == tuple(box[a] + tile[a] - 1 for a in range(3))
    for dt, seed in ((np.uint8, 1), (np.uint16, 2), (np.float32, 3)):
        if dt == np.float32:
            vol = np.stack([wl.float_specials_plane(9, 11, seed + z) for z in range(7)])
        else:
            vol = np.stack([wl.uniform_plane(9, 11, dt, seed + z) for z in range(7)])
        want = oracle.median_filter_3d(vol, *box)
        for exact in (False, True):
            got = dg.run_schedule_on_volume(S, vol, exact_merge_path=exact)
            assert got.view(np.uint8).tobytes() == want.view(np.uint8).tobytes(), (dt, exact)


@pytest.mark.parametrize("k,tw,th,mode", [(9, 4, 4, "asap"), (25, 16, 16, "asap"), (25, 16, 16, "phase"),
                                          (35, 16, 8, "asap"), (75, 16, 8, "asap")])
def test_items_as_the_kernel_assumes(k, tw, th, mode):
    """What the kernel takes for granted about the items: a round lists its
    sorts first and then its chunks by non-increasing search steps (a wave
    runs its first merging lane's step count), merge outputs start
    at multiples of ALIGN elements (each step writes one aligned run of four),
    chunks hold at most the round's chunk length, every merge read stays
    READ_PAST elements inside the arena after its window, and multi-line sort
    items gather lines that lie inside the footprint."""
    S = dg.schedule(k, tw, th, rounds=mode)
    m = (1 << dg.OFF_BITS) - 1
    fp = dg.GUARD + S.fw * S.fh
    assert S.arena % (2 * dg.ALIGN) == 0
    lines = 0
    for r in range(len(S.rounds) - 1):
        C = int(S.chunk_len[r])
        # sorts first, then chunks by non-increasing search steps: a wave's
        # first merging lane holds the largest step count of the wave
        w3 = S.items[S.rounds[r]:S.rounds[r + 1], 3].astype(np.int64)
        srt = (w3 & dg.SORT_FLAG) != 0
        assert not np.any(srt[1:] & ~srt[:-1])
        st = (w3[~srt] >> dg.STEP_SHIFT) & 15
        assert np.all(np.diff(st) <= 0)
        for w0, w1, w2, w3 in S.items[S.rounds[r]:S.rounds[r + 1]].astype(np.int64):
            if w3 & dg.SORT_FLAG:
                n, N, nl = w0 >> dg.OFF_BITS, w3 & 63, (w3 >> 6) & 7
                lstep = (w3 >> dg.LSTEP_SHIFT) & ((1 << dg.LSTEP_BITS) - 1)
                assert 1 <= nl and n * nl <= N <= dg.SORT_MAX
                last = (w0 & m) + (nl - 1) * lstep + (n - 1) * (w1 & m)
                assert dg.GUARD <= (w0 & m) and last < fp
                lines += nl > 1
                continue
            assert (w2 & m) % dg.ALIGN == 0 and 1 <= (w2 >> dg.OFF_BITS) <= C
            for off, n in ((w0 & m, w0 >> dg.OFF_BITS), (w1 & m, w1 >> dg.OFF_BITS)):
                assert off >= 1 and off + n + dg.READ_PAST <= S.arena
    if 2 * (k - th + 1) <= dg.SORT_MAX:
        assert lines > 0       # the core's short columns are sorted several to a network


def test_round_count_k25_16x16():
    """Rounds over the whole schedule: 12 barriers at k = 25, 16 x 16 (28
    with binary reductions from singletons, one recursion level at a time)."""
    assert dg.schedule(25, 16, 16, rounds="asap").stats["rounds"] <= 12


@pytest.mark.parametrize("k,tw,th,mode", [(5, 4, 2, "asap"), (9, 4, 4, "phase"), (13, 8, 8, "asap"),
                                          (25, 16, 8, "asap")])
def test_byte_elements_exact_model(k, tw, th, mode):
    """8-bit data held in 8-bit elements (the one-plane kernel's LDS form):
    the sentinel 0xff equals the largest data value, so windows full of 255
    need the clamped A index; the kernel's exact procedure gives the
    oracle's median, as it does with 16-bit elements."""
    S = dg.schedule(k, tw, th, rounds=mode)
    t = wl.tie_heavy_plane(19, 23, np.uint8, levels=3, seed=k)
    img = np.where(t == 0, 0, np.where(t == 1, 254, 255)).astype(np.uint8)
    want = oracle.median_filter(img, k)
    np.testing.assert_array_equal(dg.run_schedule_on_image(S, img, True, byte_elements=True), want)
    u = wl.uniform_plane(17, 29, np.uint8, seed=k)
    np.testing.assert_array_equal(dg.run_schedule_on_image(S, u, True, byte_elements=True),
                                  oracle.median_filter(u, k))
