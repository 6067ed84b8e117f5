"""Emit the data-aware schedules (dagen) as a binary blob plus a host table.

For every odd k in 3..75 (square windows) and every rectangular window
k_w x k_h with odd sides up to RECT_MAX_SIDE, and each LDS element size
(2 bytes for 8/16-bit data, 4 bytes for 32-bit data), root tiles are chosen:
per LDS budget the one with the lowest estimated work per pixel (merge
outputs, co-rank searches, footprint loads) whose arena fits. Schedules depend
only on (k_w, k_h, t_w, t_h) and are stored once each; they are computed in a
process pool.

Outputs in the generated directory:
* mf_da_blob.bin   -- all schedules, little-endian uint32 words;
* mf_da_table.h    -- size of the blob and one entry per (k_w, k_h, element
  size, tile).
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import dagen

LDS_BYTES = 160 * 1024
KS = list(range(3, 76, 2))
TILE_CANDIDATES = [(t, t) for t in (1, 2, 4, 8, 16, 32)] + [(2 * t, t) for t in (1, 2, 4, 8, 16)]
# rectangular windows: both sides odd, 1..RECT_MAX_SIDE, sides different
RECT_MAX_SIDE = 31
RECT_SHAPES = [(kw, kh) for kw in range(1, RECT_MAX_SIDE + 1, 2)
               for kh in range(1, RECT_MAX_SIDE + 1, 2) if kw != kh]
# 3-D boxes (cubic k) and the root tiles tried for them
K3 = [3, 5, 7, 9, 11, 13, 15]
TILES3 = [(1, 1, 1), (2, 2, 2), (4, 2, 2), (4, 4, 2), (4, 4, 4), (8, 4, 4), (8, 8, 4)]


def tile_options(kw: int, kh: int) -> list:
    """Root tiles tried for a kw x kh window: power-of-two sides, t_w <= kw,
    t_h <= kh (a non-empty core); square windows use TILE_CANDIDATES,
    rectangular ones every such pair up to 32 x 32 (a thin window needs a
    thin tile: t_w = 1 for k_w = 1)."""
    if kw == kh:
        opts = TILE_CANDIDATES
    else:
        p2 = (1, 2, 4, 8, 16, 32)
        opts = [(tw, th) for tw in p2 for th in p2]
    return [(tw, th) for (tw, th) in opts if tw <= kw and th <= kh]


def _cost(S: dagen.Schedule) -> float:
    px = S.tw * S.th
    return (S.stats["per_pixel_outputs"] + 10.0 * S.stats["chunks"] / px + 8.0 * S.stats["sorts"] / px
            + S.fw * S.fh / px)


# LDS budgets of the candidates: 3, 2 and 1 work-groups per CU
LDS_BUDGETS = (LDS_BYTES // 3, LDS_BYTES // 2, LDS_BYTES)


# round modes (dagen.schedule): index 0 = rounds per recursion level, 1 =
# rounds over the whole schedule (fewer barriers, more LDS); the table stores
# the index, mf_options.form = index + 1
MODES = ("phase", "asap")


def _schedule_or_none(key):
    kw, kh, tw, th = key[:4]
    mode = key[4] if len(key) > 4 else dagen.ROUNDS
    try:
        return dagen.schedule(kw, tw, th, kh=kh, rounds=mode)
    except (AssertionError, RuntimeError):
        return None


def candidates(k: int, elem_bytes: int, cache: dict, kh: int | None = None,
               budgets=LDS_BUDGETS, modes=("asap",)):
    """(tile_w, tile_h, round mode index) options for a k x kh window (kh
    defaults to k), best first.

    One root tile per work-group. For each LDS budget (3, 2 or 1 work-groups
    per CU) and round mode, the root tile with the lowest estimated work whose
    arena fits; duplicates removed. More work-groups per CU hide more of the
    merge rounds' latency, larger tiles amortise more work, whole-schedule
    rounds need fewer barriers but more LDS: the tuner decides."""
    kh = k if kh is None else kh
    out = []
    for mode in modes:
        mi = MODES.index(mode)
        for budget in budgets:
            best = None
            for (tw, th) in tile_options(k, kh):
                key = (k, kh, tw, th, mode)
                if key not in cache:
                    cache[key] = _schedule_or_none(key)
                S = cache[key]
                if S is None or S.arena * elem_bytes > budget:
                    continue
                c = _cost(S)
                if best is None or c < best[0]:
                    best = (c, tw, th)
            if best is not None and (best[1], best[2], mi) not in out:
                out.append((best[1], best[2], mi))
    assert out, k
    # largest tile (least work) first, whole-schedule rounds first among equals:
    # the default without a tuned table
    out.sort(key=lambda c: (-c[0] * c[1], -c[2]))
    return out


MAX_GROUPS = 32      # lane groups per work-group: at least 16 lanes each


def lane_groups(S: dagen.Schedule, elem_bytes: int = 4) -> int:
    """Lane groups G for a small root tile: enough groups that a group's
    kDaThreads/G lanes are at least half the schedule's mean items per round
    (each lane then runs one or two items a round, and fewer idle), a power
    of two <= MAX_GROUPS, and G arenas within half the LDS (two work-groups
    per CU)."""
    rounds = max(1, len(S.rounds) - 1)
    mean = max(1.0, len(S.items) / rounds)
    g = 1
    while g < MAX_GROUPS and dagen.LANES / (2 * g) >= mean / 2:
        g *= 2
    while g > 1 and g * S.arena * elem_bytes > LDS_BYTES // 2:
        g //= 2
    return g


def global_tile(k: int, cache: dict):
    """Root tile of the global-memory form for a square k x k window: the
    lowest estimated work among the candidates whose arena the item format
    can address, with no LDS budget (the lists live in a device workspace);
    rounds per recursion level (each pass then holds two whole levels)."""
    best = None
    for (tw, th) in tile_options(k, k):
        key = (k, k, tw, th, "phase")
        if key not in cache:
            cache[key] = _schedule_or_none(key)
        S = cache[key]
        if S is None:
            continue
        c = _cost(S)
        if best is None or c < best[0]:
            best = (c, tw, th)
    return best[1], best[2]


def _cost3(S: dagen.Schedule) -> float:
    px = S.tw * S.th * S.tz
    return (S.stats["per_pixel_outputs"] + 10.0 * S.stats["chunks"] / px + 8.0 * S.stats["sorts"] / px
            + S.fw * S.fh * S.fd / px)


def tile3(k: int, elem_bytes: int, cache3: dict):
    """Root tile of the 3-D k x k x k box: the lowest estimated work among
    TILES3 whose LDS arena fits one work-group per CU."""
    best = None
    for t in TILES3:
        if max(t) > k:
            continue
        if t not in cache3.setdefault(k, {}):
            try:
                cache3[k][t] = dagen.schedule3(k, k, k, *t, rounds="asap")
            except (AssertionError, RuntimeError):
                cache3[k][t] = None
        S = cache3[k][t]
        if S is None or S.arena * elem_bytes > LDS_BYTES:
            continue
        c = _cost3(S)
        if best is None or c < best[0]:
            best = (c, t)
    return best[1]


def choose_tile(k: int, elem_bytes: int, cache: dict, kh: int | None = None):
    kh = k if kh is None else kh
    tw, th, mi = candidates(k, elem_bytes, cache, kh)[0]
    return (k, kh, tw, th, MODES[mi])


def windows() -> list:
    """Every (k_w, k_h) the generated table covers."""
    return [(k, k) for k in KS] + RECT_SHAPES


def generate(out_dir: str, workers: int | None = None) -> dict:
    os.makedirs(out_dir, exist_ok=True)
    keys = [(kw, kh, tw, th, mode) for (kw, kh) in windows() for (tw, th) in tile_options(kw, kh)
            for mode in (MODES if kw == kh else ("asap",))]
    # largest first so that the pool's tail is short
    keys.sort(key=lambda t: -(t[0] + t[2]) * (t[1] + t[3]))
    workers = workers or min(8, os.cpu_count() or 1)
    if workers > 1:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            cache = dict(zip(keys, ex.map(_schedule_or_none, keys, chunksize=4)))
    else:
        cache = {key: _schedule_or_none(key) for key in keys}
    entries = []
    placed = {}
    cache3: dict = {}
    words: list[np.ndarray] = []
    pos = 0

    def place(S: dagen.Schedule, key) -> tuple:
        """Blob words of one schedule (stored once per key): items first
        (16-byte aligned), then round boundaries, per-round chunk lengths,
        per-round recursion levels and median offsets."""
        nonlocal pos
        if key not in placed:
            pad = (-pos) % 4
            if pad:
                words.append(np.zeros(pad, np.uint32))
                pos += pad
            offs = []
            for arr in (S.items.reshape(-1), S.rounds, S.chunk_len, S.round_phase, S.outputs):
                offs.append(pos)
                words.append(arr.astype(np.uint32))
                pos += len(arr)
            c_off, r_off, l_off, p_off, o_off = offs
            placed[key] = (c_off, len(S.items), r_off, len(S.rounds) - 1, l_off, p_off, o_off, S.arena)
        return placed[key]

    for es in (2, 4):
        for (kw, kh) in windows():
            # rectangular windows keep one tile (no tuned choice), shared by
            # both element sizes: the best one that lets three work-groups of
            # 32-bit elements share a CU, the budget most square windows up
            # to k = 31 are tuned to; the lane groups per work-group follow
            # the element size
            if kw == kh:
                opts = [(tw, th, 1, 1, mi) for (tw, th, mi) in candidates(kw, es, cache, modes=MODES)]
            else:
                # small tiles run several to a work-group in lane groups;
                # their schedule is cut for the group's lanes
                tw, th, mi = candidates(kw, 4, cache, kh, LDS_BUDGETS[:1])[0]
                opts = [(tw, th, 1, lane_groups(cache[(kw, kh, tw, th, MODES[mi])], es), mi)]
            for (tw, th, T, G, mi) in opts:
                key = (kw, kh, tw, th, G, MODES[mi])
                S = cache[(kw, kh, tw, th, MODES[mi])] if G == 1 else \
                    dagen.schedule(kw, tw, th, kh=kh, lanes=dagen.LANES // G, rounds=MODES[mi])
                assert S.arena * es * T * G <= LDS_BYTES
                entries.append((kw, kh, 1, es, tw, th, 1, T, G, 0, mi) + place(S, key))
        # global-memory form (square windows): lists in a device workspace,
        # so the tile is not bounded by the LDS
        for k in KS:
            tw, th = global_tile(k, cache)
            entries.append((k, k, 1, es, tw, th, 1, 1, 1, 1, 0) +
                           place(cache[(k, k, tw, th, "phase")], (k, k, tw, th, 1, "phase")))
        # 3-D boxes; small tiles run several to a work-group in lane groups
        for k in K3:
            t = tile3(k, es, cache3)
            G = lane_groups(cache3[k][t], es)
            S = cache3[k][t] if G == 1 else dagen.schedule3(k, k, k, *t, lanes=dagen.LANES // G, rounds="asap")
            assert S.arena * es * G <= LDS_BYTES
            entries.append((k, k, k, es) + t + (1, G, 0, 1) + place(S, (k, k, k) + t + (G,)))
    blob = np.concatenate(words).astype("<u4")
    bpath = os.path.join(out_dir, "mf_da_blob.bin")
    data = blob.tobytes()
    if not os.path.exists(bpath) or open(bpath, "rb").read() != data:
        with open(bpath, "wb") as f:
            f.write(data)
    lines = ["// Generated by emit_da.py: data-aware schedules, one entry per",
             "// (k_w, k_h, k_z, element size, root tile t_w x t_h x t_z, tiles per lane,",
             "// lane groups, memory: 0 = LDS arena, 1 = device workspace, round mode:",
             "// 0 = per recursion level, 1 = over the whole schedule).",
             "#pragma once",
             "#define MF_DA_BLOB_WORDS %d" % len(blob),
             "#define MF_DA_CHUNK %d" % dagen.CHUNK,
             "#define MF_DA_GUARD %d" % dagen.GUARD,
             "#define MF_DA_SENT %d" % dagen.SENT_W,
             "#define MF_DA_RECT_MAX_SIDE %d" % RECT_MAX_SIDE,
             "#define MF_DA_TABLE_ENTRIES \\"]
    for e in entries:
        lines.append("    {" + ", ".join("%d" % v for v in e) + "}, \\")
    lines.append("")
    text = "\n".join(lines) + "\n"
    hpath = os.path.join(out_dir, "mf_da_table.h")
    if not os.path.exists(hpath) or open(hpath).read() != text:
        with open(hpath, "w") as f:
            f.write(text)
    return {"blob_bytes": len(data), "entries": len(entries), "schedules": len(placed)}
