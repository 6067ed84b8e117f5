"""Build-time generator of the data-oblivious hierarchical selection network.

The hierarchical-tiling median filter (Sugy 2025, Section 3) is turned into a
straight-line program of min/max operations over the values of one root tile's
footprint. The generator

* builds comparator networks from textbook constructions: Batcher's odd-even
  merge generalised to arbitrary list sizes, odd-even merge sort, and a
  multi-way merge as a balanced tree of two-way merges (Section 4.1 names
  these families);
* follows the tile recursion of Section 3.1 (square tiles split horizontally,
  other tiles on their longer side) with the initialisation of Section 3.3
  (sorted columns, sorted extra rows, core by multi-way merge of the sorted
  columns) and the splits of Section 3.4;
* forgets extrema after every merge into a core: with n sorted candidates and
  u window values not yet seen, only the middle min(n, u+1) can still be the
  median (forgetfulness, Section 2.2);
* records the program in SSA form with hash-consing, so pruning is dead-code
  elimination from the t_w*t_h medians: a compare-exchange whose min (or max)
  feeds nothing kept disappears, which is the pruning of Sections 3.3 and 4.1.

Values are referred to in root-footprint coordinates: x in [0, k+t_w-1),
y in [0, k+t_h-1); the pixel (px, py) of the root tile owns the window
x in [px, px+k), y in [py, py+k).

Loads come in two kinds, matching what the GPU kernel keeps in LDS:

* ``('col', x, i)``: element i (ascending) of footprint column x sorted over
  the root core rows y in [t_h-1, k) -- shared between horizontally adjacent
  tiles and sorted once per work-group;
* ``('raw', x, y)``: an unsorted footprint value.

The module also has a numpy evaluator of a program over all root tiles of an
image (a CPU model used by the tests to check the network before it is
compiled) and op counts used for the VALU roofline.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LD, MIN, MAX = 0, 1, 2


class Prog:
    """SSA program of loads and min/max, hash-consed."""

    def __init__(self):
        self.ops: list[tuple] = []   # (LD, key) | (MIN, a, b) | (MAX, a, b)
        self._memo: dict = {}
        self.outputs: list[int] = []

    def _add(self, op):
        v = self._memo.get(op)
        if v is None:
            v = len(self.ops)
            self.ops.append(op)
            self._memo[op] = v
        return v

    def load(self, key) -> int:
        return self._add((LD, key))

    def min(self, a: int, b: int) -> int:
        if a == b:
            return a
        return self._add((MIN, min(a, b), max(a, b)))

    def max(self, a: int, b: int) -> int:
        if a == b:
            return a
        return self._add((MAX, min(a, b), max(a, b)))

    def cas(self, a: int, b: int):
        return self.min(a, b), self.max(a, b)


# --------------------------------------------------------------- networks

def merge(P: Prog, A: list[int], B: list[int]) -> list[int]:
    """Batcher's odd-even merge of two ascending lists of any sizes.

    The elements at even positions of both inputs are merged into v, those at
    odd positions into w; the result is v[0], then the compare-exchange of
    w[i] with v[i+1] for each i, then whatever of v or w has no partner
    (Knuth, TAOCP vol. 3, 5.3.4).
    """
    if not A:
        return list(B)
    if not B:
        return list(A)
    if len(A) == 1 and len(B) == 1:
        lo, hi = P.cas(A[0], B[0])
        return [lo, hi]
    v = merge(P, A[0::2], B[0::2])
    w = merge(P, A[1::2], B[1::2])
    z = [v[0]]
    for i, wi in enumerate(w):
        if i + 1 < len(v):
            lo, hi = P.cas(wi, v[i + 1])
            z += [lo, hi]
        else:
            z.append(wi)
    z += v[len(w) + 1:]
    return z


def sort(P: Prog, L: list[int]) -> list[int]:
    """Odd-even merge sort of any length (split in halves, merge)."""
    if len(L) <= 1:
        return list(L)
    h = len(L) // 2
    return merge(P, sort(P, L[:h]), sort(P, L[h:]))


def multiway(P: Prog, lists: list[list[int]]) -> list[int]:
    """Multi-way merge as a balanced binary tree of two-way merges."""
    lists = [l for l in lists if l]
    if not lists:
        return []
    while len(lists) > 1:
        nxt = []
        for i in range(0, len(lists) - 1, 2):
            nxt.append(merge(P, lists[i], lists[i + 1]))
        if len(lists) % 2:
            nxt.append(lists[-1])
        lists = nxt
    return lists[0]


def trim(L: list[int], unseen: int) -> list[int]:
    """Keep the middle min(len, unseen+1) candidates (forgetfulness)."""
    keep = min(len(L), unseen + 1)
    d = (len(L) - keep) // 2
    assert (len(L) - keep) % 2 == 0, "candidates + unseen must be odd"
    return L[d:d + keep]


# -------------------------------------------------------------- geometry

def root_tile_heuristic(k: int) -> int:
    """t(k) = 2^(floor(log2 k) - 1) of Section 4.2 (k >= 3), 1 for k = 1."""
    if k < 3:
        return 1
    return 2 ** (int(math.floor(math.log2(k))) - 1)


def split_sequence(tw: int, th: int) -> list[tuple[int, int]]:
    """Tile sizes from the root to the 1x1 leaf (recursion of Section 3.1)."""
    seq = [(tw, th)]
    while (tw, th) != (1, 1):
        if tw >= th:
            tw //= 2
        else:
            th //= 2
        seq.append((tw, th))
    return seq


@dataclass
class TileParts:
    """Partition of a t_w x t_h tile's footprint for a k x k kernel (Section 3.2)."""
    footprint: tuple[int, int]
    core: tuple[int, int]
    extra_cols_per_side: int
    extra_rows_per_side: int
    corner_block: tuple[int, int]


def tile_parts(k: int, tw: int, th: int) -> TileParts:
    return TileParts(footprint=(k + tw - 1, k + th - 1), core=(k - tw + 1, k - th + 1),
                     extra_cols_per_side=tw - 1, extra_rows_per_side=th - 1,
                     corner_block=(tw - 1, th - 1))


def level_table(k: int, tw: int, th: int):
    """(t_w, t_h, core size c, unseen u, kept candidates) for every level.

    A child's core adds c_child - c_parent new values to the parent's kept
    candidates, and forgetting keeps min(held, u+1) of them.
    """
    N = k * k
    rows = []
    kept = None
    c_prev = None
    for (a, b) in split_sequence(tw, th):
        c = (k - a + 1) * (k - b + 1)
        u = N - c
        held = c if kept is None else kept + (c - c_prev)
        kept = min(held, u + 1)
        rows.append((a, b, c, u, kept))
        c_prev = c
    return rows


# ------------------------------------------------------ the tile program

@dataclass
class _State:
    ox: int
    oy: int
    tw: int
    th: int
    core: list[int]
    xcols: dict = field(default_factory=dict)   # x -> sorted list over core rows
    xrows: dict = field(default_factory=dict)   # y -> sorted list over core cols


def build_tile_program(k: int, tw: int, th: int, inline_cols: bool = False,
                       kh: int | None = None) -> Prog:
    """Straight-line selection network for one tw x th root tile.

    The window is k columns by kh rows (kh defaults to k, the square filter):
    footprint (k+tw-1) x (kh+th-1), sorted columns over the kh-th+1 core rows.
    outputs[py*tw + px] is the median of the window of pixel (px, py).
    With inline_cols the tile sorts its own footprint columns from raw loads
    (pruned to the ranks it uses) instead of loading pre-sorted shared
    columns: no shared column buffer, more work per tile (small k).
    """
    kw = k
    kh = k if kh is None else kh
    assert kw % 2 == 1 and kw >= 1 and kh % 2 == 1 and kh >= 1
    assert tw >= 1 and th >= 1 and (tw & (tw - 1)) == 0 and (th & (th - 1)) == 0
    assert tw <= kw and th <= kh
    P = Prog()
    N = kw * kh
    Lc = kh - th + 1

    def col(x):
        if inline_cols:
            return sort(P, [P.load(("raw", x, y)) for y in range(th - 1, kh)])
        return [P.load(("col", x, i)) for i in range(Lc)]

    def raw(x, y):
        return P.load(("raw", x, y))

    # Initialisation (Section 3.3): sorted columns (loads of pre-sorted data),
    # sorted extra rows, core = multi-way merge of the sorted core columns.
    core_x = range(tw - 1, kw)
    core = multiway(P, [col(x) for x in core_x])
    core = trim(core, N - len(core_x) * Lc)
    st = _State(0, 0, tw, th, core)
    for x in list(range(0, tw - 1)) + list(range(kw, kw + tw - 1)):
        st.xcols[x] = col(x)
    for y in list(range(0, th - 1)) + list(range(kh, kh + th - 1)):
        st.xrows[y] = sort(P, [raw(x, y) for x in core_x])

    out = {}

    def recurse(s: _State):
        if s.tw == 1 and s.th == 1:
            assert len(s.core) == 1
            out[(s.ox, s.oy)] = s.core[0]
            return
        if s.tw >= s.th:
            h = s.tw // 2
            for child_ox, added in ((s.ox, range(s.ox + h - 1, s.ox + s.tw - 1)),
                                    (s.ox + h, range(s.ox + kw, s.ox + kw + h))):
                ncx = (kw - h + 1)
                ncy = (kh - s.th + 1)
                c = merge(P, s.core, multiway(P, [s.xcols[x] for x in added]))
                c = trim(c, N - ncx * ncy)
                ch = _State(child_ox, s.oy, h, s.th, c)
                for x in list(range(child_ox, child_ox + h - 1)) + \
                        list(range(child_ox + kw, child_ox + kw + h - 1)):
                    ch.xcols[x] = s.xcols[x]
                for y, row in s.xrows.items():
                    ch.xrows[y] = merge(P, row, sort(P, [raw(x, y) for x in added]))
                recurse(ch)
        else:
            h = s.th // 2
            for child_oy, added in ((s.oy, range(s.oy + h - 1, s.oy + s.th - 1)),
                                    (s.oy + h, range(s.oy + kh, s.oy + kh + h))):
                ncx = (kw - s.tw + 1)
                ncy = (kh - h + 1)
                c = merge(P, s.core, multiway(P, [s.xrows[y] for y in added]))
                c = trim(c, N - ncx * ncy)
                ch = _State(s.ox, child_oy, s.tw, h, c)
                for y in list(range(child_oy, child_oy + h - 1)) + \
                        list(range(child_oy + kh, child_oy + kh + h - 1)):
                    ch.xrows[y] = s.xrows[y]
                for x, cl in s.xcols.items():
                    ch.xcols[x] = merge(P, cl, sort(P, [raw(x, y) for y in added]))
                recurse(ch)

    recurse(st)
    P.outputs = [out[(px, py)] for py in range(th) for px in range(tw)]
    return P


def build_sort_program(n: int) -> Prog:
    """Odd-even merge sort of n loads ('in', i); outputs ascending."""
    P = Prog()
    P.outputs = sort(P, [P.load(("in", i)) for i in range(n)])
    return P


# ------------------------------------------------------------ analysis

def live_ops(P: Prog) -> list[int]:
    """Indices of the ops the outputs depend on, in program order."""
    need = bytearray(len(P.ops))
    for o in P.outputs:
        need[o] = 1
    for v in range(len(P.ops) - 1, -1, -1):
        if need[v]:
            op = P.ops[v]
            if op[0] != LD:
                need[op[1]] = 1
                need[op[2]] = 1
    return [v for v in range(len(P.ops)) if need[v]]


def op_counts(P: Prog) -> dict:
    live = live_ops(P)
    n_ld = sum(1 for v in live if P.ops[v][0] == LD)
    n_mm = len(live) - n_ld
    return {"loads": n_ld, "minmax": n_mm, "ops_total": len(P.ops)}


def max_live(P: Prog) -> int:
    """Peak number of simultaneously live values when the live ops run in
    program order (a register-pressure estimate for the emitted code)."""
    live = live_ops(P)
    last_use = {}
    for v in live:
        op = P.ops[v]
        if op[0] != LD:
            last_use[op[1]] = v
            last_use[op[2]] = v
    for o in P.outputs:
        last_use[o] = len(P.ops)
    cur = peak = 0
    ends: dict[int, int] = {}
    for v in live:
        op = P.ops[v]
        if op[0] != LD:
            for a in {op[1], op[2]}:
                if last_use.get(a) == v:
                    cur -= 1
        cur += 1
        peak = max(peak, cur)
    return peak


# ------------------------------------------------------------ CPU model

def evaluate_on_image(P: Prog, img: np.ndarray, k: int, tw: int, th: int,
                      kh: int | None = None) -> np.ndarray:
    """Run a tile program over every root tile of `img` (replicate border),
    window k columns by kh rows (kh defaults to k).

    A debugging model of the GPU kernel: sorted columns come from numpy sorts
    of the footprint columns, every op is applied to all tiles at once.
    """
    kw = k
    kh = k if kh is None else kh
    H, W = img.shape
    nty, ntx = -(-H // th), -(-W // tw)
    ys = np.clip(np.arange(nty * th + kh - 1) - (kh - 1) // 2, 0, H - 1)
    xs = np.clip(np.arange(ntx * tw + kw - 1) - (kw - 1) // 2, 0, W - 1)
    pad = img[ys][:, xs]
    fh, fw = kh + th - 1, kw + tw - 1
    # footprint of every tile: (nty, ntx, fh, fw)
    win = np.lib.stride_tricks.sliding_window_view(pad, (fh, fw))[::th, ::tw]
    core_sorted = np.sort(win[:, :, th - 1:kh, :], axis=2)  # (nty, ntx, Lc, fw)
    vals = [None] * len(P.ops)
    for v in live_ops(P):
        op = P.ops[v]
        if op[0] == LD:
            kind, a, b = op[1]
            vals[v] = core_sorted[:, :, b, a] if kind == "col" else win[:, :, b, a]
        elif op[0] == MIN:
            vals[v] = np.minimum(vals[op[1]], vals[op[2]])
        else:
            vals[v] = np.maximum(vals[op[1]], vals[op[2]])
    out = np.empty((nty * th, ntx * tw), dtype=img.dtype)
    for i, o in enumerate(P.outputs):
        py, px = divmod(i, tw)
        out[py::th, px::tw] = vals[o]
    return out[:H, :W]


def demand_order(P: Prog) -> list[int]:
    """Live ops in the order a depth-first walk from each output first needs
    them (post-order). Values are produced close to their first use, which
    keeps the number of simultaneously live registers low."""
    order = []
    seen = bytearray(len(P.ops))
    for o in P.outputs:
        stack = [(o, False)]
        while stack:
            v, expanded = stack.pop()
            if seen[v]:
                continue
            op = P.ops[v]
            if expanded or op[0] == LD:
                seen[v] = 1
                order.append(v)
                continue
            stack.append((v, True))
            # operand pushed last is visited first
            stack.append((op[2], False))
            stack.append((op[1], False))
    return order


def peak_live(P: Prog, order: list[int], reload_loads: bool = False) -> int:
    """Peak simultaneously live values when `order` runs. With reload_loads a
    load is assumed to be re-issued at each use (never kept live)."""
    pos = {v: i for i, v in enumerate(order)}
    last = {}
    for v in order:
        op = P.ops[v]
        if op[0] != LD:
            last[op[1]] = pos[v]
            last[op[2]] = pos[v]
    for o in P.outputs:
        last[o] = len(order)
    cur = peak = 0
    dying = {}
    for i, v in enumerate(order):
        if reload_loads and P.ops[v][0] == LD:
            continue
        cur += 1
        peak = max(peak, cur)
        dying.setdefault(last.get(v, i), []).append(v)
        for d in dying.pop(i, []):
            cur -= 1
    return peak
