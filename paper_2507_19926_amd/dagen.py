"""Build-time schedule generator for the data-aware hierarchical median filter.

The data-aware variant (Sugy 2025, Section 5) keeps the tile recursion of
Section 3 but realises every sort and merge with data-dependent work in LDS:

* sorting a column, an extra row or a group of corners (footprint values
  that lie on one line) is one per-lane sorting network over at most
  SORT_MAX values held in registers (Section 5.1: the many small sorts run as
  sorting networks per thread); longer lines are cut into such pieces, which
  are then merged;
* a multi-way merge is a binary reduction of two-way merges, halving the
  number of lists each round (Section 5.1);
* every two-way merge is executed with merge path: its output is cut into
  chunks, each chunk finds its start in both inputs by a co-rank binary
  search and then merges sequentially, four outputs per step (Section 5.1).

Forgetting (Section 2.2) and pruning become output windows: after a merge
into a core only the middle min(n, u+1) ranks are kept, and a backward pass
from the medians gives every list the window of ranks any consumer can read,
so no element outside it is ever produced.

The generator records, for one root tile of t_w x t_h pixels, a DAG of list
nodes, assigns each node the recursion level (phase) that creates it,
schedules the work of each phase in dependency rounds, allocates LDS (first
fit, freed after the last reader) and emits compact items of 4 words.

Every stored list is followed by SENT_W sentinel slots holding the largest
element value, so a merge never tests whether an input is exhausted: the
elements after an input window are sentinels or list elements ranked after
every output the merge must produce, and they are never chosen while needed
outputs remain.

Items (4 uint32 words):

* merge chunk: w0 = a_off | na << 18, w1 = b_off | nb << 18,
  w2 = out_off | nvalid << 18, w3 = r0 | steps << 18 | last << 22.
  The lane finds the co-rank of rank r0 (the chunk's first output, counted in
  the merge of the two input windows; A first on ties) over a range of fewer
  than 2^steps positions, then emits the round's chunk length C of outputs,
  four per step (C is uniform over a round and a multiple of four; chunks
  start at multiples of C, and a ragged end gets one more chunk ending at the
  next multiple of four, overlapping the one before and rewriting the same
  values; out_off is then a multiple of four). When `last` is set the lane
  then writes the SENT_W sentinels from out_off + nvalid.
* sort: w0 = base | n << 18, w1 = stride | lo << 18, w2 = out_off | (hi-lo) << 18,
  w3 = SORT_FLAG | N | L << 6 | step << 9: the n*L footprint values at
  base + j*step + i*stride (L parallel lines of n values) are sorted by the
  network for N (a power of two >= n*L, padded with the largest value);
  ranks [lo, hi) are written from out_off, followed by the SENT_W sentinels.

Per round: the item range (work-group barrier between rounds) and the chunk
length C. Offsets are in elements of the LDS arena: a guard of GUARD elements
(its last SENT_W slots hold the sentinel value and stand in for empty input
windows), then the raw footprint (row-major, fw = k_w+t_w-1 wide), then the
lists; the arena ends with a pad that absorbs the reads and writes a chunk
makes past its needed outputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CHUNK = 4           # shortest merge-path chunk; every chunk length is a multiple of it
LANES = 512         # threads of a data-aware work-group: a round's outputs are
                    # cut into about this many chunks
OFF_BITS = 18       # arena offsets and sizes share a 32-bit word
MAX_OFF = 1 << OFF_BITS
MAX_LEN = 1 << (32 - OFF_BITS)
SORT_MAX = 32       # largest per-lane sorting network
ROUNDS = "asap"     # round assignment: "asap" over the whole DAG, or "phase"
                    # (ASAP within each recursion level)
SENT_W = 4          # sentinel slots after every stored list (a merge step reads 4 ahead)
GUARD = 8           # arena elements before the footprint; the last SENT_W hold sentinels
SENTINEL_SLOT = GUARD - SENT_W
ALIGN = 4           # stored lists start at multiples of ALIGN elements
READ_PAST = 2 * SENT_W  # elements a merge may read after an input window's
                    # end: its head stays within the SENT_W after it, and a
                    # step reads four elements from the head (16-bit ones as
                    # the aligned dwords that hold them)
SORT_FLAG = 1 << 31
LSTEP_SHIFT = 9     # sort items: w3 = SORT_FLAG | N | lines << 6 | line step << 9
LSTEP_BITS = 22
STEP_SHIFT = 18
LAST_BIT = 1 << 22


@dataclass
class Node:
    nid: int
    size: int                       # full logical length
    a: tuple | None = None          # (node, lo, hi) input views
    b: tuple | None = None
    raw: tuple | None = None        # (x, y) for a single footprint value
    line: tuple | None = None       # sort node: (base, stride, n, lines, line step) footprint offsets
    phase: int = 0
    need_lo: int = 0
    need_hi: int = 0
    consumers: list = field(default_factory=list)
    off: int = -1
    rnd: int = -1
    role: str = ""
    store: int = 0                  # allocated elements (window + pad + sentinel)


class Dag:
    def __init__(self, fw: int, fh: int = 0):
        self.nodes: list[Node] = []
        self.fw = fw
        self.fh = fh            # footprint rows (needed for 3-D points)
        self.phase = 0
        self.role = ""
        self._raw = {}

    def raw(self, x: int, y: int) -> tuple:
        key = (x, y)
        if key not in self._raw:
            n = Node(len(self.nodes), 1, raw=key, phase=-1)
            self.nodes.append(n)
            self._raw[key] = n
        n = self._raw[key]
        return (n, 0, 1)

    def merge(self, A: tuple, B: tuple) -> tuple:
        if A[2] - A[1] == 0:
            return B
        if B[2] - B[1] == 0:
            return A
        n = Node(len(self.nodes), (A[2] - A[1]) + (B[2] - B[1]), a=A, b=B, phase=self.phase,
                 role=self.role)
        self.nodes.append(n)
        return (n, 0, n.size)

    def reduce(self, lists: list[tuple]) -> tuple:
        """Binary reduction of two-way merges (balanced, in list order)."""
        lists = [l for l in lists if l[2] - l[1] > 0]
        if not lists:
            return (None, 0, 0)
        while len(lists) > 1:
            nxt = [self.merge(lists[i], lists[i + 1]) for i in range(0, len(lists) - 1, 2)]
            if len(lists) % 2:
                nxt.append(lists[-1])
            lists = nxt
        return lists[0]

    def offset(self, p: tuple) -> int:
        """Arena offset of footprint point (x, y) or (x, y, z)."""
        x, y = p[0], p[1]
        z = p[2] if len(p) > 2 else 0
        return GUARD + (z * self.fh + y) * self.fw + x

    def _line(self, pts: list[tuple]) -> Node:
        """Sort node over footprint points that lie on one line (equal steps)."""
        offs = [self.offset(p) for p in pts]
        stride = offs[1] - offs[0] if len(offs) > 1 else 1
        assert stride > 0 and all(offs[i] == offs[0] + i * stride for i in range(len(offs)))
        n = Node(len(self.nodes), len(pts), line=(offs[0], stride, len(pts), 1, 0), phase=self.phase,
                 role=self.role)
        self.nodes.append(n)
        return n

    def sort_lines(self, lines: list[list[tuple]]) -> tuple:
        """Sorted list of the footprint values on several parallel lines of
        equal length and step, the lines themselves equally spaced: one
        sorting network when they hold at most SORT_MAX values together,
        else each line sorted alone; the sorted pieces are then merged."""
        if not lines:
            return (None, 0, 0)
        n = len(lines[0])
        per = max(1, min(7, SORT_MAX // max(n, 1)))     # at most 7 lines per item
        pieces = []
        for g in range(0, len(lines), per):
            grp = lines[g:g + per]
            if len(grp) == 1 or n == 0:
                pieces.append(self.sort(grp[0]))
                continue
            first = [self.offset(p) for p in grp[0]]
            stride = first[1] - first[0] if n > 1 else 1
            lstep = self.offset(grp[1][0]) - first[0]
            for j, ln in enumerate(grp):
                offs = [self.offset(p) for p in ln]
                assert len(ln) == n and all(offs[i] == first[0] + j * lstep + i * stride for i in range(n))
            node = Node(len(self.nodes), n * len(grp), line=(first[0], stride, n, len(grp), lstep),
                        phase=self.phase, role=self.role)
            self.nodes.append(node)
            pieces.append((node, 0, node.size))
        return self.reduce(pieces)

    def sort(self, pts: list[tuple]) -> tuple:
        """Sorted list of the footprint values at pts ((x, y) or (x, y, z) on
        one line):
        sorting networks over pieces of at most SORT_MAX values, merged."""
        if not pts:
            return (None, 0, 0)
        npc = -(-len(pts) // SORT_MAX)
        step = -(-len(pts) // npc)
        pieces = [self._line(pts[i:i + step]) for i in range(0, len(pts), step)]
        return self.reduce([(p, 0, p.size) for p in pieces])


def trim(ref: tuple, unseen: int) -> tuple:
    n, lo, hi = ref
    size = hi - lo
    keep = min(size, unseen + 1)
    assert (size - keep) % 2 == 0
    d = (size - keep) // 2
    return (n, lo + d, lo + d + keep)


def build_dag(k: int, tw: int, th: int, kh: int | None = None):
    """DAG of the hierarchical recursion for one tw x th root tile.

    The window is k columns by kh rows (kh defaults to k: the square filter);
    the footprint is (k+tw-1) x (kh+th-1) and the core of a tile is the
    intersection of its pixels' windows, so every split, added column or row
    and forgetful trim follows from those two sides.

    Returns (dag, outputs) with outputs[py*tw+px] a (node, lo, lo+1) view of
    that pixel's median."""
    kw = k
    kh = k if kh is None else kh
    assert kw % 2 == 1 and kh % 2 == 1 and tw <= kw and th <= kh
    D = Dag(kw + tw - 1)
    N = kw * kh
    core_y = range(th - 1, kh)
    core_x = range(tw - 1, kw)

    def col(x, ys):
        D.role = "sort_col"
        return D.sort([(x, y) for y in ys])

    def row(y, xs):
        D.role = "sort_row"
        return D.sort([(x, y) for x in xs])

    D.phase = 0
    # the core: sorted core columns (several to one network when short),
    # merged
    D.role = "sort_col"
    core = D.sort_lines([[(x, y) for y in core_y] for x in core_x])
    core = trim(core, N - len(core_x) * len(core_y))
    xcols = {x: col(x, core_y) for x in list(range(0, tw - 1)) + list(range(kw, kw + tw - 1))}
    xrows = {y: row(y, core_x) for y in list(range(0, th - 1)) + list(range(kh, kh + th - 1))}
    outputs = {}

    def recurse(ox, oy, w, h, core, xcols, xrows, level):
        if w == 1 and h == 1:
            assert core[2] - core[1] == 1
            outputs[(ox, oy)] = core
            return
        D.phase = level + 1
        children = []
        if w >= h:
            hh = w // 2
            for cox, added in ((ox, range(ox + hh - 1, ox + w - 1)), (ox + hh, range(ox + kw, ox + kw + hh))):
                D.phase = level + 1
                D.role = "core_extra"
                e = D.reduce([xcols[x] for x in added])
                D.role = "core_merge"
                c = D.merge(core, e)
                c = trim(c, N - (kw - hh + 1) * (kh - h + 1))
                ncols = {x: xcols[x] for x in list(range(cox, cox + hh - 1)) + list(range(cox + kw, cox + kw + hh - 1))}
                nrows = {}
                for y, r in xrows.items():
                    D.role = "sort_corner"
                    cs = D.sort([(x, y) for x in added])
                    D.role = "extend"
                    nrows[y] = D.merge(r, cs)
                children.append((cox, oy, hh, h, c, ncols, nrows))
        else:
            hh = h // 2
            for coy, added in ((oy, range(oy + hh - 1, oy + h - 1)), (oy + hh, range(oy + kh, oy + kh + hh))):
                D.phase = level + 1
                D.role = "core_extra"
                e = D.reduce([xrows[y] for y in added])
                D.role = "core_merge"
                c = D.merge(core, e)
                c = trim(c, N - (kw - w + 1) * (kh - hh + 1))
                nrows = {y: xrows[y] for y in list(range(coy, coy + hh - 1)) + list(range(coy + kh, coy + kh + hh - 1))}
                ncols = {}
                for x, cl in xcols.items():
                    D.role = "sort_corner"
                    cs = D.sort([(x, y) for y in added])
                    D.role = "extend"
                    ncols[x] = D.merge(cl, cs)
                children.append((ox, coy, w, hh, c, ncols, nrows))
        for ch in children:
            recurse(*ch, level + 1)

    recurse(0, 0, tw, th, core, xcols, xrows, 0)
    outs = [outputs[(px, py)] for py in range(th) for px in range(tw)]
    return D, outs


def build_dag3(kx: int, ky: int, kz: int, tx: int, ty: int, tz: int):
    """DAG of the hierarchical recursion for a tx x ty x tz root tile of a 3-D
    box median (kx x ky x kz, odd sides): the recursion of build_dag with a
    third axis.

    A tile's footprint is (kx+tx-1) x (ky+ty-1) x (kz+tz-1); its core (the
    intersection of its voxels' boxes) spans [t_a-1, k_a) on every axis a.
    Besides the trimmed sorted core a tile keeps, for every axis a and every
    footprint coordinate c outside the core on a, a face list (the values at
    a = c over the core ranges of the other two axes), for every pair of
    axes and pair of outside coordinates an edge list (over the core range of
    the third axis), and reads corners (outside on all three) as raw values.
    A split halves the longest side (x before y before z on ties); each
    child's core grows by the face lists of its added coordinates on the
    split axis and is trimmed; its other faces grow by the edge lists at the
    added coordinates; its edges that do not involve the split axis grow by
    the sorted corners at the added coordinates.

    Returns (dag, outputs) with outputs[(pz*ty + py)*tx + px] a (node, lo,
    lo+1) view of that voxel's median."""
    k = (kx, ky, kz)
    t0 = (tx, ty, tz)
    for a in range(3):
        assert k[a] % 2 == 1 and 1 <= t0[a] <= k[a]
    D = Dag(kx + tx - 1, ky + ty - 1)
    N = kx * ky * kz
    core_r = [range(t0[a] - 1, k[a]) for a in range(3)]
    extra_c = [list(range(0, t0[a] - 1)) + list(range(k[a], k[a] + t0[a] - 1)) for a in range(3)]

    def line(axis, fixed: dict, rng) -> tuple:
        """Sorted values along `axis` over rng, the other coordinates fixed."""
        pts = []
        for v in rng:
            p = dict(fixed)
            p[axis] = v
            pts.append((p[0], p[1], p[2]))
        return D.sort(pts)

    D.phase = 0
    D.role = "sort_line"
    # z-lines over the core z range at every (x, y) the core, x faces, y faces
    # and xy edges need
    zl = {}
    for x in list(core_r[0]) + extra_c[0]:
        for y in list(core_r[1]) + extra_c[1]:
            if x in extra_c[0] and y in extra_c[1]:
                continue
            zl[(x, y)] = line(2, {0: x, 1: y}, core_r[2])
    D.role = "core_init"
    core = D.reduce([zl[(x, y)] for x in core_r[0] for y in core_r[1]])
    core = trim(core, N - len(core_r[0]) * len(core_r[1]) * len(core_r[2]))
    D.role = "face_init"
    face = [dict(), dict(), dict()]
    for c in extra_c[0]:
        face[0][c] = D.reduce([zl[(c, y)] for y in core_r[1]])
    for c in extra_c[1]:
        face[1][c] = D.reduce([zl[(x, c)] for x in core_r[0]])
    for c in extra_c[2]:
        D.role = "sort_line"
        xs = [line(0, {1: y, 2: c}, core_r[0]) for y in core_r[1]]
        D.role = "face_init"
        face[2][c] = D.reduce(xs)
    D.role = "sort_line"
    edge = {(0, 1): {}, (0, 2): {}, (1, 2): {}}
    for cx in extra_c[0]:
        for cy in extra_c[1]:
            edge[(0, 1)][(cx, cy)] = line(2, {0: cx, 1: cy}, core_r[2])
        for cz in extra_c[2]:
            edge[(0, 2)][(cx, cz)] = line(1, {0: cx, 2: cz}, core_r[1])
    for cy in extra_c[1]:
        for cz in extra_c[2]:
            edge[(1, 2)][(cy, cz)] = line(0, {1: cy, 2: cz}, core_r[0])
    outputs = {}

    def recurse(o, t, core, face, edge, level):
        if t == (1, 1, 1):
            assert core[2] - core[1] == 1
            outputs[o] = core
            return
        a = max(range(3), key=lambda i: (t[i], -i))     # longest side, x first on ties
        b, c = [i for i in range(3) if i != a]
        half = t[a] // 2
        children = []
        for side in (0, 1):
            D.phase = level + 1
            if side == 0:
                co = o[a]
                added = list(range(o[a] + half - 1, o[a] + t[a] - 1))
            else:
                co = o[a] + half
                added = list(range(o[a] + k[a], o[a] + k[a] + half))
            nt = list(t)
            nt[a] = half
            no = list(o)
            no[a] = co
            D.role = "core_extra"
            e = D.reduce([face[a][x] for x in added])
            D.role = "core_merge"
            cm = D.merge(core, e)
            cm = trim(cm, N - (k[0] - nt[0] + 1) * (k[1] - nt[1] + 1) * (k[2] - nt[2] + 1))
            nface = [dict(), dict(), dict()]
            keep_a = list(range(co, co + half - 1)) + list(range(co + k[a], co + k[a] + half - 1))
            nface[a] = {x: face[a][x] for x in keep_a}
            for f in (b, c):
                g = c if f == b else b
                pair = (min(a, f), max(a, f))
                for cf, lst in face[f].items():
                    D.role = "face_extra"
                    ex = D.reduce([edge[pair][(x, cf) if a < f else (cf, x)] for x in added])
                    D.role = "face_merge"
                    nface[f][cf] = D.merge(lst, ex)
            nedge = {(0, 1): {}, (0, 2): {}, (1, 2): {}}
            for pair in nedge:
                if a in pair:
                    ia = pair.index(a)
                    nedge[pair] = {key: v for key, v in edge[pair].items() if key[ia] in keep_a}
                else:
                    for (c1, c2), lst in edge[pair].items():
                        D.role = "sort_corner"
                        pts = []
                        for x in added:
                            q = [0, 0, 0]
                            q[pair[0]], q[pair[1]], q[a] = c1, c2, x
                            pts.append(tuple(q))
                        cs = D.sort(pts)
                        D.role = "extend"
                        nedge[pair][(c1, c2)] = D.merge(lst, cs)
            children.append((tuple(no), tuple(nt), cm, nface, nedge))
        for ch in children:
            recurse(*ch, level + 1)

    recurse((0, 0, 0), t0, core, face, edge, 0)
    outs = [outputs[(px, py, pz)] for pz in range(tz) for py in range(ty) for px in range(tx)]
    return D, outs


def propagate_windows(D: Dag, outs: list[tuple]) -> None:
    """Backward pass: the ranks of every node that some consumer can read."""
    for n in D.nodes:
        n.need_lo, n.need_hi = n.size, 0
    for (n, lo, hi) in outs:
        n.need_lo, n.need_hi = min(n.need_lo, lo), max(n.need_hi, hi)
    for n in reversed(D.nodes):
        if n.a is None or n.need_hi <= n.need_lo:
            continue
        lo, hi = n.need_lo, n.need_hi
        for (src, other) in ((n.a, n.b), (n.b, n.a)):
            m, s_lo, s_hi = src
            ls, lo_other = s_hi - s_lo, other[2] - other[1]
            a0 = max(0, lo - lo_other)
            a1 = min(ls, hi)
            if a1 > a0:
                m.need_lo = min(m.need_lo, s_lo + a0)
                m.need_hi = max(m.need_hi, s_lo + a1)
                m.consumers.append(n)


@dataclass
class Schedule:
    k: int                      # window columns
    tw: int
    th: int
    fw: int
    fh: int
    items: np.ndarray           # (n_items, 4) uint32
    rounds: np.ndarray          # (n_rounds + 1,) int32 item offsets
    chunk_len: np.ndarray       # (n_rounds,) int32 merge chunk length C per round
    round_phase: np.ndarray     # (n_rounds,) int32 recursion level of each round (0 = initialisation)
    outputs: np.ndarray         # (tw*th,) int32 arena offsets
    arena: int                  # elements of LDS the schedule needs (pad included)
    merge_outputs: int          # elements produced by all merges
    stats: dict
    kh: int = 0                 # window rows (0: k, the square filter)
    fd: int = 1                 # footprint depth (3-D boxes; 1 for planes)
    kz: int = 1                 # box depth (3-D)
    tz: int = 1                 # root tile depth (3-D)

    @property
    def kw(self) -> int:
        return self.k

    @property
    def rows(self) -> int:
        return self.kh or self.k

    @property
    def chunks(self) -> np.ndarray:
        return self.items


def _window_inputs(n: Node):
    """Input windows (storage offset, count) and the first output rank
    relative to the merge of those windows, for node n's needed window. An
    empty window points at the arena's sentinel slot."""
    lo, hi = n.need_lo, n.need_hi
    res = []
    starts = []
    for (src, other) in ((n.a, n.b), (n.b, n.a)):
        m, s_lo, s_hi = src
        ls, lo_other = s_hi - s_lo, other[2] - other[1]
        a0 = max(0, lo - lo_other)
        a1 = min(ls, hi)
        if a1 < a0:
            a1 = a0
        if a1 == a0:
            res.append((SENTINEL_SLOT, 0))
        else:
            # storage of m covers [m.need_lo, m.need_hi) and its sentinel
            res.append((m.off + (s_lo + a0 - m.need_lo), a1 - a0))
        starts.append(a0)
    r0 = lo - starts[0] - starts[1]
    return res[0], res[1], r0


# comparators of Batcher's odd-even merge sort of N = 2^p values
_OEMS_CES = {1: 0, 2: 1, 4: 5, 8: 19, 16: 63, 32: 191}


def _ceil_to(n: int, m: int) -> int:
    return -(-n // m) * m


def _pow2_at_least(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


def schedule(k: int, tw: int, th: int, chunk: int = CHUNK, lanes: int = LANES,
             kh: int | None = None, rounds: str | None = None) -> Schedule:
    """Rounds of sorts and windowed merges for root tile tw x th. A round's
    merges are cut into chunks of one length C = a multiple of `chunk`, at
    least ceil(outputs / lanes), so that one round keeps about `lanes`
    threads busy with chains as short as the round allows (a lane runs a
    co-rank search, then C sequential merge steps). `rounds` is "phase"
    (ASAP within each recursion level) or "asap" (over the whole schedule;
    fewer rounds and barriers, more LDS), default ROUNDS."""
    kh = k if kh is None else kh
    D, outs = build_dag(k, tw, th, kh)
    S = _schedule_dag(D, outs, k + tw - 1, (kh + th - 1), 1, tw * th, chunk, lanes, rounds)
    S.k, S.tw, S.th, S.kh = k, tw, th, kh
    return S


def schedule3(kx: int, ky: int, kz: int, tx: int, ty: int, tz: int, chunk: int = CHUNK,
              lanes: int = LANES, rounds: str | None = None) -> Schedule:
    """As schedule, for the 3-D box kx x ky x kz and root tile tx x ty x tz."""
    D, outs = build_dag3(kx, ky, kz, tx, ty, tz)
    S = _schedule_dag(D, outs, kx + tx - 1, ky + ty - 1, kz + tz - 1, tx * ty * tz, chunk, lanes, rounds)
    S.k, S.tw, S.th, S.kh, S.kz, S.tz = kx, tx, ty, ky, kz, tz
    return S


def _schedule_dag(D: Dag, outs: list, fw: int, fh: int, fd: int, npx: int, chunk: int, lanes: int,
                  rounds: str | None = None) -> Schedule:
    """Rounds, LDS allocation and items of a DAG whose footprint is
    fw x fh x fd (fd = 1 for planes) and whose tile has npx outputs."""
    propagate_windows(D, outs)
    work = [n for n in D.nodes if (n.a is not None or n.line is not None) and n.need_hi > n.need_lo]
    mode = ROUNDS if rounds is None else rounds
    assert mode in ("asap", "phase")
    if mode == "asap":
        # rounds: ASAP over the whole DAG (a node runs in the round after its
        # last input), so the reductions that build the next level's added
        # lists overlap the current level's core merge
        depth = {}
        for n in work:
            d = 0
            if n.a is not None:
                for src in (n.a, n.b):
                    m = src[0]
                    if m.nid in depth:
                        d = max(d, depth[m.nid] + 1)
            depth[n.nid] = d
        order = [[] for _ in range(max(depth.values()) + 1)]
        for n in work:
            order[depth[n.nid]].append(n)
    else:
        # rounds: per phase, ASAP by dependency depth within the phase
        depth = {}
        for n in work:
            d = 0
            if n.a is not None:
                for src in (n.a, n.b):
                    m = src[0]
                    if m.nid in depth and m.phase == n.phase:
                        d = max(d, depth[m.nid] + 1)
            depth[n.nid] = d
        phases = sorted(set(n.phase for n in work))
        order = []
        for p in phases:
            pm = [n for n in work if n.phase == p]
            dmax = max(depth[n.nid] for n in pm)
            for d in range(dmax + 1):
                order.append([n for n in pm if depth[n.nid] == d])
    for r, group in enumerate(order):
        for n in group:
            n.rnd = r
    # last round in which each node is read (outputs: forever)
    last_read = {}
    for n in work:
        if n.a is None:
            continue
        for src in (n.a, n.b):
            m = src[0]
            last_read[m.nid] = max(last_read.get(m.nid, -1), n.rnd)
    for (n, _, _) in outs:
        last_read[n.nid] = len(order) + 1
    # allocation: guard + raw footprint fixed at [0, GUARD + fw*fh); first fit
    # for the rest, every block a multiple of ALIGN elements at a multiple of
    # ALIGN, so a chunk's steps of four outputs write aligned runs
    base = _ceil_to(GUARD + fw * fh * fd, ALIGN)
    free = [(base, 1 << 40)]         # (start, end) holes, sorted
    peak = base

    def alloc(size):
        nonlocal peak
        size = _ceil_to(size, ALIGN)
        for i, (s, e) in enumerate(free):
            if e - s >= size:
                free[i] = (s + size, e)
                if free[i][0] == free[i][1]:
                    free.pop(i)
                peak = max(peak, s + size)
                return s
        raise RuntimeError("arena exhausted")

    def release(s, size):
        size = _ceil_to(size, ALIGN)
        free.append((s, s + size))
        free.sort()
        merged = []
        for a, b in free:
            if merged and merged[-1][1] == a:
                merged[-1] = (merged[-1][0], b)
            else:
                merged.append((a, b))
        free[:] = merged

    items = []
    rounds = [0]
    clens = []
    st_mode = mode
    cmax = chunk
    for r, group in enumerate(order):
        merges = [n for n in group if n.a is not None]
        total = sum(n.need_hi - n.need_lo for n in merges)
        C = max(chunk, -(-total // lanes))
        C = -(-C // chunk) * chunk
        cmax = max(cmax, C)
        for n in group:
            nout = n.need_hi - n.need_lo
            n.store = (_ceil_to(nout, ALIGN) if n.a is not None else nout) + SENT_W
            n.off = alloc(n.store)
        sorts = []
        chunks = []
        for n in group:
            nout = n.need_hi - n.need_lo
            if n.line is not None:
                b0, stride, cnt, nl, lstep = n.line
                N = _pow2_at_least(cnt * nl)
                assert N <= SORT_MAX and b0 < MAX_OFF and stride < MAX_OFF and n.off < MAX_OFF
                assert 1 <= nl <= 7 and 0 <= lstep < (1 << LSTEP_BITS)
                sorts.append((N, (b0 | (cnt << OFF_BITS), stride | (n.need_lo << OFF_BITS),
                                  n.off | (nout << OFF_BITS),
                                  SORT_FLAG | N | (nl << 6) | (lstep << LSTEP_SHIFT))))
                continue
            (aoff, na), (boff, nb), r0 = _window_inputs(n)
            assert 0 <= r0 and r0 + nout <= na + nb, (n.nid, r0, nout, na, nb)
            # chunks at multiples of C; a ragged end gets one more chunk that
            # ends at the next multiple of ALIGN (it overlaps the one before,
            # rewriting the same values, and its few outputs past the end land
            # in the sentinel slots, which its lane then rewrites)
            starts = list(range(0, nout - C + 1, C)) if nout >= C else [0]
            if nout > C and nout % C:
                starts.append(_ceil_to(nout, ALIGN) - C)
            for ci, c0 in enumerate(starts):
                last = ci == len(starts) - 1
                nvalid = min(C, nout - c0)
                rr = r0 + c0
                lo_i, hi_i = max(0, rr - nb), min(rr, na)
                steps = max(hi_i - lo_i, 0).bit_length()
                for off in (aoff, boff, n.off + c0):
                    assert 0 <= off < MAX_OFF
                assert na < MAX_LEN and nb < MAX_LEN and nvalid < MAX_LEN and rr < (1 << STEP_SHIFT)
                assert steps < 16
                chunks.append((steps, (aoff | (na << OFF_BITS), boff | (nb << OFF_BITS),
                                       (n.off + c0) | (nvalid << OFF_BITS),
                                       rr | (steps << STEP_SHIFT) | (LAST_BIT if last else 0))))
        # sorts first (by network size), then chunks by search depth: the 64
        # lanes of a wave then run the same code with about the same trip count
        sorts.sort(key=lambda t: t[0])
        chunks.sort(key=lambda t: -t[0])
        items.extend(it for _, it in sorts)
        items.extend(it for _, it in chunks)
        rounds.append(len(items))
        clens.append(C)
        # free storage whose last reader ran in this round
        for n in work:
            if last_read.get(n.nid, -1) == r and n.off >= 0:
                release(n.off, n.store)
                n.off = -2 - n.off  # mark released (keeps the value recoverable)
    arena = _ceil_to(peak + READ_PAST, 2 * ALIGN)
    it = np.array(items, dtype=np.int64).reshape(-1, 4)
    m = (1 << OFF_BITS) - 1
    if len(it):
        isort = (it[:, 3] & SORT_FLAG) != 0
        mg = it[~isort]
        # merge reads: one element before each window (co-rank guard) up to
        # READ_PAST elements after the window end; writes: the chunk's
        # outputs rounded up to four, then SENT_W sentinels
        for col in range(2):
            assert np.all((mg[:, col] & m) >= 1)
            assert np.all((mg[:, col] & m) + (mg[:, col] >> OFF_BITS) + READ_PAST <= arena)
        nv = mg[:, 2] >> OFF_BITS
        assert np.all((mg[:, 2] & m) + np.maximum(-(-nv // 4) * 4, nv + SENT_W) <= arena)
        assert np.all((mg[:, 2] & m) % ALIGN == 0) and arena % (2 * ALIGN) == 0
        srt = it[isort]
        assert np.all((srt[:, 0] & m) + (srt[:, 1] & m) * ((srt[:, 0] >> OFF_BITS) - 1) < GUARD + fw * fh * fd)
        assert np.all((srt[:, 2] & m) + (srt[:, 2] >> OFF_BITS) + SENT_W <= arena)
    outputs = []
    for (n, lo, hi) in outs:
        off = n.off if n.off >= 0 else (-2 - n.off)
        outputs.append(off + (lo - n.need_lo))
    assert all(0 <= o < peak for o in outputs)
    merges = [n for n in work if n.a is not None]
    merge_outputs = sum(n.need_hi - n.need_lo for n in merges)
    sort_outputs = sum(n.need_hi - n.need_lo for n in work if n.line is not None)
    by_role = {}
    for n in work:
        by_role[n.role] = by_role.get(n.role, 0) + (n.need_hi - n.need_lo)
    nmerge_items = int(np.sum((it[:, 3] & SORT_FLAG) == 0)) if len(it) else 0
    # compare-exchanges of the sorting networks the sort items run
    sort_ces = sum(_OEMS_CES[int(w3) & 63] for w3 in it[:, 3] if int(w3) & SORT_FLAG) if len(it) else 0
    st = {"rounds": len(order), "chunks": nmerge_items, "round_mode": st_mode, "sorts": len(items) - nmerge_items,
          "merge_outputs": merge_outputs, "sort_outputs": sort_outputs,
          "per_pixel_by_role": {r: round(v / npx, 1) for r, v in sorted(by_role.items())},
          "per_pixel_outputs": merge_outputs / npx, "arena": arena,
          "per_pixel_sort_ces": sort_ces / npx,
          "merges": len(merges)}
    # recursion level of each round (non-decreasing): the shallowest level
    # among its nodes (the level whose core the round advances; with ASAP
    # rounds later levels' sorts and reductions run early), as a running max
    rphase, top = [], 0
    for group in order:
        top = max(top, min(n.phase for n in group))
        rphase.append(top)
    return Schedule(0, 0, 0, fw, fh, np.array(items, dtype=np.uint32).reshape(-1, 4),
                    np.array(rounds, dtype=np.int32), np.array(clens, dtype=np.int32),
                    np.array(rphase, dtype=np.int32), np.array(outputs, dtype=np.int32), arena,
                    merge_outputs, st, 0, fd)


# ------------------------------------------------------------- CPU model

def _sentinel(dtype) -> int:
    return {1: 0xFF, 2: 0xFFFF}.get(np.dtype(dtype).itemsize, 0xFFFFFFFF)


def _to_keys(win: np.ndarray, dtype, byte_elements: bool = False):
    """Elements as the kernel holds them: 16-bit for 8/16-bit data (8-bit
    for 8-bit data with byte_elements), else 32-bit (float32 through the
    order-preserving key)."""
    et = np.uint16 if np.dtype(dtype).itemsize <= 2 else np.uint32
    if byte_elements and np.dtype(dtype) == np.uint8:
        et = np.uint8
    if dtype == np.float32:
        b = win.view(np.uint32)
        return et, b ^ np.where(b >> 31 == 1, np.uint32(0xFFFFFFFF), np.uint32(0x80000000))
    return et, win.astype(et)


def _from_keys(out: np.ndarray, dtype) -> np.ndarray:
    if dtype == np.float32:
        k32 = out.astype(np.uint32)
        bits = k32 ^ np.where(k32 >> 31 == 1, np.uint32(0x80000000), np.uint32(0xFFFFFFFF))
        return bits.view(np.float32)
    return out.astype(dtype)


def _execute(S: Schedule, keys: np.ndarray, et, clamp: bool, exact: bool) -> np.ndarray:
    """Run every round's items on T arenas at once (keys: (T, footprint)
    elements) and return the (T, tile pixels) medians. The arena starts
    filled with noise, so nothing may rely on unwritten slots."""
    T = keys.shape[0]
    MAXV = _sentinel(et)
    g = np.random.default_rng(S.arena)
    arena = g.integers(0, MAXV + 1, size=(T, S.arena), dtype=np.uint64).astype(et)
    arena[:, SENTINEL_SLOT:GUARD] = MAXV
    arena[:, GUARD:GUARD + keys.shape[1]] = keys
    mask = (1 << OFF_BITS) - 1
    rows = np.arange(T)
    for ri in range(len(S.rounds) - 1):
        C = int(S.chunk_len[ri])
        rnd = S.items[S.rounds[ri]:S.rounds[ri + 1]].astype(np.int64)
        # a wave searches with its largest step count; any count at least an
        # item's own gives its position, and the model takes the round's
        mg3 = rnd[(rnd[:, 3] & SORT_FLAG) == 0, 3]
        wave_steps = int(((mg3 >> STEP_SHIFT) & 15).max()) if len(mg3) else 0
        for c in rnd:
            w0, w1, w2, w3 = (int(v) for v in c)
            if w3 & SORT_FLAG:
                base, n = w0 & mask, w0 >> OFF_BITS
                stride, lo = w1 & mask, w1 >> OFF_BITS
                ooff, cnt = w2 & mask, w2 >> OFF_BITS
                N, nl, lstep = w3 & 63, (w3 >> 6) & 7, (w3 >> LSTEP_SHIFT) & ((1 << LSTEP_BITS) - 1)
                assert n * nl <= N <= SORT_MAX
                vals = np.full((T, N), MAXV, dtype=et)
                idx = (base + lstep * np.arange(nl)[:, None] + stride * np.arange(n)[None, :]).reshape(-1)
                vals[:, :n * nl] = arena[:, idx]
                vals = np.sort(vals, axis=1)
                arena[:, ooff:ooff + cnt] = vals[:, lo:lo + cnt]
                arena[:, ooff + cnt:ooff + cnt + SENT_W] = MAXV
                continue
            aoff, na = w0 & mask, w0 >> OFF_BITS
            boff, nb = w1 & mask, w1 >> OFF_BITS
            ooff, nvalid = w2 & mask, w2 >> OFF_BITS
            r0, steps, last = w3 & ((1 << STEP_SHIFT) - 1), (w3 >> STEP_SHIFT) & 15, bool(w3 & LAST_BIT)
            if not exact:
                A = arena[:, aoff:aoff + na]
                B = arena[:, boff:boff + nb]
                m = np.sort(np.concatenate([A, B], axis=1), axis=1)
                arena[:, ooff:ooff + nvalid] = m[:, r0:r0 + nvalid]
                if last:
                    arena[:, ooff + nvalid:ooff + nvalid + SENT_W] = MAXV
                continue
            # co-rank search by halving steps, reads clamped into the window
            # (a probe past the range reads its last element; taking it means
            # taking every position); a wave runs its largest step count, and
            # any count at least the item's own gives its position
            lo_i, hi_i = max(0, r0 - nb), min(r0, na)
            pos = np.full(T, lo_i, dtype=np.int64)
            for s in range(wave_steps - 1, -1, -1):
                tc = np.minimum(pos + (1 << s) - 1, hi_i - 1)
                av = arena[rows, aoff + tc]
                bv = arena[rows, boff + r0 - 1 - tc]
                pos = np.where(av <= bv, tc + 1, pos)
            # merge steps of four outputs: the four smallest of A[ia..ia+3]
            # and B[ib..ib+3] are min(A[ia+i], B[ib+3-i]) (a half-cleaner),
            # i taken from A exactly when A[ia+i] <= B[ib+3-i]; they are
            # written in order after a bitonic sort of four. The 8- and
            # 16-bit kernels advance the B head by the B elements taken (it
            # lags where the clamp pulls the A head back), the 32-bit kernel
            # sets it from the A head
            ia = pos.copy()
            b_counts = np.dtype(et).itemsize <= 2
            ib = r0 - ia
            for q0 in range(0, nvalid, 4):
                if not b_counts:
                    ib = r0 + q0 - ia
                av = [arena[rows, aoff + ia + i] for i in range(4)]
                bv = [arena[rows, boff + ib + i] for i in range(4)]
                take = [av[i] <= bv[3 - i] for i in range(4)]
                c = [np.where(take[i], av[i], bv[3 - i]) for i in range(4)]
                for (x, y) in ((0, 2), (1, 3), (0, 1), (2, 3)):
                    c[x], c[y] = np.minimum(c[x], c[y]), np.maximum(c[x], c[y])
                for i in range(4):
                    arena[:, ooff + q0 + i] = c[i]
                nA = sum(t.astype(np.int64) for t in take)
                ia = ia + nA
                ib = ib + 4 - nA
                if clamp:
                    ia = np.minimum(ia, na)
            if last:
                arena[:, ooff + nvalid:ooff + nvalid + SENT_W] = MAXV
    return arena[:, S.outputs]


def run_schedule_on_image(S: Schedule, img: np.ndarray, exact_merge_path: bool = False,
                          byte_elements: bool = False) -> np.ndarray:
    """Execute a schedule on every root tile of img (replicate border).

    With exact_merge_path=False each merge chunk is checked against a sort of
    its two input windows; with True every item is executed the way the
    kernel executes it, for all tiles at once: the co-rank search with its
    step count and clamped reads, the C merge steps that read the sentinels
    and run past the needed outputs, the sentinel writes, and the ia clamp
    that 16-bit and 32-bit data use (8-bit data held in 16-bit elements never
    equals the sentinel and runs without it). With byte_elements, 8-bit data
    is held in 8-bit elements, as the one-plane kernel holds it: the
    sentinel 0xff then equals the largest data value and the clamp is on."""
    kw, kh, tw, th = S.kw, S.rows, S.tw, S.th
    H, W = img.shape
    nty, ntx = -(-H // th), -(-W // tw)
    ys = np.clip(np.arange(nty * th + kh - 1) - (kh - 1) // 2, 0, H - 1)
    xs = np.clip(np.arange(ntx * tw + kw - 1) - (kw - 1) // 2, 0, W - 1)
    pad = img[ys][:, xs]
    win = np.lib.stride_tricks.sliding_window_view(pad, (S.fh, S.fw))[::th, ::tw]
    T = nty * ntx
    et, keys = _to_keys(np.ascontiguousarray(win.reshape(T, S.fw * S.fh)), img.dtype, byte_elements)
    med = _execute(S, keys, et, img.dtype.itemsize >= 2 or et == np.uint8, exact_merge_path)
    out = np.empty((nty * th, ntx * tw), dtype=et)
    for i in range(tw * th):
        py, px = divmod(i, tw)
        out[py::th, px::tw] = med[:, i].reshape(nty, ntx)
    return _from_keys(out[:H, :W], img.dtype)


def run_schedule_on_volume(S: Schedule, vol: np.ndarray, exact_merge_path: bool = False) -> np.ndarray:
    """As run_schedule_on_image, for a 3-D schedule (schedule3) on every root
    tile of a (D, H, W) volume (each axis clamped)."""
    kx, ky, kz, tx, ty, tz = S.k, S.kh, S.kz, S.tw, S.th, S.tz
    Dd, H, W = vol.shape
    ntz, nty, ntx = -(-Dd // tz), -(-H // ty), -(-W // tx)
    zs = np.clip(np.arange(ntz * tz + kz - 1) - (kz - 1) // 2, 0, Dd - 1)
    ys = np.clip(np.arange(nty * ty + ky - 1) - (ky - 1) // 2, 0, H - 1)
    xs = np.clip(np.arange(ntx * tx + kx - 1) - (kx - 1) // 2, 0, W - 1)
    pad = vol[zs][:, ys][:, :, xs]
    win = np.lib.stride_tricks.sliding_window_view(pad, (S.fd, S.fh, S.fw))[::tz, ::ty, ::tx]
    T = ntz * nty * ntx
    et, keys = _to_keys(np.ascontiguousarray(win.reshape(T, S.fw * S.fh * S.fd)), vol.dtype)
    med = _execute(S, keys, et, vol.dtype.itemsize >= 2, exact_merge_path)
    out = np.empty((ntz * tz, nty * ty, ntx * tx), dtype=et)
    for i in range(tx * ty * tz):
        pz, rem = divmod(i, tx * ty)
        py, px = divmod(rem, tx)
        out[pz::tz, py::ty, px::tx] = med[:, i].reshape(ntz, nty, ntx)
    return _from_keys(out[:Dd, :H, :W], vol.dtype)


def _merge_path_chunk(A, B, r0, n):
    """Co-rank search + sequential merge, A first on ties (stable)."""
    na, nb = len(A), len(B)
    lo, hi = max(0, r0 - nb), min(r0, na)
    while lo < hi:                   # smallest i with A[i] > B[r0-i-1]
        i = (lo + hi) // 2
        if A[i] <= B[r0 - i - 1]:
            lo = i + 1
        else:
            hi = i
    i, j = lo, r0 - lo
    out = []
    for _ in range(n):
        if j >= nb or (i < na and A[i] <= B[j]):
            out.append(A[i]); i += 1
        else:
            out.append(B[j]); j += 1
    return out
