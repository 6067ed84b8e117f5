"""Build-time schedule generator for the data-aware hierarchical median filter.

The data-aware variant (Sugy 2025, Section 5) keeps the tile recursion of
Section 3 but realises every sort and merge with data-dependent two-way
merges in LDS:

* sorting a column, an extra row or a group of corners is a binary reduction
  of two-way merges starting from single footprint values (Section 5.1:
  many small sorts, merged pairwise);
* a multi-way merge is a binary reduction of two-way merges, halving the
  number of lists each round (Section 5.1);
* every two-way merge is executed with merge path: its output is cut into
  chunks, each chunk finds its start in both inputs by a co-rank binary
  search and then merges sequentially (Section 5.1).

Forgetting (Section 2.2) and pruning become output windows: after a merge
into a core only the middle min(n, u+1) ranks are kept, and a backward pass
from the medians gives every list the window of ranks any consumer can read,
so no element outside it is ever produced.

The generator records, for one root tile of t_w x t_h pixels, a DAG of list
nodes, assigns each node the recursion level (phase) that creates it,
schedules the merges of each phase in dependency rounds, allocates LDS
(first fit, freed after the last reader) and emits compact descriptors:

* one chunk = 4 words: a_off | na << 18, b_off | nb << 18, out_off | n << 18,
  r0 (the rank, within the merge of the two input windows, of the chunk's
  first output);
* rounds = ranges of chunks separated by a work-group barrier;
* outputs = LDS offset of each pixel's median.

Offsets are in elements of the LDS arena; the raw footprint occupies
[0, fw*fh) row-major with fw = k+t_w-1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CHUNK = 4           # shortest merge-path chunk (outputs)
LANES = 512         # threads of a data-aware work-group: a round's outputs are
                    # cut into about this many chunks
OFF_BITS = 18       # arena offsets and sizes share a 32-bit word
MAX_OFF = 1 << OFF_BITS
MAX_LEN = 1 << (32 - OFF_BITS)


@dataclass
class Node:
    nid: int
    size: int                       # full logical length
    a: tuple | None = None          # (node, lo, hi) input views
    b: tuple | None = None
    raw: tuple | None = None        # (x, y) for a single footprint value
    phase: int = 0
    need_lo: int = 0
    need_hi: int = 0
    consumers: list = field(default_factory=list)
    off: int = -1
    rnd: int = -1
    role: str = ""


class Dag:
    def __init__(self, fw: int):
        self.nodes: list[Node] = []
        self.fw = fw
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

    def sort(self, values: list[tuple]) -> tuple:
        return self.reduce(values)


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
        return D.sort([D.raw(x, y) for y in ys])

    def row(y, xs):
        D.role = "sort_row"
        return D.sort([D.raw(x, y) for x in xs])

    D.phase = 0
    cols = [col(x, core_y) for x in core_x]
    D.role = "core_init"
    core = D.reduce(cols)
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
                    cs = D.sort([D.raw(x, y) for x in added])
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
                    cs = D.sort([D.raw(x, y) for y in added])
                    D.role = "extend"
                    ncols[x] = D.merge(cl, cs)
                children.append((ox, coy, w, hh, c, ncols, nrows))
        for ch in children:
            recurse(*ch, level + 1)

    recurse(0, 0, tw, th, core, xcols, xrows, 0)
    outs = [outputs[(px, py)] for py in range(th) for px in range(tw)]
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
    chunks: np.ndarray          # (n_chunks, 4) uint32
    rounds: np.ndarray          # (n_rounds + 1,) int32 chunk offsets
    outputs: np.ndarray         # (tw*th,) int32 arena offsets
    arena: int                  # elements of LDS the schedule needs
    merge_outputs: int          # elements produced by all merges
    stats: dict
    kh: int = 0                 # window rows (0: k, the square filter)

    @property
    def kw(self) -> int:
        return self.k

    @property
    def rows(self) -> int:
        return self.kh or self.k


def _window_inputs(n: Node):
    """Input windows (storage offset, count) and the first output rank
    relative to the merge of those windows, for node n's needed window."""
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
        # storage of m covers [m.need_lo, m.need_hi)
        off = m.off + (s_lo + a0 - (m.need_lo if m.raw is None else 0))
        res.append((off, a1 - a0))
        starts.append(a0)
    r0 = lo - starts[0] - starts[1]
    return res[0], res[1], r0


def schedule(k: int, tw: int, th: int, chunk: int = CHUNK, lanes: int = LANES,
             kh: int | None = None) -> Schedule:
    """Rounds of windowed merges for root tile tw x th. Every round's outputs
    are cut into chunks of max(chunk, ceil(outputs / lanes)) so that one
    round keeps about `lanes` threads busy with chains as short as the round
    allows (a lane runs a co-rank search, then its chunk sequentially)."""
    kh = k if kh is None else kh
    D, outs = build_dag(k, tw, th, kh)
    propagate_windows(D, outs)
    fw, fh = k + tw - 1, kh + th - 1
    merges = [n for n in D.nodes if n.a is not None and n.need_hi > n.need_lo]
    # rounds: per phase, ASAP by dependency depth within the phase
    depth = {}
    for n in merges:
        d = 0
        for src in (n.a, n.b):
            m = src[0]
            if m.a is not None and m.need_hi > m.need_lo and m.phase == n.phase:
                d = max(d, depth[m.nid] + 1)
        depth[n.nid] = d
    phases = sorted(set(n.phase for n in merges))
    order = []
    for p in phases:
        pm = [n for n in merges if n.phase == p]
        dmax = max(depth[n.nid] for n in pm)
        for d in range(dmax + 1):
            order.append([n for n in pm if depth[n.nid] == d])
    for r, group in enumerate(order):
        for n in group:
            n.rnd = r
    # last round in which each node is read (outputs: forever)
    last_read = {}
    for n in merges:
        for src in (n.a, n.b):
            m = src[0]
            last_read[m.nid] = max(last_read.get(m.nid, -1), n.rnd)
    for (n, _, _) in outs:
        last_read[n.nid] = len(order) + 1
    # allocation: raw footprint fixed at [0, fw*fh); first fit for the rest
    for n in D.nodes:
        if n.raw is not None:
            n.off = n.raw[1] * fw + n.raw[0]
    free = [(fw * fh, 1 << 40)]      # (start, end) holes, sorted
    peak = fw * fh
    live_by_end = {}

    def alloc(size):
        nonlocal peak
        for i, (s, e) in enumerate(free):
            if e - s >= size:
                free[i] = (s + size, e)
                if free[i][0] == free[i][1]:
                    free.pop(i)
                peak = max(peak, s + size)
                return s
        raise RuntimeError("arena exhausted")

    def release(s, size):
        free.append((s, s + size))
        free.sort()
        merged = []
        for a, b in free:
            if merged and merged[-1][1] == a:
                merged[-1] = (merged[-1][0], b)
            else:
                merged.append((a, b))
        free[:] = merged

    chunks = []
    rounds = [0]
    for r, group in enumerate(order):
        for n in group:
            n.off = alloc(n.need_hi - n.need_lo)
        total = sum(n.need_hi - n.need_lo for n in group)
        step = max(chunk, -(-total // lanes))
        rchunks = []
        for n in group:
            (aoff, na), (boff, nb), r0 = _window_inputs(n)
            nout = n.need_hi - n.need_lo
            assert 0 <= r0 and r0 + nout <= na + nb, (n.nid, r0, nout, na, nb)
            for c0 in range(0, nout, step):
                c = min(step, nout - c0)
                for off in (aoff, boff, n.off + c0):
                    assert 0 <= off < MAX_OFF
                assert na < MAX_LEN and nb < MAX_LEN and c < MAX_LEN
                # a lane's work: co-rank search steps plus sequential outputs
                span = min(r0 + c0, na) - max(0, r0 + c0 - nb)
                cost = max(span, 0).bit_length() + c
                rchunks.append((cost, (aoff | (na << OFF_BITS), boff | (nb << OFF_BITS),
                                       (n.off + c0) | (c << OFF_BITS), r0 + c0)))
        # costliest first: the chunks of one wave (64 consecutive lanes) then
        # take about the same time, so fewer lanes sit idle in a busy wave
        rchunks.sort(key=lambda t: -t[0])
        chunks.extend(ch for _, ch in rchunks)
        rounds.append(len(chunks))
        # free storage whose last reader ran in this round
        for n in merges:
            if last_read.get(n.nid, -1) == r and n.off >= 0:
                release(n.off, n.need_hi - n.need_lo)
                n.off = -2 - n.off  # mark released (keeps the value recoverable)
    # every access of the kernel stays inside the arena
    ch = np.array(chunks, dtype=np.int64).reshape(-1, 4)
    if len(ch):
        m = (1 << OFF_BITS) - 1
        for col in range(3):
            assert np.all((ch[:, col] & m) + (ch[:, col] >> OFF_BITS) <= peak)
        assert np.all(ch[:, 3] + (ch[:, 2] >> OFF_BITS) <= (ch[:, 0] >> OFF_BITS) + (ch[:, 1] >> OFF_BITS))
    outputs = []
    for (n, lo, hi) in outs:
        off = n.off if n.off >= 0 else (-2 - n.off)
        if n.raw is not None:
            outputs.append(n.off)
        else:
            outputs.append(off + (lo - n.need_lo))
    assert all(0 <= o < peak for o in outputs)
    merge_outputs = sum(n.need_hi - n.need_lo for n in merges)
    by_role = {}
    for n in merges:
        by_role[n.role] = by_role.get(n.role, 0) + (n.need_hi - n.need_lo)
    st = {"rounds": len(order), "chunks": len(chunks), "merge_outputs": merge_outputs,
          "per_pixel_by_role": {r: round(v / (tw * th), 1) for r, v in sorted(by_role.items())},
          "per_pixel_outputs": merge_outputs / (tw * th), "arena": peak,
          "merges": len(merges)}
    return Schedule(k, tw, th, fw, fh, np.array(chunks, dtype=np.uint32).reshape(-1, 4),
                    np.array(rounds, dtype=np.int32), np.array(outputs, dtype=np.int32), peak,
                    merge_outputs, st, kh)


# ------------------------------------------------------------- CPU model

def run_schedule_on_image(S: Schedule, img: np.ndarray, exact_merge_path: bool = False) -> np.ndarray:
    """Execute a schedule on every root tile of img (replicate border).

    Each chunk merges its two input windows and keeps ranks [r0, r0+n); with
    exact_merge_path the chunk is executed the way the kernel does it (co-rank
    binary search, then a sequential merge), per tile."""
    kw, kh, tw, th = S.kw, S.rows, S.tw, S.th
    H, W = img.shape
    nty, ntx = -(-H // th), -(-W // tw)
    ys = np.clip(np.arange(nty * th + kh - 1) - (kh - 1) // 2, 0, H - 1)
    xs = np.clip(np.arange(ntx * tw + kw - 1) - (kw - 1) // 2, 0, W - 1)
    pad = img[ys][:, xs]
    win = np.lib.stride_tricks.sliding_window_view(pad, (S.fh, S.fw))[::th, ::tw]
    T = nty * ntx
    arena = np.zeros((T, S.arena), dtype=img.dtype)
    arena[:, :S.fw * S.fh] = win.reshape(T, S.fw * S.fh)
    mask = (1 << OFF_BITS) - 1
    for ri in range(len(S.rounds) - 1):
        for c in S.chunks[S.rounds[ri]:S.rounds[ri + 1]]:
            aoff, na = int(c[0]) & mask, int(c[0]) >> OFF_BITS
            boff, nb = int(c[1]) & mask, int(c[1]) >> OFF_BITS
            ooff, n = int(c[2]) & mask, int(c[2]) >> OFF_BITS
            r0 = int(c[3])
            A = arena[:, aoff:aoff + na]
            B = arena[:, boff:boff + nb]
            if not exact_merge_path:
                m = np.sort(np.concatenate([A, B], axis=1), axis=1)
                arena[:, ooff:ooff + n] = m[:, r0:r0 + n]
            else:
                for t in range(T):
                    arena[t, ooff:ooff + n] = _merge_path_chunk(A[t], B[t], r0, n)
    out = np.empty((nty * th, ntx * tw), dtype=img.dtype)
    for i, off in enumerate(S.outputs):
        py, px = divmod(i, tw)
        out[py::th, px::tw] = arena[:, off].reshape(nty, ntx)
    return out[:H, :W]


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

