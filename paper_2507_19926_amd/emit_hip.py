"""Emit HIP source for the data-oblivious kernels from the generated networks.

For every configured (k, t_w, t_h) this writes one translation unit that

* defines the straight-line selection network of ``netgen.build_tile_program``
  as a device function over a value type V (``uint32_t`` for 32-bit data,
  ``us2`` = two packed 16-bit lanes for 8/16-bit data), reading sorted
  columns and raw values from LDS at compile-time offsets and handing each
  median to a sink as soon as it is produced;
* defines the odd-even merge sort of the column length as a register network;
* instantiates ``mf_obl_kernel`` (csrc/mf_oblivious.hip) for both value types
  and registers their launchers in a table the dispatcher reads.

Only live operations are emitted (pruning = dead-code elimination), in the
order a depth-first walk from each median needs them, which keeps register
pressure close to the tile recursion's own state.
"""
from __future__ import annotations

import os

from . import netgen as ng


def _net_body(P: ng.Prog, k: int, tw: int, th: int, indent: str = "    ", kh: int | None = None) -> list[str]:
    """Emit the live ops. Every load stays inside the root footprint
    (x < k+tw-1, y < kh+th-1) and the sorted column length (i < kh-th+1): the
    kernel's LDS buffers are sized for exactly that (kh = k: square)."""
    kh = k if kh is None else kh
    lines = []
    order = ng.demand_order(P)
    out_index = {}
    for i, o in enumerate(P.outputs):
        out_index.setdefault(o, []).append(i)
    for v in order:
        op = P.ops[v]
        if op[0] == ng.LD:
            kind, a, b = op[1]
            if kind == "col":
                x, i = a, b
                assert 0 <= x < k + tw - 1 and 0 <= i < kh - th + 1, op
                lines.append("%sconst V v%d = col[(%d) * Q + %d];" % (indent, v, i * tw + x % tw, x // tw))
            else:
                x, y = a, b
                assert 0 <= x < k + tw - 1 and 0 <= y < kh + th - 1, op
                lines.append("%sconst V v%d = raw[(%d) * Q + %d];" % (indent, v, y * tw + x % tw, x // tw))
        else:
            lines.append("%sconst V v%d = %s(v%d, v%d);"
                         % (indent, v, "vmin" if op[0] == ng.MIN else "vmax", op[1], op[2]))
        for i in out_index.get(v, ()):
            assert 0 <= i < tw * th
            lines.append("%ssink(%d, %d, v%d);" % (indent, i % tw, i // tw, v))
    return lines


def sort_network_pairs(n: int) -> list[tuple[int, int]]:
    """Compare-exchange pairs (i, j), i < j, of the odd-even merge sort of n
    wires, in an order valid for in-place execution."""
    P = ng.Prog()
    wires = [P.load(("in", i)) for i in range(n)]
    outs = ng.sort(P, wires)
    # Replay: each CAS creates a (min, max) pair; track which wire holds which
    # SSA value to recover the in-place pairs.
    holder = {v: i for i, v in enumerate(wires)}
    pairs = []
    for v, op in enumerate(P.ops):
        if op[0] == ng.MIN:
            a, b = op[1], op[2]
            i, j = sorted((holder[a], holder[b]))
            pairs.append((i, j))
            mx = P._memo[(ng.MAX, a, b)]
            # the min lands on the lower wire, the max on the upper one
            holder[v] = i
            holder[mx] = j
    assert [holder[o] for o in outs] == list(range(n))
    return pairs


def emit_sort(n: int) -> str:
    lines = ["template <class V> __device__ __forceinline__ void mf_sort_%d(V* a) {" % n]
    for i, j in sort_network_pairs(n):
        lines.append("    { const V lo = vmin(a[%d], a[%d]); a[%d] = vmax(a[%d], a[%d]); a[%d] = lo; }"
                     % (i, j, j, i, j, i))
    lines.append("}")
    return "\n".join(lines)


LDS_BYTES = 160 * 1024


def persistent_lds_bytes(kw: int, kh: int, tw: int, th: int, ry: int, nw: int) -> int:
    """LDS of the persistent oblivious kernel (footprint union, sorted column
    segments, staging chunks, output tile) for the larger of its two value
    types, following the block geometry of csrc/mf_oblivious.hip (MfObGeom);
    the kernel's own static_assert checks the same budget at compile time."""
    worst = 0
    for pack in (True, False):
        bwh = 64 * tw
        cols = bwh + kw - 1
        ty = nw * ry
        rows = ty * th + kh - 1
        q = -(-cols // tw)
        raw = rows * tw * q * 4
        colb = ty * (kh - th + 1) * tw * q * 4
        span = bwh + cols if pack else cols
        nch = (18 + span * (2 if pack else 4) + 15) // 16
        stage = -(-rows * nch // 64) * 64 * 16
        out = ty * th * (2 * bwh if pack else bwh) * (2 if pack else 4)
        worst = max(worst, raw + colb + stage + out)
    return worst


def net_name(k: int, tw: int, th: int, inline: bool, kh: int | None = None) -> str:
    win = "%d" % k if kh is None or kh == k else "%dx%d" % (k, kh)
    return "MfNet_k%s_%dx%d%s" % (win, tw, th, "i" if inline else "")


def emit_config_tu(k: int, tw: int, th: int, shapes, inline: bool = False, kh: int | None = None) -> str:
    """One translation unit: the network for (k, tw, th) and one kernel
    instantiation per (tile rows per wave, waves per work-group) shape. The
    window is k columns by kh rows (kh = k: the square filter). Square
    networks get the persistent form up to k = 17; rectangular ones whenever
    its LDS fits."""
    kh = k if kh is None else kh
    if kh == k:
        persistent = k <= 17
    else:
        persistent = not inline and all(persistent_lds_bytes(k, kh, tw, th, ry, nw) <= LDS_BYTES
                                        for (ry, nw) in shapes)
    P = ng.build_tile_program(k, tw, th, inline_cols=inline, kh=kh)
    cnt = ng.op_counts(P)
    peak = ng.peak_live(P, ng.demand_order(P))
    name = net_name(k, tw, th, inline, kh)
    lc = kh - th + 1
    body = _net_body(P, k, tw, th, indent="        ", kh=kh)
    win = "k=%d" % k if kh == k else "window %dx%d (columns x rows)" % (k, kh)
    src = [
        "// Generated: hierarchical selection network, %s, root tile %dx%d." % (win, tw, th),
        "// live min/max ops per root tile: %d (%.2f per pixel), LDS loads: %d"
        % (cnt["minmax"], cnt["minmax"] / (tw * th), cnt["loads"]),
        '#include "mf_oblivious.hip"',
        "",
        emit_sort(lc) if lc > 1 else "template <class V> __device__ __forceinline__ void mf_sort_1(V*) {}",
        "",
        "struct %s {" % name,
        "    static constexpr int K = %d, KH = %d, TW = %d, TH = %d, LC = %d;" % (k, kh, tw, th, lc),
        "    static constexpr bool INLINE_COLS = %s;" % ("true" if inline else "false"),
        "    static constexpr bool PERSISTENT = %s;" % ("true" if persistent else "false"),
        # networks whose live values just about fit 256 VGPRs are built for
        # two waves per SIMD (plain and batched kernels, packed 16-bit data)
        "    static constexpr int MIN_WAVES = %d;" % (2 if peak <= 270 else 1),
        "    template <class V> static __device__ __forceinline__ void sort_column(V* a) { mf_sort_%d(a); }" % lc,
        "    template <int Q, class V, class Sink>",
        "    static __device__ __forceinline__ void run(const V* __restrict__ col,",
        "                                               const V* __restrict__ raw, Sink& sink) {",
    ] + body + [
        "    }",
        "};",
        "",
    ] + ["MF_OBL_INSTANTIATE(%s, %d, %d)" % (name, ry, nw) for (ry, nw) in shapes] + [
        "",
    ]
    return "\n".join(src)


def generate(out_dir: str, configs, rect_configs=()) -> list[str]:
    """Write one .hip per config plus the launcher tables (square windows:
    mf_obl_table.inc; rectangular windows, configs (k_w, k_h, t_w, t_h, rows
    per wave, waves[, inline]): mf_obl_rect_table.inc); return the .hip
    paths."""
    os.makedirs(out_dir, exist_ok=True)
    paths = []
    table = []
    tiles = {}
    for cfg in configs:
        (k, tw, th, ry, nw), inline = cfg[:5], (len(cfg) > 5 and cfg[5])
        tiles.setdefault((k, tw, th, inline), []).append((ry, nw))
        table.append("MF_OBL_ENTRY(%s, %d, %d, %d, %d, %d, %d)"
                     % (net_name(k, tw, th, inline), k, tw, th, ry, nw, 1 if inline else 0))
    for (k, tw, th, inline), shapes in tiles.items():
        path = os.path.join(out_dir, "mf_obl_k%d_%dx%d%s.hip" % (k, tw, th, "i" if inline else ""))
        text = emit_config_tu(k, tw, th, shapes, inline)
        old = open(path).read() if os.path.exists(path) else None
        if old != text:
            with open(path, "w") as f:
                f.write(text)
        paths.append(path)
    rtable = []
    rtiles = {}
    for cfg in rect_configs:
        (kw, kh, tw, th, ry, nw), inline = cfg[:6], (len(cfg) > 6 and cfg[6])
        assert kw != kh
        rtiles.setdefault((kw, kh, tw, th, inline), []).append((ry, nw))
        rtable.append("MF_OBL_RECT_ENTRY(%s, %d, %d, %d, %d, %d, %d, %d)"
                      % (net_name(kw, tw, th, inline, kh), kw, kh, tw, th, ry, nw, 1 if inline else 0))
    for (kw, kh, tw, th, inline), shapes in rtiles.items():
        path = os.path.join(out_dir, "mf_obl_k%dx%d_%dx%d%s.hip" % (kw, kh, tw, th, "i" if inline else ""))
        text = emit_config_tu(kw, tw, th, shapes, inline, kh)
        old = open(path).read() if os.path.exists(path) else None
        if old != text:
            with open(path, "w") as f:
                f.write(text)
        paths.append(path)
    for name, head, rows in (
            ("mf_obl_table.inc",
             "// (network, k, t_w, t_h, tile rows per wave, waves per work-group, inline column sort)", table),
            ("mf_obl_rect_table.inc",
             "// (network, k_w, k_h, t_w, t_h, tile rows per wave, waves per work-group, inline column sort)",
             rtable)):
        tpath = os.path.join(out_dir, name)
        text = "// Generated list of compiled oblivious configurations:\n" + head + "\n" + "\n".join(rows) + "\n"
        old = open(tpath).read() if os.path.exists(tpath) else None
        if old != text:
            with open(tpath, "w") as f:
                f.write(text)
    return paths
