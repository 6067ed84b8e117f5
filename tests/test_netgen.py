"""CPU checks of the network generator: comparator networks by the 0-1
principle, tile geometry against the worked dimensions of Section 3.2, and the
whole hierarchical program (run by the numpy model) against the oracle."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_2507_19926_amd import netgen as ng
from paper_2507_19926_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _run(P, inputs):
    """Evaluate a program whose loads are ('in', i) on a batch (B, n) of rows."""
    vals = {}
    for v in ng.live_ops(P):
        op = P.ops[v]
        if op[0] == ng.LD:
            vals[v] = inputs[:, op[1][1]]
        elif op[0] == ng.MIN:
            vals[v] = np.minimum(vals[op[1]], vals[op[2]])
        else:
            vals[v] = np.maximum(vals[op[1]], vals[op[2]])
    return np.stack([vals[o] for o in P.outputs], axis=1)


def _all_01(n):
    return np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.int8)


@pytest.mark.parametrize("n", range(1, 15))
def test_sort_network_zero_one(n):
    # 0-1 principle (Knuth TAOCP 3, 5.3.4): a network sorts every input iff it
    # sorts every 0/1 input.
    P = ng.build_sort_program(n)
    x = _all_01(n)
    np.testing.assert_array_equal(_run(P, x), np.sort(x, axis=1))


def test_merge_network_zero_one():
    for p in range(0, 11):
        for q in range(0, 11):
            P = ng.Prog()
            A = [P.load(("in", i)) for i in range(p)]
            B = [P.load(("in", p + i)) for i in range(q)]
            P.outputs = ng.merge(P, A, B)
            # every pair of sorted 0/1 lists
            rows = []
            for a in range(p + 1):
                for b in range(q + 1):
                    rows.append([0] * (p - a) + [1] * a + [0] * (q - b) + [1] * b)
            x = np.array(rows, dtype=np.int8).reshape(len(rows), p + q)
            if p + q == 0:
                continue
            np.testing.assert_array_equal(_run(P, x), np.sort(x, axis=1), err_msg="%d,%d" % (p, q))


def test_multiway_random():
    g = wl.rng(0)
    for sizes in ([3, 3, 3], [5, 2, 7, 1], [4] * 7, [1] * 9, [6, 6]):
        P = ng.Prog()
        lists, off = [], 0
        for s in sizes:
            lists.append([P.load(("in", off + i)) for i in range(s)])
            off += s
        P.outputs = ng.multiway(P, lists)
        x = g.integers(0, 5, size=(300, off))
        # inputs must be sorted within each list
        o = 0
        for s in sizes:
            x[:, o:o + s] = np.sort(x[:, o:o + s], axis=1)
            o += s
        np.testing.assert_array_equal(_run(P, x), np.sort(x, axis=1))


def test_tile_geometry_worked_example():
    with open(os.path.join(GOLDEN, "tile_geometry.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        parts = ng.tile_parts(case["k"], case["tw"], case["th"])
        assert list(parts.footprint) == case["footprint"]
        assert list(parts.core) == case["core"]
        assert parts.extra_cols_per_side == case["extra_cols_per_side"]
        assert parts.extra_rows_per_side == case["extra_rows_per_side"]
        assert list(parts.corner_block) == case["corner_block"]
    for case in g["splits"]:
        assert [list(s) for s in ng.split_sequence(*case["root"])][:len(case["sequence"])] == case["sequence"]


def test_root_tile_heuristic_bounds():
    # k/4 < t(k) < k/2 for odd k >= 3 (Section 4.2)
    for k in range(3, 200, 2):
        t = ng.root_tile_heuristic(k)
        assert k / 4 < t < k / 2 and (t & (t - 1)) == 0


def test_level_table_keeps_u_plus_one():
    for k in (5, 9, 17, 35, 75):
        t = ng.root_tile_heuristic(k)
        rows = ng.level_table(k, t, t)
        assert rows[-1] == (1, 1, k * k, 0, 1)
        for (_, _, c, u, kept) in rows:
            assert kept <= u + 1 and kept <= c and (c + u) == k * k


CASES = [(1, 1, 1), (3, 1, 1), (3, 2, 1), (3, 2, 2), (5, 2, 2), (5, 4, 2), (5, 1, 4),
         (7, 2, 2), (7, 4, 4), (9, 4, 4), (9, 8, 2), (11, 4, 4), (13, 4, 2), (15, 2, 8)]


@pytest.mark.parametrize("k,tw,th", CASES)
def test_tile_program_matches_oracle(k, tw, th):
    P = ng.build_tile_program(k, tw, th)
    for dtype, shape, seed in ((np.uint8, (23, 37), 1), (np.uint16, (19, 16), 2),
                               (np.uint32, (9, 30), 3)):
        img = wl.uniform_plane(*shape, dtype, seed=seed + k)
        np.testing.assert_array_equal(ng.evaluate_on_image(P, img, k, tw, th),
                                      oracle.median_filter(img, k))
    ties = wl.tie_heavy_plane(21, 26, np.uint8, levels=3, seed=k)
    np.testing.assert_array_equal(ng.evaluate_on_image(P, ties, k, tw, th),
                                  oracle.median_filter(ties, k))


@pytest.mark.parametrize("k,tw,th", [(3, 2, 1), (3, 2, 2), (5, 4, 2), (5, 2, 2), (7, 4, 2)])
def test_inline_column_program_matches_oracle(k, tw, th):
    P = ng.build_tile_program(k, tw, th, inline_cols=True)
    assert all(op[1][0] == "raw" for op in P.ops if op[0] == ng.LD)
    img = wl.uniform_plane(23, 37, np.uint8, seed=k)
    np.testing.assert_array_equal(ng.evaluate_on_image(P, img, k, tw, th), oracle.median_filter(img, k))


@pytest.mark.parametrize("kw,kh,tw,th", [(5, 3, 4, 2), (3, 5, 2, 4), (9, 3, 4, 2), (3, 9, 2, 4), (7, 5, 4, 4),
                                         (5, 9, 4, 4), (15, 5, 4, 4), (5, 15, 4, 4), (3, 1, 2, 1), (1, 3, 1, 2)])
def test_rect_tile_program_matches_oracle(kw, kh, tw, th):
    """The rectangular network (k_w columns, k_h rows: separate radii, the
    sorted columns over k_h-t_h+1 core rows) against the oracle's kw x kh
    median, on random and tie-heavy images."""
    P = ng.build_tile_program(kw, tw, th, kh=kh)
    for dtype, shape, seed in ((np.uint8, (23, 37), 1), (np.uint16, (19, 16), 2), (np.uint32, (9, 30), 3)):
        img = wl.uniform_plane(*shape, dtype, seed=seed + kw * 7 + kh)
        np.testing.assert_array_equal(ng.evaluate_on_image(P, img, kw, tw, th, kh),
                                      oracle.median_filter_rect(img, kw, kh))
    ties = wl.tie_heavy_plane(21, 26, np.uint8, levels=3, seed=kw + kh)
    np.testing.assert_array_equal(ng.evaluate_on_image(P, ties, kw, tw, th, kh),
                                  oracle.median_filter_rect(ties, kw, kh))
    # every load stays inside the rectangular footprint
    for op in P.ops:
        if op[0] == ng.LD:
            kind, a, b = op[1]
            assert 0 <= a < kw + tw - 1
            assert 0 <= b < (kh - th + 1 if kind == "col" else kh + th - 1)


def test_every_compiled_rect_network_matches_oracle():
    """Each rectangular network the library compiles (build.RECT_OBL_CONFIGS),
    run by the CPU model on one ragged image, against the oracle."""
    from paper_2507_19926_amd import build as mfbuild
    for kw, kh, tw, th in (tuple(c[:4]) for c in mfbuild.RECT_OBL_CONFIGS):
        P = ng.build_tile_program(kw, tw, th, kh=kh)
        img = wl.uniform_plane(3 * th + 5, 3 * tw + 7, np.uint16, seed=kw * 97 + kh)
        np.testing.assert_array_equal(ng.evaluate_on_image(P, img, kw, tw, th, kh),
                                      oracle.median_filter_rect(img, kw, kh), err_msg="%dx%d" % (kw, kh))
