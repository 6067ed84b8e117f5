"""Autotuner: pick the variant, root tile and tiles per work-group for every
(value class, k) by timing each compiled configuration on the GPU.

The paper chooses "the most efficient configuration" per kernel size and data
type (Section 4.3); this script does that for this library. It enumerates the
configurations the library was built with (``mf_list_configs``), times each on
a seeded synthetic plane of the class's dtype, and writes a JSON table:

    {"p16": {"<k>": [variant, tile_w, tile_h, group, form, rows], ...},
     "u16": {...}, "u32": {...}, "device": ..., "timings_ms": {...}}

``p16`` is timed on uint8 data and covers uint8 (and uint16 where ``u16``
has no entry): the oblivious networks pack two 16-bit values per VGPR for
both, but the data-aware kernel holds 8-bit data in bytes and 16-bit data in
16-bit elements, so ``u16`` is timed apart; ``u32`` covers uint32/float32.
The build reads ``tuned.json`` next to this file and compiles the choices
into the library's AUTO table.

Usage (on a GPU): python -m paper_2507_19926_amd.autotune [--out PATH] [--ks K ...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "tuned.json")

CLASSES = {"p16": 0, "u16": 1, "u32": 2}   # class -> representative mf_dtype


def _time_config(x, y, k, cfg, reps, stream):
    import torch
    from .ops import median_filter
    variant, tw, th, group, form, rows = cfg
    kw = dict(variant=variant, tile=(tw, th), group=group, form=form, rows=rows, out=y)
    median_filter(x, k, **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        median_filter(x, k, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(shape=(4480, 6720), ks=None, verbose: bool = True) -> dict:
    import numpy as np
    import torch

    from . import _lib, workloads as wl
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ks = ks or list(range(3, 76, 2))
    H, W = shape
    table = {"device": torch.cuda.get_device_properties(0).gcnArchName, "shape": [H, W],
             "timings_ms": {}}
    for cls, code in CLASSES.items():
        dt = {0: np.uint8, 1: np.uint16, 2: np.uint32}[code]
        x = torch.from_numpy(wl.uniform_plane(H, W, dt, seed=77)).to(dev)
        y = torch.empty_like(x)
        best = {}
        for k in ks:
            cfgs = _lib.list_configs(code, k)
            times = {}
            for cfg in cfgs:
                reps = 3 if cfg[0] == _lib.MF_VARIANT_DATA_AWARE and k >= 35 else 8
                times[",".join(map(str, cfg))] = round(_time_config(x, y, k, cfg, reps, stream), 4)
            pick = min(times, key=times.get)
            best[str(k)] = [int(v) for v in pick.split(",")]
            table["timings_ms"]["%s_k%d" % (cls, k)] = times
            if verbose:
                print(cls, k, pick, times[pick], "ms", flush=True)
        table[cls] = best
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TUNED)
    ap.add_argument("--shape", type=int, nargs=2, default=(4480, 6720),
                    help="plane rows and columns to time on (default: one 30 MP plane)")
    ap.add_argument("--ks", type=int, nargs="+", default=None,
                    help="re-time only these k and merge them into the existing table")
    args = ap.parse_args()
    t = tune(shape=tuple(args.shape), ks=args.ks)
    if args.ks and os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
        for cls in CLASSES:
            old.setdefault(cls, {}).update(t[cls])
        old.setdefault("timings_ms", {}).update(t["timings_ms"])
        t = old
    with open(args.out, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
    print("wrote", args.out)


if __name__ == "__main__":
    sys.exit(main())
