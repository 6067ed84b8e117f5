#!/usr/bin/env python3
"""Benchmark of the hierarchical-tiling median filter on one MI355X.

One step = the whole filter over one 30-megapixel RGB frame: three planar
uint8 planes of 6720 x 4480 (synthetic smooth gradients + 5 % salt-and-pepper,
standing in for the paper's photographs), each filtered with the k x k median
(replicate border). The headline is k = 17, the paper's teaser configuration.

Inputs are resident in HBM before timing starts; four distinct frames are
rotated (720 MB of input + output) so the 256 MB MALL cannot hold the working
set. Every kernel launch is bracketed by HIP events on the stream it runs on;
the roofline object uses their average duration.

Prints ONE JSON line (rank 0, N = 1). --gpus N with N > 1 exits: this build
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s per k (uint8 30MP, k=3..75) + %roofline; batched vs per-image speedup"
PAPER_L40S_MSAMPLE_S_K17 = 6720 * 4480 * 3 / 2.2e-3 / 1e6   # 2.2 ms teaser figure, context only

HBM_PEAK_BPS = 8.0e12            # MI355X HBM3E, bytes/s
VALU_LANES_PER_S = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock = 39.3e12 32-bit lane-ops/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--k", type=int, default=17, help="headline kernel diameter")
    p.add_argument("--sweep-steps", type=int, default=5, help="timed steps per k of the sweep (0 = no sweep)")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle work for the CPU baseline")
    p.add_argument("--only-headline", action="store_true", help="time only the headline k (for profilers)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a plain 256 MiB device copy (counter calibration) and exit")
    return p.parse_args()


def algorithmic_ops_per_pixel(dtype_code: int, k: int):
    """(variant, tile, element-ops per output pixel) for what the library runs.

    Oblivious: live min/max of the generated network per root tile / pixels,
    plus the column sort network (one sort of k-t_h+1 values per image column
    and tile row, i.e. per t_h pixels)."""
    from paper_2507_19926_amd import _lib, netgen as ng
    variant, tw, th = _lib.query_config(dtype_code, k)
    if variant == _lib.MF_VARIANT_OBLIVIOUS:
        P = ng.build_tile_program(k, tw, th)
        net = ng.op_counts(P)["minmax"] / (tw * th)
        srt = ng.op_counts(ng.build_sort_program(k - th + 1))["minmax"] / th
        return variant, (tw, th), net + srt
    return variant, (tw, th), None


def roofline(dtype_code: int, k: int, pixels_per_launch: int, launch_s: float):
    from paper_2507_19926_amd import _lib
    es = {0: 1, 1: 2, 2: 4, 3: 4}[dtype_code]
    bytes_per_launch = 2 * es * pixels_per_launch
    variant, tile, ops_px = algorithmic_ops_per_pixel(dtype_code, k)
    packed = dtype_code in (0, 1)
    valu_peak = VALU_LANES_PER_S * (2 if packed else 1)    # element-ops/s
    t_hbm = bytes_per_launch / HBM_PEAK_BPS
    t_alu = (ops_px * pixels_per_launch / valu_peak) if ops_px else 0.0
    if ops_px is not None and t_alu > t_hbm:
        achieved = ops_px * pixels_per_launch / launch_s
        return {"bound": "alu", "achieved": achieved / 1e12, "peak": valu_peak / 1e12,
                "unit": "Tops/s", "frac": achieved / valu_peak, "traffic": None,
                "ops_per_pixel": round(ops_px, 2), "variant": variant, "tile": list(tile)}
    achieved = bytes_per_launch / launch_s
    return {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK_BPS / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_BPS, "traffic": None,
            "ops_per_pixel": round(ops_px, 2) if ops_px else None, "variant": variant, "tile": list(tile)}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2507_19926_amd import _lib, workloads as wl
    from paper_2507_19926_amd.ops import median_filter

    _lib.lib()  # fail loudly if the HIP library is missing
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        n = 256 << 20
        a = torch.empty(n, dtype=torch.uint8, device=dev).fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 3}))
        return

    H, W = wl.RGB30_H, wl.RGB30_W
    base = wl.rgb30_planes()
    nsets = 4
    ins, outs = [], []
    for s in range(nsets):
        frame = base if s == 0 else np.roll(base, shift=97 * s, axis=2)
        ins.append(torch.from_numpy(np.ascontiguousarray(frame)).to(dev))
        outs.append(torch.empty((3, H, W), dtype=torch.uint8, device=dev))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)

    def run(k, steps, warmup):
        for i in range(warmup):
            s = i % nsets
            median_filter(ins[s], k, out=outs[s])
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(3 * steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            s = i % nsets
            for c in range(3):
                e0, e1 = evs[3 * i + c]
                e0.record(stream)
                median_filter(ins[s][c], k, out=outs[s][c])
                e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launch_ms = [e0.elapsed_time(e1) for (e0, e1) in evs]
        return wall, float(np.mean(launch_ms)) / 1e3

    px_step = 3 * H * W
    # headline
    wall, launch_s = run(args.k, args.steps, args.warmup)
    value = px_step * args.steps / wall / 1e6
    roof = roofline(_lib.MF_U8, args.k, H * W, launch_s)
    per_k = {}
    if args.sweep_steps > 0 and not args.only_headline:
        for k in wl.RGB30_KS:
            try:
                _lib.query_config(_lib.MF_U8, k)
            except _lib.MfError:
                per_k[str(k)] = "unsupported"
                continue
            w, ls = run(k, args.sweep_steps, 2)
            r = roofline(_lib.MF_U8, k, H * W, ls)
            per_k[str(k)] = {"mpix_s": round(px_step * args.sweep_steps / w / 1e6, 1),
                             "kernel_ms": round(ls * 1e3, 4), "bound": r["bound"],
                             "frac": round(r["frac"], 4), "variant": r["variant"], "tile": r["tile"]}
    cpu = None
    if not args.no_cpu:
        import oracle  # CPU baseline only
        nthreads = len(os.sched_getaffinity(0))
        probe = 16
        t = time.perf_counter()
        oracle.median_filter(base[0], args.k, rows=(0, probe), nthreads=nthreads)
        dt = time.perf_counter() - t
        # rows of the frame (plane after plane) that take about cpu_seconds
        rows = int(min(3 * H, max(probe, probe * args.cpu_seconds / max(dt, 1e-6))))
        t = time.perf_counter()
        done = 0
        for c in range(3):
            n = min(H, rows - done)
            if n <= 0:
                break
            oracle.median_filter(base[c], args.k, rows=(0, n), nthreads=nthreads)
            done += n
        dt = time.perf_counter() - t
        cpu = {"value": round(done * W / dt / 1e6, 3), "unit": "Mpixel/s", "cores": nthreads,
               "kind": "oracle",
               "sample": "%d of the %d rows of the 3-plane frame (%d px) at k=%d, %.1f s"
                         % (done, 3 * H, done * W, args.k, dt)}

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": round(value / PAPER_L40S_MSAMPLE_S_K17, 3) if args.k == 17 else None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "30MP RGB uint8, 3 planar 6720x4480 planes, k=%d, replicate border" % args.k,
                   "k": args.k, "H": H, "W": W, "planes": 3, "frames_rotated": nsets},
        "roofline": roof, "cpu_baseline": cpu, "per_k": per_k,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
