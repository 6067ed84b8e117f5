#!/usr/bin/env python3
"""Benchmark of the hierarchical-tiling median filter on one MI355X.

One step = the whole filter over one 30-megapixel RGB frame: three planar
uint8 planes of 6720 x 4480 (synthetic smooth gradients + 5 % salt-and-pepper,
standing in for the paper's photographs), each filtered with the k x k median
(replicate border). The headline is k = 17, the paper's teaser configuration.

Inputs are resident in HBM before timing starts; eight distinct frames are
rotated (1.4 GB of input + output) so the 256 MB MALL cannot hold the working
set. One step is one launch (the frame's three planes through
median_filter_planes), bracketed by HIP events on the stream it runs on; the
roofline object uses their average duration.

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
LDS_PEAK_BPS = 256 * 128 * 2.4e9  # 128 B/clock/CU of LDS bandwidth x 256 CUs x 2.4 GHz = 78.6 TB/s
VALU_LANES_PER_S = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock = 39.3e12 32-bit lane-ops/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--k", type=int, default=17, help="headline kernel diameter")
    p.add_argument("--window", default=None,
                   help="KWxKH: time this rectangular window (kw columns, kh rows) in place of k "
                        "(for profiling one data-aware schedule)")
    p.add_argument("--sweep-steps", type=int, default=50,
                   help="timed launches per k of the sweeps, median reported (0 = no sweep)")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle work for the CPU baseline")
    p.add_argument("--only-headline", action="store_true", help="time only the headline k (for profilers)")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the dtype sweep, the batched comparison and the autograd timing")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a plain 256 MiB device copy (counter calibration) and exit")
    return p.parse_args()


def algorithmic_ops_per_pixel(dtype_code: int, k: int, kh: int | None = None):
    """(variant, tile, element-ops per output pixel, packed) for what the
    library runs (k x k window, or k columns by kh rows). `packed` tells
    whether two element-ops share one 32-bit lane-op (packed 16-bit min/max).

    Oblivious: live min/max of the generated network per root tile / pixels,
    plus the column sort network (one sort of k-t_h+1 values per image column
    and tile row, i.e. per t_h pixels). Column-strip form (k = 3): 3 ops to
    sort the three values of a column (v_min3, v_med3, v_max3), one sorted
    column per pixel, plus 4 ops for the pruned merge of three sorted columns
    (max of minima, median of medians, min of maxima, median of the three);
    these are 32-bit lane-ops, one element each.

    Data-aware: two lane-ops per merge output (the compare that picks the
    smaller head and the min that produces it) plus two per compare-exchange
    of the per-lane sorting networks (min and max), from the schedule; the
    kernel computes on unpacked 32-bit lanes."""
    from paper_2507_19926_amd import _lib, dagen, netgen as ng
    if kh is not None and kh != k:
        variant, tw, th = _lib.query_rect_config(dtype_code, k, kh)
        form = 0
    else:
        kh = k
        variant, tw, th, _, form, _ = _lib.query_options(dtype_code, k)
    packed = dtype_code in (_lib.MF_U8, _lib.MF_U16)
    if variant == _lib.MF_VARIANT_OBLIVIOUS:
        if form == 3:
            return variant, (tw, th), 3.0 + 4.0, False
        P = ng.build_tile_program(k, tw, th, kh=kh)
        net = ng.op_counts(P)["minmax"] / (tw * th)
        srt = ng.op_counts(ng.build_sort_program(kh - th + 1))["minmax"] / th
        return variant, (tw, th), net + srt, packed
    st = dagen.schedule(k, tw, th, kh=kh).stats
    return variant, (tw, th), 2.0 * (st["per_pixel_outputs"] + st["per_pixel_sort_ces"]), False


def measured_traffic(k: int, tile):
    """HBM bytes per launch from the committed counter measurement of this
    kernel (profiles/traffic_*.json), or None when there is none or the
    kernel's sources changed since it was taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        with open(path) as f:
            t = json.load(f)
        if "k=%d" % k not in t.get("workload", "") or "%dx%d" % tuple(tile) not in t.get("kernel", ""):
            continue
        h = hashlib.sha256()
        try:
            for src in t["source_files"]:
                with open(os.path.join(ROOT, src), "rb") as f:
                    h.update(f.read())
        except OSError:
            return None
        if h.hexdigest()[:16] == t["source_sha256_16"]:
            return t["traffic_bytes_per_launch"]
    return None


def roofline(dtype_code: int, k: int, pixels_per_launch: int, launch_s: float, kh: int | None = None):
    from paper_2507_19926_amd import _lib
    es = {0: 1, 1: 2, 2: 4, 3: 4}[dtype_code]
    bytes_per_launch = 2 * es * pixels_per_launch
    variant, tile, ops_px, packed = algorithmic_ops_per_pixel(dtype_code, k, kh)
    valu_peak = VALU_LANES_PER_S * (2 if packed else 1)    # element-ops/s
    t_hbm = bytes_per_launch / HBM_PEAK_BPS
    t_alu = (ops_px * pixels_per_launch / valu_peak) if ops_px else 0.0
    if ops_px is not None and t_alu > t_hbm:
        achieved = ops_px * pixels_per_launch / launch_s
        r = {"bound": "alu", "achieved": achieved / 1e12, "peak": valu_peak / 1e12,
             "unit": "Tops/s", "frac": achieved / valu_peak, "traffic": None,
             "ops_per_pixel": round(ops_px, 2), "variant": variant, "tile": list(tile)}
        if variant == _lib.MF_VARIANT_DATA_AWARE:
            # LDS view of the same launch: each merge output is one element
            # read and one written (2 bytes for 8/16-bit data, 4 for 32-bit)
            from paper_2507_19926_amd import dagen
            st = dagen.schedule(k, tile[0], tile[1], kh=kh).stats
            lds_es = 2 if dtype_code in (0, 1) else 4
            r["merge_outputs_per_pixel"] = round(st["per_pixel_outputs"], 2)
            r["sort_ces_per_pixel"] = round(st["per_pixel_sort_ces"], 2)
            r["lds_frac"] = round(st["per_pixel_outputs"] * pixels_per_launch * 2 * lds_es / launch_s
                                  / LDS_PEAK_BPS, 4)
        return r
    achieved = bytes_per_launch / launch_s
    return {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK_BPS / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_BPS, "traffic": None,
            "ops_per_pixel": round(ops_px, 2) if ops_px else None, "variant": variant, "tile": list(tile)}


def _time(fn, steps, warmup, stream):
    """Median over `steps` launches of the HIP-event time of one call of fn
    (events recorded on `stream`, the stream fn launches on), in seconds."""
    import numpy as np
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs])) / 1e3


def measured_peaks(dev, stream):
    """Measured ceilings beside the public figures: device-to-device copy
    bandwidth (bytes read + written) and the packed 16-bit min/max rate of
    dependent instruction chains (mf_peak_minmax)."""
    import ctypes
    import torch

    from paper_2507_19926_amd import _lib
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device=dev).fill_(3)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_bps = 2 * n * reps / (e0.elapsed_time(e1) / 1e3)
    del a, b
    blocks, iters = 8192, 128
    out = torch.empty(blocks * 256, dtype=torch.int32, device=dev)
    L = _lib.lib()
    h = ctypes.c_void_p(stream.cuda_stream)
    _lib.check(L.mf_peak_minmax(out.data_ptr(), blocks, iters, h))
    e0.record(stream)
    _lib.check(L.mf_peak_minmax(out.data_ptr(), blocks, iters, h))
    e1.record(stream)
    torch.cuda.synchronize()
    ops = blocks * 256 * iters * 512
    return {"copy_TBps": round(copy_bps / 1e12, 3), "copy_frac_of_8TBps": round(copy_bps / HBM_PEAK_BPS, 3),
            "pk_minmax_Tops": round(ops / (e0.elapsed_time(e1) / 1e3) / 1e12, 2),
            "pk_minmax_frac_of_peak": round(ops / (e0.elapsed_time(e1) / 1e3) / (2 * VALU_LANES_PER_S), 3)}


def run_extras(args, dev, stream):
    """dtype sweep (4096^2 planes), batched plan vs per-image launches, the
    global-memory multi-pass form on the 30 MP frame, and the differentiable
    form's forward/backward on 32x3x512x512 float32."""
    import numpy as np
    import torch

    from paper_2507_19926_amd import _lib, workloads as wl
    from paper_2507_19926_amd.ops import (BatchedPlan, median_filter, median_filter_argmedian,
                                          median_filter_backward)
    out = {}
    # dtype sweep: at least 8 distinct input/output pairs per dtype, more than
    # 512 MB in all (the 256 MB MALL cannot hold them), rotated per launch;
    # median over the sweep steps
    sweep = {}
    side = wl.SWEEP_SIDE
    for name, dt, code in (("u16", np.uint16, _lib.MF_U16), ("u32", np.uint32, _lib.MF_U32),
                           ("f32", np.float32, _lib.MF_F32)):
        base = wl.sweep_plane(dt)
        pair_bytes = 2 * base.nbytes
        nsets = max(8, -(-(512 << 20) // pair_bytes) + 1)
        xs = [torch.from_numpy(np.ascontiguousarray(np.roll(base, 131 * s, axis=1))).to(dev) for s in range(nsets)]
        ys = [torch.empty_like(x) for x in xs]
        res = {}
        for k in wl.SWEEP_KS:
            state = {"i": 0}

            def one():
                i = state["i"] = state["i"] + 1
                median_filter(xs[i % nsets], k, out=ys[i % nsets])
            t = _time(one, args.sweep_steps, 2, stream)
            r = roofline(code, k, side * side, t)
            res[str(k)] = {"mpix_s": round(side * side / t / 1e6, 1), "kernel_ms_median": round(t * 1e3, 4),
                           "bound": r["bound"], "frac": round(r["frac"], 4), "variant": r["variant"],
                           "tile": r["tile"]}
        res["buffer_sets"] = nsets
        res["working_set_MB"] = round(nsets * pair_bytes / 1e6, 1)
        sweep[name] = res
        del xs, ys
    out["dtype_sweep_4096"] = sweep

    # batched: 256 mixed images, one plan launch vs 256 plain launches
    batch = wl.mixed_batch()
    xs = [torch.from_numpy(a).to(dev) for a, _ in batch]
    ks = [k for _, k in batch]
    outs = [torch.empty_like(x) for x in xs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = BatchedPlan(xs, outs, ks)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0

    def per_image():
        for x, k, o in zip(xs, ks, outs):
            median_filter(x, k, out=o)
    t_plain = _time(per_image, 20, 2, stream)
    t_plan = _time(plan.launch, 20, 2, stream)
    npx = sum(int(x.numel()) for x in xs)
    nb, blocks = plan.info()
    out["batched"] = {"images": len(xs), "pixels": npx, "plan_ms": round(t_plan * 1e3, 3),
                      "per_image_ms": round(t_plain * 1e3, 3), "speedup": round(t_plain / t_plan, 3),
                      "plan_mpix_s": round(npx / t_plan / 1e6, 1), "plan_create_ms": round(t_create * 1e3, 1),
                      "buckets": nb}
    plan.close()
    del xs, outs

    # global-memory multi-pass form: the 30 MP frame's three planes at k = 75
    # (and k = 25) with a 1 GiB workspace, run in slices of tiles
    from paper_2507_19926_amd.ops import median_filter_global
    frame = torch.from_numpy(np.ascontiguousarray(wl.rgb30_planes())).to(dev)
    fo = torch.empty_like(frame)
    gl = {}
    for k in (25, 75):
        slot, allb, tw, th, passes = _lib.global_workspace(_lib.MF_U8, k, 3, frame.shape[1], frame.shape[2])
        budget = 1 << 30
        median_filter_global(frame, k, out=fo, budget_bytes=budget)
        t = _time(lambda: median_filter_global(frame, k, out=fo, budget_bytes=budget), 5, 0, stream)
        slice_tiles = min(budget // slot, allb // slot)
        gl[str(k)] = {"frame_ms_median": round(t * 1e3, 3), "mpix_s": round(frame.numel() / t / 1e6, 1),
                      "tile": [tw, th], "passes": passes, "slot_bytes": slot, "workspace_bytes": min(budget, allb),
                      "slices": -(-(allb // slot) // slice_tiles), "all_tiles_bytes": allb}
    out["global_multipass_rgb30"] = gl
    del frame, fo

    # 3-D boxes: a 256^3 uint8 volume (uniform values), k x k x k
    from paper_2507_19926_amd.ops import median_filter_3d
    vol = torch.from_numpy(wl.volume_u8(256)).to(dev)
    vo = torch.empty_like(vol)
    b3 = {}
    for k in (3, 5, 7, 9):
        t = _time(lambda: median_filter_3d(vol, k, out=vo), 5, 1, stream)
        b3[str(k)] = {"volume_ms_median": round(t * 1e3, 3), "mvoxel_s": round(vol.numel() / t / 1e6, 1)}
    out["box3d_256cubed_u8"] = b3
    del vol, vo

    # differentiable form
    x = torch.from_numpy(wl.autograd_tensor()).to(dev)
    g = torch.from_numpy(wl.grad_out_like(tuple(x.shape))).to(dev)
    ag = {}
    for k in (7, 15):
        holder = {}

        def fwd():
            holder["idx"] = median_filter_argmedian(x, k)[1]
        t_f = _time(fwd, 20, 1, stream)
        idx = holder["idx"]
        t_b = _time(lambda: median_filter_backward(g, idx, k), 20, 1, stream)
        n = x.numel()
        ag[str(k)] = {"fwd_ms": round(t_f * 1e3, 3), "bwd_ms": round(t_b * 1e3, 3),
                      "fwd_mpix_s": round(n / t_f / 1e6, 1), "bwd_mpix_s": round(n / t_b / 1e6, 1),
                      "bwd_hbm_frac": round(12 * n / t_b / HBM_PEAK_BPS, 4)}
    out["autograd_32x3x512x512"] = ag
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2507_19926_amd import _lib, workloads as wl
    from paper_2507_19926_amd.ops import median_filter, median_filter_rect

    _lib.lib()  # fail loudly if the HIP library is missing
    kw = kh = args.k
    if args.window:
        kw, kh = (int(v) for v in args.window.lower().split("x"))
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
    nsets = 8
    ins, outs = [], []
    for s in range(nsets):
        frame = base if s == 0 else np.roll(base, shift=97 * s, axis=2)
        ins.append(torch.from_numpy(np.ascontiguousarray(frame)).to(dev))
        outs.append(torch.empty((3, H, W), dtype=torch.uint8, device=dev))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)

    def filt(s, k, rows=None):
        if rows is None or rows == k:
            median_filter(ins[s], k, out=outs[s])
        else:
            median_filter_rect(ins[s], k, rows, out=outs[s])

    def run(k, steps, warmup, rows=None):
        for i in range(warmup):
            filt(i % nsets, k, rows)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            s = i % nsets
            e0, e1 = evs[i]
            e0.record(stream)
            filt(s, k, rows)     # the 3 planes in one launch
            e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launch_ms = [e0.elapsed_time(e1) for (e0, e1) in evs]
        return wall, float(np.mean(launch_ms)) / 1e3, float(np.median(launch_ms)) / 1e3

    px_step = 3 * H * W
    # headline
    wall, launch_s, launch_med_s = run(kw, args.steps, args.warmup, kh)
    value = px_step * args.steps / wall / 1e6
    roof = roofline(_lib.MF_U8, kw, px_step, launch_s, kh)
    square = kw == kh
    roof["traffic"] = (measured_traffic(kw, roof["tile"])
                       if square and roof["variant"] == _lib.MF_VARIANT_OBLIVIOUS else None)
    roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    roof["algorithmic_bytes_per_launch"] = 2 * px_step
    roof["launch"] = "one launch per step: the frame's 3 planes (%s)" % ("median_filter_planes" if square else "median_filter_rect")
    roof["launch_ms_mean"] = round(launch_s * 1e3, 4)
    roof["launch_ms_median"] = round(launch_med_s * 1e3, 4)
    per_k = {}
    if args.sweep_steps > 0 and not args.only_headline:
        for k in wl.RGB30_KS:
            try:
                _lib.query_config(_lib.MF_U8, k)
            except _lib.MfError:
                per_k[str(k)] = "unsupported"
                continue
            w, _, ls = run(k, args.sweep_steps, 2)
            r = roofline(_lib.MF_U8, k, px_step, ls)
            per_k[str(k)] = {"mpix_s": round(px_step / ls / 1e6, 1),
                             "frame_ms_median": round(ls * 1e3, 4), "bound": r["bound"],
                             "frac": round(r["frac"], 4), "variant": r["variant"], "tile": r["tile"],
                             "ops_per_pixel": r.get("ops_per_pixel"), "merge_outputs_per_pixel": r.get("merge_outputs_per_pixel")}
    rect = {}
    if args.sweep_steps > 0 and not args.only_headline:
        for rkw, rkh in wl.RGB30_RECT:
            _, _, ls = run(rkw, args.sweep_steps, 2, rkh)
            r = roofline(_lib.MF_U8, rkw, px_step, ls, rkh)
            rect["%dx%d" % (rkw, rkh)] = {"mpix_s": round(px_step / ls / 1e6, 1),
                                          "frame_ms_median": round(ls * 1e3, 4),
                                          "bound": r["bound"], "frac": round(r["frac"], 4),
                                          "variant": r["variant"], "tile": r["tile"],
                                          "ops_per_pixel": r.get("ops_per_pixel"), "merge_outputs_per_pixel": r.get("merge_outputs_per_pixel")}
    extras = {}
    if not args.no_extras and not args.only_headline:
        extras = run_extras(args, dev, stream)
        extras["measured_peaks"] = mp = measured_peaks(dev, stream)
        if roof["bound"] == "alu" and roof["unit"] == "Tops/s" and roof["peak"] > 70:
            roof["frac_of_measured_minmax_rate"] = round(roof["achieved"] / mp["pk_minmax_Tops"], 4)

    cpu = None
    if not args.no_cpu:
        import oracle  # CPU baseline only
        nthreads = len(os.sched_getaffinity(0))
        probe = 256       # long enough that the rate it gives holds for the whole sample
        oracle.median_filter_rect(base[0], kw, kh, rows=(0, 32), nthreads=nthreads)   # warm-up (threads, caches)
        t = time.perf_counter()
        oracle.median_filter_rect(base[0], kw, kh, rows=(0, probe), nthreads=nthreads)
        dt = time.perf_counter() - t
        # rows of the frame (plane after plane, whole frames repeated if one
        # frame is shorter than that) that take about cpu_seconds
        rows = int(min(8 * 3 * H, max(probe, probe * args.cpu_seconds / max(dt, 1e-6))))
        t = time.perf_counter()
        done = 0
        while done < rows:
            c = (done // H) % 3
            n = min(H - done % H, rows - done)
            oracle.median_filter_rect(base[c], kw, kh, rows=(done % H, done % H + n), nthreads=nthreads)
            done += n
        dt = time.perf_counter() - t
        cpu = {"value": round(done * W / dt / 1e6, 3), "unit": "Mpixel/s", "cores": nthreads,
               "kind": "oracle",
               "sample": "%d rows of 6720 px (%.2f passes over the 3-plane frame, %d px) at %s, %.1f s"
                         % (done, done / (3 * H), done * W,
                            "k=%d" % kw if square else "window %dx%d" % (kw, kh), dt)}

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": round(value / PAPER_L40S_MSAMPLE_S_K17, 3) if square and kw == 17 else None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "30MP RGB uint8, 3 planar 6720x4480 planes, %s, replicate border"
                               % ("k=%d" % kw if square else "window %dx%d (kw x kh)" % (kw, kh)),
                   "k": kw, "kh": kh, "H": H, "W": W, "planes": 3, "frames_rotated": nsets},
        "roofline": roof, "cpu_baseline": cpu, "per_k": per_k, "rect_kw_x_kh": rect, **extras,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
