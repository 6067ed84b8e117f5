"""Build the HIP library ``libmedfilt.so`` for gfx950, in-tree.

Steps: generate the oblivious network translation units (emit_hip), compile
every HIP/C++ source with hipcc (in parallel), link one shared library next to
this file. The library is what the Python binding loads; nothing is built at
import time.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

from . import emit_da, emit_hip

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
GEN = os.path.join(BUILD, "gen")
LIB = os.path.join(PKG, "libmedfilt.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Oblivious configurations compiled into the library: (k, t_w, t_h, tile rows
# per wave, waves per work-group[, inline column sort]). The first entry for
# each k is the default; the others can be requested through mf_options (and
# are what the tuner compares).
OBL_CONFIGS = [
    (3, 2, 1, 8, 4), (3, 2, 1, 8, 1), (3, 1, 1, 8, 4), (3, 2, 2, 4, 4),
    (3, 2, 1, 8, 4, True), (3, 2, 2, 4, 4, True), (3, 2, 2, 8, 1, True),
    (3, 2, 1, 2, 4), (3, 2, 2, 1, 4), (3, 2, 1, 2, 4, True), (3, 2, 2, 1, 4, True),
    (5, 4, 2, 2, 4), (5, 4, 2, 4, 1), (5, 2, 2, 2, 4),
    (5, 4, 2, 2, 4, True), (5, 2, 2, 4, 4, True), (5, 4, 2, 1, 4), (5, 2, 2, 1, 4, True),
    (7, 4, 2, 2, 4), (7, 4, 2, 4, 1), (7, 2, 2, 2, 4), (7, 4, 2, 1, 4),
    (9, 4, 4, 1, 4), (9, 4, 4, 2, 1), (9, 8, 2, 1, 4),
    (11, 4, 4, 1, 4), (11, 4, 4, 2, 1), (11, 4, 2, 2, 4),
    (13, 4, 4, 1, 4), (13, 4, 4, 1, 1),
    (15, 4, 4, 1, 4), (15, 4, 4, 1, 1),
    (17, 4, 4, 1, 4), (17, 4, 4, 1, 1),
    (19, 4, 4, 1, 4),
    (21, 4, 4, 1, 4),
]

# Oblivious networks for rectangular windows: (k_w, k_h, t_w, t_h, tile rows
# per wave, waves per work-group); other k_w x k_h windows run data-aware.
RECT_OBL_CONFIGS = [
    (3, 1, 2, 1, 8, 4), (1, 3, 1, 2, 4, 4),
    (5, 3, 4, 2, 2, 4), (3, 5, 2, 4, 1, 4), (7, 3, 4, 2, 2, 4), (3, 7, 2, 4, 1, 4),
    (9, 3, 4, 2, 2, 4), (3, 9, 2, 4, 1, 4),
    (7, 5, 4, 4, 1, 4), (5, 7, 4, 4, 1, 4), (9, 5, 4, 4, 1, 4), (5, 9, 4, 4, 1, 4),
    (9, 7, 4, 4, 1, 4), (7, 9, 4, 4, 1, 4), (15, 5, 4, 4, 1, 4), (5, 15, 4, 4, 1, 4),
    # larger shapes: the root tile with the fewest min/max per pixel among
    # those whose network's live values stay near the register file (wide
    # windows take wide tiles, tall windows tall ones)
    (5, 1, 4, 1, 4, 4), (1, 5, 1, 4, 1, 4), (9, 1, 8, 1, 1, 4), (1, 9, 1, 8, 1, 4),
    (11, 3, 8, 1, 1, 4), (3, 11, 1, 8, 1, 4), (31, 3, 8, 1, 1, 4), (3, 31, 1, 8, 1, 4),
    (11, 5, 8, 1, 1, 4), (5, 11, 4, 4, 1, 4), (13, 5, 8, 1, 1, 4), (5, 13, 4, 4, 1, 4),
    (17, 5, 8, 1, 1, 4), (5, 17, 4, 4, 1, 4), (11, 7, 8, 2, 1, 4), (7, 11, 4, 4, 1, 4),
    (21, 7, 8, 1, 1, 4), (7, 21, 2, 8, 1, 4), (13, 9, 8, 2, 1, 4), (9, 13, 4, 4, 1, 4),
    (17, 9, 8, 2, 1, 4), (9, 17, 4, 4, 1, 4),
    (31, 5, 8, 1, 1, 4), (5, 31, 1, 8, 1, 4), (31, 7, 8, 1, 1, 4), (7, 31, 2, 8, 1, 4),
    (21, 9, 8, 2, 1, 4), (9, 21, 2, 8, 1, 4), (31, 9, 8, 2, 1, 4), (9, 31, 2, 8, 1, 4),
    # the remaining shapes with sides 3..17, same rule (4x4 where a wider or
    # taller tile's persistent kernel would not fit the LDS)
    (3, 13, 1, 8, 1, 4), (3, 15, 1, 8, 1, 4), (3, 17, 1, 8, 1, 4), (7, 13, 4, 4, 1, 4),
    (7, 15, 4, 4, 1, 4), (7, 17, 4, 4, 1, 4), (9, 11, 4, 4, 1, 4), (9, 15, 4, 4, 1, 4),
    (11, 9, 8, 2, 1, 4), (11, 13, 4, 4, 1, 4), (11, 15, 4, 4, 1, 4), (11, 17, 4, 4, 1, 4),
    (13, 3, 8, 1, 1, 4), (13, 7, 8, 2, 1, 4), (13, 11, 4, 4, 1, 4), (13, 15, 4, 4, 1, 4),
    (13, 17, 4, 4, 1, 4), (15, 3, 8, 1, 1, 4), (15, 7, 8, 2, 1, 4), (15, 9, 8, 2, 1, 4),
    (15, 11, 4, 4, 1, 4), (15, 13, 4, 4, 1, 4), (15, 17, 4, 4, 1, 4), (17, 3, 8, 1, 1, 4),
    (17, 7, 8, 2, 1, 4), (17, 11, 4, 4, 1, 4), (17, 13, 4, 4, 1, 4), (17, 15, 4, 4, 1, 4),
    # one-dimensional windows (running medians along rows or columns)
    (7, 1, 4, 1, 4, 4), (1, 7, 1, 4, 1, 4),
] + [c for n in range(11, 32, 2) for c in ((n, 1, 8, 1, 1, 4), (1, n, 1, 8, 1, 4))]

HIP_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=%s" % ARCH, "-fPIC",
    # no packed-fp32 instructions anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _up_to_date(obj: str) -> bool:
    """True when obj and its dependency file exist and no dependency is newer."""
    dep = obj + ".d"
    if not (os.path.exists(obj) and os.path.exists(dep)):
        return False
    t = os.path.getmtime(obj)
    with open(dep) as f:
        text = f.read().replace("\\\n", " ")
    files = text.split(":", 1)[1].split() if ":" in text else []
    return all(os.path.exists(d) and os.path.getmtime(d) <= t for d in files)


def _compile(src: str, obj: str, extra=(), incremental: bool = False) -> tuple[str, str]:
    if incremental and _up_to_date(obj):
        return obj, ""
    cmd = [HIPCC] + HIP_FLAGS + list(extra) + [
        "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", GEN,
        "-MD", "-MF", obj + ".d", "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), p.stderr[-6000:]))
    return obj, p.stderr


def _write_auto_table() -> None:
    """AUTO choices per (value class, k) from tuned.json (autotune.py), as
    MF_AUTO(class, k, variant, tile_w, tile_h, group, form, rows) lines; class 0 = 8-bit
    (and 16-bit where class 2 has no entry), 1 = 32-bit, 2 = 16-bit. Without
    tuned.json the table is empty and the library falls back to its built-in
    order (oblivious first)."""
    import json
    lines = ["// Generated from tuned.json: measured fastest configuration per (class, k)."]
    path = os.path.join(PKG, "tuned.json")
    if os.path.exists(path):
        with open(path) as f:
            t = json.load(f)
        for cls, code in (("p16", 0), ("u32", 1), ("u16", 2)):
            for k, cfg in sorted(t.get(cls, {}).items(), key=lambda kv: int(kv[0])):
                variant, tw, th, group = cfg[:4]
                form = cfg[4] if len(cfg) > 4 else 0
                rows = cfg[5] if len(cfg) > 5 else 0
                lines.append("MF_AUTO(%d, %d, %d, %d, %d, %d, %d, %d)"
                             % (code, int(k), variant, tw, th, group, form, rows))
    text = "\n".join(lines) + "\n"
    out = os.path.join(GEN, "mf_auto_table.inc")
    if not os.path.exists(out) or open(out).read() != text:
        with open(out, "w") as f:
            f.write(text)


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Generate, compile and link. Returns the path of libmedfilt.so. With
    incremental=True, objects whose sources and headers are unchanged since
    they were compiled are reused."""
    os.makedirs(GEN, exist_ok=True)
    obl_srcs = emit_hip.generate(GEN, OBL_CONFIGS, RECT_OBL_CONFIGS)
    _write_auto_table()
    emit_da.generate(GEN)
    blob_cpp = os.path.join(GEN, "mf_da_blob.cpp")
    text = ("// Generated: host image of the data-aware schedules (copied to each device once).\n"
            "__asm__(\".section .rodata\\n.balign 16\\n.global mf_da_blob_host\\n"
            "mf_da_blob_host:\\n.incbin \\\"%s\\\"\\n.previous\\n\");\n"
            % os.path.join(GEN, "mf_da_blob.bin"))
    if not os.path.exists(blob_cpp) or open(blob_cpp).read() != text:
        with open(blob_cpp, "w") as f:
            f.write(text)
    srcs = [os.path.join(CSRC, "mf_api.cpp"), os.path.join(CSRC, "mf_plan.cpp"), os.path.join(CSRC, "mf_data_aware.hip"),
            os.path.join(CSRC, "mf_autograd.hip"), os.path.join(CSRC, "mf_strip.hip"), os.path.join(CSRC, "mf_peaks.hip"),
            os.path.join(CSRC, "mf_noalloc.hip"), blob_cpp] + obl_srcs
    objs = []
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = []
        for s in srcs:
            obj = os.path.join(BUILD, os.path.basename(s) + ".o")
            objs.append(obj)
            extra = ["-x", "hip"] if s.endswith(".hip") else []
            # the schedule blob is pulled in by .incbin, which the dependency
            # file does not list: always rebuilt
            futs.append(ex.submit(_compile, s, obj, extra, incremental and s != blob_cpp))
        for f in futs:
            _, err = f.result()
            if verbose and err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=%s" % ARCH, "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n%s" % p.stderr[-4000:])
    os.replace(tmp, LIB)
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)
    if os.path.exists(LIB):
        os.remove(LIB)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
