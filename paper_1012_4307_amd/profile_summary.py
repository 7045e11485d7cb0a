"""Condense rocprofv3 CSV output into the short text summaries kept with the
measurements, and the per-launch HBM traffic of the fused cycle kernels.

    python -m paper_1012_4307_amd.profile_summary stats  <kernel_trace.csv> <out.txt> --cmd "..."
    python -m paper_1012_4307_amd.profile_summary traffic <fetch counter_collection.csv> \\
        <write counter_collection.csv> <out.txt> <traffic.json> --cmd-fetch "..." --cmd-write "..."

``stats`` tabulates kernel time by kernel and launch grid (the fused kernels
run once per level, so the grid size names the level).  ``traffic`` reads
FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the finest-level fused
kernels (the FP32 up kernel, the FP32 down kernels that form the nested
Bi-CGSTAB's p and s, the FP64 down and up kernels) and of the copy probe,
scales each counter by what it reads for the copy probe of known size (bytes
moved / counter bytes), and records the scaled bytes per launch together with
a digest of those kernels' sources, so a reader can tell when the figures no
longer describe the code.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the sources of the kernels whose counters are recorded: the device helpers
# (ecs_internal.h) and the part of kernels_vcycle.hip that defines the fused
# down and up kernels and their helpers (everything before the tail section;
# the tail kernel and the host launchers follow it)
CSRC = os.path.join(ROOT, "paper_1012_4307_amd", "csrc")
KERNEL_SOURCES = [os.path.join(CSRC, "ecs_internal.h"), os.path.join(CSRC, "kernels_vcycle.hip")]
TAIL_MARKER = b"\n// ----------------------------------------------------------------- tail\n"
COPY_BYTES = 512 << 20   # the copy probe moves 512 MiB each way
# class (as bench.py's timing classes) and kernel name pattern; the finest
# grid of each is the one recorded
# (the single right-hand side instantiations: a trailing ", false" where the
# kernel also has a multi-right-hand-side form)
CLASSES = (("up", r"k_up_rb<float, \d+(, false)?>"), ("down_p", r"k_down_rb<float, \d+, 1(, false)?>"),
           ("down_s", r"k_down_rb<float, \d+, 2(, false)?>"), ("down_f64", r"k_down_rb<double, \d+, 0(, false)?>"),
           ("up_f64", r"k_up_rb<double, \d+(, false)?>"))
# algorithmic bytes per fine node: every input read once, every output written
# once.  FP32 complex 8 B, real 4 B: up reads the coarse correction (a quarter
# node), b, k^2 and writes u (5.5 reals = 22 B); the p-forming down kernel
# reads r, p, v, k^2 and writes p and the coarse residual (9.5 reals = 38 B);
# the s-forming one reads r, v, k^2 and writes s and the coarse residual
# (7.5 reals = 30 B).  FP64: down 3.5 reals = 28 B, up 5.5 reals = 44 B.
ALGO_BYTES_PER_NODE = dict(up=22, down_p=38, down_s=30, down_f64=28, up_f64=44)


def sources_digest() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            text = fh.read()
        if f.endswith("kernels_vcycle.hip"):
            cut = text.find(TAIL_MARKER)
            if cut < 0:
                raise SystemExit("kernels_vcycle.hip: tail section marker not found")
            text = text[:cut]
        h.update(text)
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    nm = name.replace("ecs::(anonymous namespace)::", "").replace("void ", "")
    return re.split(r"[(]", nm)[0]


def trace_class_avg(events, cls: str):
    """Average duration (the trace's unit) of the finest-grid launches of the
    timing class `cls` among chrome-trace events (a kernel event: ph "X",
    cat "kernel", args.grid in workgroups), or None when the class has no
    pattern here or no launch of it is among the events."""
    pats = dict(CLASSES)
    if cls not in pats:
        return None
    agg = collections.defaultdict(list)
    for e in events:
        if e.get("ph") != "X" or e.get("cat") != "kernel":
            continue
        if not re.fullmatch(pats[cls], short_name(e.get("name", ""))):
            continue
        g = e.get("args", {}).get("grid", [0, 0, 0])
        agg[int(g[0]) * int(g[1]) * int(g[2])].append(float(e["dur"]))
    if not agg:
        return None
    durs = agg[max(agg)]
    return sum(durs) / len(durs)


def stats(trace_csv: str, out_txt: str, cmd: str, top: int = 40) -> None:
    agg = collections.defaultdict(list)
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            key = (short_name(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) *
                   int(r["Grid_Size_Z"]))
            agg[key].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in agg.values())
    lines = [f"command: {cmd}", f"source: {os.path.basename(trace_csv)}",
             f"total kernel time {total / 1e6:.1f} ms over {sum(len(v) for v in agg.values())} dispatches",
             "", f"{'kernel':48s} {'grid threads':>12s} {'calls':>7s} {'avg us':>9s} {'median us':>9s} "
                 f"{'total ms':>9s} {'%':>6s}"]
    for (name, grid), v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"{name[:48]:48s} {grid:12d} {len(v):7d} {sum(v) / len(v) / 1e3:9.2f} "
                     f"{statistics.median(v) / 1e3:9.2f} {sum(v) / 1e6:9.2f} {100 * sum(v) / total:6.2f}")
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter(path: str, counter: str):
    """{(kernel, grid): [KiB per dispatch]} for one counter."""
    out = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            out[(short_name(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return out


def _finest(d, pattern: str):
    keys = [k for k in d if re.fullmatch(pattern, k[0])]
    if not keys:
        raise SystemExit(f"no dispatch of {pattern}")
    k = max(keys, key=lambda k: k[1])
    return k, statistics.median(d[k])


def traffic(fetch_csv: str, write_csv: str, out_txt: str, out_json: str, cmd_fetch: str, cmd_write: str,
            algo: dict) -> None:
    fe = _counter(fetch_csv, "FETCH_SIZE")
    wr = _counter(write_csv, "WRITE_SIZE")
    (_, _), copy_fetch = _finest(fe, r"k_copy16")
    (_, _), copy_write = _finest(wr, r"k_copy16")
    fetch_scale = COPY_BYTES / (copy_fetch * 1024)
    write_scale = COPY_BYTES / (copy_write * 1024)
    kernels = {}
    lines = [f"command (FETCH_SIZE): {cmd_fetch}", f"command (WRITE_SIZE): {cmd_write}", "",
             f"copy probe ({COPY_BYTES} B read + written): FETCH_SIZE {copy_fetch:.1f} KiB -> scale "
             f"{fetch_scale:.4f}; WRITE_SIZE {copy_write:.1f} KiB -> scale {write_scale:.4f}", "",
             f"{'class':8s} {'kernel':26s} {'grid':>8s} {'FETCH KiB':>11s} {'WRITE KiB':>11s} {'HBM bytes':>12s} "
             f"{'algorithmic':>12s} {'ratio':>6s}"]
    for cls, pat in CLASSES:
        (name, grid), f_kib = _finest(fe, pat)
        w_kib = statistics.median(wr[(name, grid)])
        hbm = f_kib * 1024 * fetch_scale + w_kib * 1024 * write_scale
        kernels[cls] = dict(kernel=name, grid_threads=grid, fetch_kib=f_kib, write_kib=w_kib,
                            hbm_bytes_per_launch=round(hbm), algorithmic_bytes_per_launch=algo[cls])
        lines.append(f"{cls:8s} {name:26s} {grid:8d} {f_kib:11.1f} {w_kib:11.1f} {hbm:12.0f} {algo[cls]:12d} "
                     f"{hbm / algo[cls]:6.3f}")
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(out_json, "w") as f:
        json.dump(dict(sources_digest=sources_digest(), fetch_scale=fetch_scale, write_scale=write_scale,
                       kernels=kernels, commands=dict(fetch=cmd_fetch, write=cmd_write)), f, indent=1)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("trace")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("out")
    t.add_argument("json")
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--n", type=int, default=2049)
    a = ap.parse_args()
    if a.what == "stats":
        stats(a.trace, a.out, a.cmd)
    else:
        nodes = a.n * a.n
        traffic(a.fetch, a.write, a.out, a.json, a.cmd_fetch, a.cmd_write,
                algo={c: nodes * b for c, b in ALGO_BYTES_PER_NODE.items()})


if __name__ == "__main__":
    main()
