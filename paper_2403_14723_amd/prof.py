"""Reduces rocprofv3 output of `bench.py` runs to a short markdown summary.

Usage (after the profiling runs on a GPU host):
    python -m paper_2403_14723_amd.prof --stats <dir of the --kernel-trace --stats run>
        --fetch <dir of the --pmc FETCH_SIZE run> --write <dir of the --pmc WRITE_SIZE run>
        --pmc <dir> [--pmc <dir> ...] --command "<the rocprofv3 commands>" --out <file.md>

Counter scale: rocprofv3 reports FETCH_SIZE and WRITE_SIZE in KiB per dispatch,
and on this device FETCH_SIZE counts half of the bytes a plain copy kernel
reads.  Both are calibrated on the largest copy kernel of the profiled run,
which moves 12*T bytes (the size of the triangle array and of each of next'
and prev'), and the calibrated bytes per launch of every kernel of the
meshing chain (and their rocprofv3 average durations) are written into the
summary with a hash of the kernel sources, so bench.py can tell whether the
counters still describe the kernels it runs.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/mesh_kernels.hip", "csrc/gp_internal.h")
MARK = "<!-- traffic:"
# the meshing chain's kernels, in launch order
CHAIN = ("k_label", "k_relink", "k_repair", "k_fixup", "k_walk", "k_tile_scan", "k_compact", "k_emit", "k_small")


def sources_sha256() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name: str) -> str:
    m = re.search(r"(k_[a-z_]+)(<\d+>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name.split("(")[0][:48]


def read_stats(d):
    out = []
    for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            out.append((short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    return out


def read_counters(d):
    """{kernel: {counter: [per-dispatch values]}}"""
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            acc[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return acc


def traffic_line(text: str):
    """The machine-readable traffic record of a summary, or None."""
    for line in text.splitlines():
        if line.startswith(MARK):
            return json.loads(line[len(MARK):].rstrip(" ->"))
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--pmc", action="append", default=[])
    ap.add_argument("--triangles", type=int, required=True, help="T of the profiled mesh (copy calibration)")
    ap.add_argument("--kernel", default="k_relink", help="kernel whose traffic is recorded")
    ap.add_argument("--command", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    copy_bytes = 12 * a.triangles
    fetch = read_counters(a.fetch)
    write = read_counters(a.write)
    cf = max(fetch["__amd_rocclr_copyBuffer"]["FETCH_SIZE"])
    cw = max(write["__amd_rocclr_copyBuffer"]["WRITE_SIZE"])
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)

    lines = [f"# {a.title}", "", "Commands (run from the repository root on the GPU host; bench.py, the",
             "package and its built library are committed files):", "", "```", a.command, "```", ""]
    lines += ["## Kernel time (rocprofv3 --kernel-trace --stats)", "",
              "| kernel | calls | avg us | % of GPU time |", "|---|---|---|---|"]
    for name, calls, avg, pct in sorted(read_stats(a.stats), key=lambda r: -r[3]):
        lines.append(f"| {name} | {calls} | {avg:.2f} | {pct:.2f} |")
    lines += ["", "## HBM traffic per launch (FETCH_SIZE, WRITE_SIZE)", "",
              f"Calibration on the largest copy kernel ({copy_bytes:,} B read and "
              f"written): FETCH_SIZE x {f_scale:.3f}, WRITE_SIZE x {w_scale:.3f} (KiB -> bytes).", "",
              "| kernel | dispatches | fetch MB | write MB |", "|---|---|---|---|"]
    rec = None
    avg_us = {name.split("<")[0]: avg for name, _, avg, _ in read_stats(a.stats)}
    chain = {}
    for k in sorted(set(fetch) | set(write)):
        fv, wv = fetch[k].get("FETCH_SIZE", []), write[k].get("WRITE_SIZE", [])
        if not fv or not wv:
            continue
        fb = sum(fv) / len(fv) * 1024 * f_scale
        wb = sum(wv) / len(wv) * 1024 * w_scale
        lines.append(f"| {k} | {len(fv)} | {fb / 1e6:.1f} | {wb / 1e6:.1f} |")
        base = short(k).split("<")[0]
        if base in CHAIN:
            chain[base] = {"fetch_bytes": round(fb), "write_bytes": round(wb), "avg_us": avg_us.get(base)}
        if base == a.kernel:
            rec = {"kernel": a.kernel, "fetch_bytes": round(fb), "write_bytes": round(wb),
                   "avg_us": avg_us.get(base), "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
                   "sources_sha256": sources_sha256()}
    if rec:
        rec["triangles"] = a.triangles
        rec["chain"] = chain
    for d in a.pmc:
        acc = read_counters(d)
        names = sorted({c for k in acc for c in acc[k]})
        if not names:
            continue
        lines += ["", f"## Counters per dispatch: {', '.join(names)}", "",
                  "| kernel | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
        for k in sorted(acc):
            if not k.startswith("k_"):
                continue
            vals = [acc[k][c] for c in names]
            lines.append(f"| {k} | " + " | ".join(f"{sum(v) / len(v):.4g}" if v else "" for v in vals) + " |")
    if rec:
        lines += ["", MARK + " " + json.dumps(rec) + " -->"]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {a.out}; traffic record: {rec}")


if __name__ == "__main__":
    main()
