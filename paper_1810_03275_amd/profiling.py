"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1810_03275_amd.profiling trace <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1810_03275_amd.profiling traffic <fetch.csv> <write.csv> <kernel> \
        <copy_bytes> <out.json> "<command>" [median|top]
    python -m paper_1810_03275_amd.profiling counters <counter_collection.csv> <out.md> \
        "<title>" "<command>"

trace   : per-kernel calls / average / total duration table from a
          `rocprofv3 --kernel-trace --stats --output-format csv` run.
counters: per-kernel median over dispatches of every counter of a
          `rocprofv3 --pmc ... --output-format csv` run.
traffic : HBM bytes per launch of one kernel from two `--pmc FETCH_SIZE` and
          `--pmc WRITE_SIZE` runs (KiB per dispatch), each scaled by the factor
          that makes the same counter read exactly copy_bytes for the largest
          __amd_rocclr_copyBuffer dispatch of the run (a plain device copy of
          known size).  The record carries the hash of the projector sources
          so that a stale record is ignored by bench.py.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("radon.hip", "common.hpp", "plan.cpp", "tv_update.hpp"):
        with open(os.path.join(ROOT, "paper_1810_03275_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("void ", "").strip()


def trace_summary(stats_csv: str, out_md: str, command: str, top: int = 14) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# Kernel trace summary", "", f"Command: `{command}`", "",
             "| kernel | calls | average (us) | total (ms) | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        t = float(r["TotalDurationNs"])
        lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['AverageNs'])/1e3:.2f} | "
                     f"{t/1e6:.3f} | {100*t/total:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_dispatch(path: str):
    d = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        key = int(r["Dispatch_Id"])
        d[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    return d, names


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: float, out_json: str,
            command: str, select: str = "median") -> dict:
    """select = "median": median over the kernel's dispatches; "top": median
    over those above 1.5 x the smallest, if any (the in-path launches, which
    also read and write the sinogram-side update, against the plain
    projections of the set-up)."""
    out = {}
    for tag, path in (("fetch", fetch_csv), ("write", write_csv)):
        d, names = _per_dispatch(path)
        copies = [v for k, v in d.items() if "copyBuffer" in names[k]]
        ref = max(copies) * 1024.0
        factor = copy_bytes / ref
        vals = [v * 1024.0 * factor for k, v in d.items() if kernel in names[k]]
        if select == "top":
            big = [v for v in vals if v > 1.5 * min(vals)]
            vals = big or vals
        vals.sort()
        med = vals[len(vals) // 2]
        out[tag] = {"bytes_per_launch": med, "scale": factor, "dispatches": len(vals),
                    "select": select}
    rec = {"kernel": kernel, "bytes_per_launch": out["fetch"]["bytes_per_launch"]
           + out["write"]["bytes_per_launch"], "fetch": out["fetch"], "write": out["write"],
           "calibration": f"plain device copy of {copy_bytes:.0f} bytes",
           "source_hash": kernel_source_hash(), "command": command}
    json.dump(rec, open(out_json, "w"), indent=1)
    return rec


def counters_summary(path: str, out_md: str, title: str, command: str, top: int = 12) -> None:
    per = defaultdict(lambda: defaultdict(float))
    names = {}
    for r in csv.DictReader(open(path)):
        key = int(r["Dispatch_Id"])
        per[key][r["Counter_Name"]] += float(r["Counter_Value"])
        names[key] = _short(r["Kernel_Name"])
    by_kernel = defaultdict(list)
    for key, vals in per.items():
        by_kernel[names[key]].append(vals)
    cols = sorted({c for vals in per.values() for c in vals})
    rows = []
    for nm, lst in by_kernel.items():
        med = {c: sorted(v.get(c, 0.0) for v in lst)[len(lst) // 2] for c in cols}
        rows.append((nm, len(lst), med))
    rows.sort(key=lambda x: -x[2].get("SQ_INSTS_VALU", 0.0))
    lines = [f"# {title}", "", f"Command: `{command}`", "",
             "| kernel | dispatches | " + " | ".join(c.replace("SQ_", "") for c in cols) + " |",
             "|---|---|" + "---|" * len(cols)]
    for nm, cnt, med in rows[:top]:
        lines.append(f"| {nm} | {cnt} | " + " | ".join(f"{med[c]:.4g}" for c in cols) + " |")
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace_summary(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]), sys.argv[6],
                      sys.argv[7], sys.argv[8] if len(sys.argv) > 8 else "median"))
    elif sys.argv[1] == "counters":
        counters_summary(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
