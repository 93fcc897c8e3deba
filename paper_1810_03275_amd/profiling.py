"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1810_03275_amd.profiling trace <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1810_03275_amd.profiling counters <counter_collection.csv> <out.md> \
        "<title>" "<command>"
    python -m paper_1810_03275_amd.profiling traffic <fetch.csv> <write.csv> <copy_bytes> \
        <out.json> "<command>"

trace   : per-kernel calls / average / total duration table from a
          `rocprofv3 --kernel-trace --stats --output-format csv` run, and the
          same as JSON next to the table.
counters: per-kernel median over dispatches of every counter of a
          `rocprofv3 --pmc ... --output-format csv` run, as a table and as
          JSON next to it.
traffic : HBM bytes per dispatch of every kernel from two `--pmc FETCH_SIZE`
          and `--pmc WRITE_SIZE` runs (KiB per dispatch), each scaled by the
          factor that makes the same counter read exactly copy_bytes for the
          largest __amd_rocclr_copyBuffer dispatch of the run (a plain device
          copy of known size); median over each kernel's dispatches.

Every JSON record carries the hash of the library's kernel sources
(kernel_source_hash), so that a reader can tell a stale record (taken on
other kernels) from a current one.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_03275_amd", "csrc")


def kernel_source_hash() -> str:
    """Hash of every source of the library (device code and launchers)."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".cpp", ".hpp")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("void ", "").strip()


def trace_summary(stats_csv: str, out_md: str, command: str, top: int = 16) -> dict:
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# Kernel trace summary", "", f"Command: `{command}`", "",
             "| kernel | calls | average (us) | total (ms) | % |", "|---|---|---|---|---|"]
    rec = {"command": command, "source_hash": kernel_source_hash(), "kernels": {}}
    for r in rows:
        t = float(r["TotalDurationNs"])
        nm = short_name(r["Name"])
        rec["kernels"][nm] = {"calls": int(r["Calls"]), "average_us": float(r["AverageNs"]) / 1e3,
                              "total_ms": t / 1e6}
    for r in rows[:top]:
        t = float(r["TotalDurationNs"])
        lines.append(f"| {short_name(r['Name'])} | {r['Calls']} | "
                     f"{float(r['AverageNs'])/1e3:.2f} | {t/1e6:.3f} | {100*t/total:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    json.dump(rec, open(os.path.splitext(out_md)[0] + ".json", "w"), indent=1)
    return rec


def _per_dispatch(path: str):
    d = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        key = int(r["Dispatch_Id"])
        d[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    return d, names


def _median(vals):
    vals = sorted(vals)
    return vals[len(vals) // 2]


def traffic(fetch_csv: str, write_csv: str, copy_bytes: float, out_json: str,
            command: str) -> dict:
    per = {}
    scale = {}
    for tag, path in (("fetch", fetch_csv), ("write", write_csv)):
        d, names = _per_dispatch(path)
        copies = [v for k, v in d.items() if "copyBuffer" in names[k]]
        factor = copy_bytes / (max(copies) * 1024.0)
        scale[tag] = factor
        by = defaultdict(list)
        for k, v in d.items():
            by[short_name(names[k])].append(v * 1024.0 * factor)
        per[tag] = by
    kernels = {}
    for nm in sorted(set(per["fetch"]) | set(per["write"])):
        f = per["fetch"].get(nm, [])
        w = per["write"].get(nm, [])
        kernels[nm] = {"fetch_bytes": _median(f) if f else None,
                       "write_bytes": _median(w) if w else None,
                       "dispatches": max(len(f), len(w))}
    rec = {"calibration": f"plain device copy of {copy_bytes:.0f} bytes",
           "scale": scale, "source_hash": kernel_source_hash(), "command": command,
           "kernels": kernels}
    json.dump(rec, open(out_json, "w"), indent=1)
    return rec


def counters_summary(path: str, out_md: str, title: str, command: str, top: int = 16) -> dict:
    per = defaultdict(lambda: defaultdict(float))
    names = {}
    for r in csv.DictReader(open(path)):
        key = int(r["Dispatch_Id"])
        per[key][r["Counter_Name"]] += float(r["Counter_Value"])
        names[key] = short_name(r["Kernel_Name"])
    by_kernel = defaultdict(list)
    for key, vals in per.items():
        by_kernel[names[key]].append(vals)
    cols = sorted({c for vals in per.values() for c in vals})
    rows = []
    for nm, lst in by_kernel.items():
        med = {c: _median([v.get(c, 0.0) for v in lst]) for c in cols}
        rows.append((nm, len(lst), med))
    key0 = "SQ_INSTS_VALU" if "SQ_INSTS_VALU" in cols else cols[0]
    rows.sort(key=lambda x: -x[2].get(key0, 0.0))
    lines = [f"# {title}", "", f"Command: `{command}`", "",
             "| kernel | dispatches | " + " | ".join(c.replace("SQ_", "") for c in cols) + " |",
             "|---|---|" + "---|" * len(cols)]
    for nm, cnt, med in rows[:top]:
        lines.append(f"| {nm} | {cnt} | " + " | ".join(f"{med[c]:.4g}" for c in cols) + " |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    rec = {"title": title, "command": command, "source_hash": kernel_source_hash(),
           "kernels": {nm: dict(med, dispatches=cnt) for nm, cnt, med in rows}}
    json.dump(rec, open(os.path.splitext(out_md)[0] + ".json", "w"), indent=1)
    return rec


def load_record(path: str):
    """A profiles/ JSON record if it was taken on the current kernel sources,
    else None."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def find_kernel(rec, prefix: str, suffix: str = ""):
    """The entry of the kernel whose short name starts with prefix (and ends
    with suffix) with the most dispatches, or None."""
    if not rec:
        return None
    best = None
    for nm, ent in rec["kernels"].items():
        if nm.startswith(prefix) and nm.endswith(suffix):
            cnt = ent.get("dispatches", ent.get("calls", 0))
            if best is None or cnt > best[1]:
                best = (nm, cnt, ent)
    return None if best is None else dict(best[2], name=best[0])


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace_summary(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5],
                                 sys.argv[6]), indent=1)[:2000])
    elif sys.argv[1] == "counters":
        counters_summary(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
