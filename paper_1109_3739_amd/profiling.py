"""Summaries of rocprofv3 output (kernel trace database, PMC counter CSV).

    python -m paper_1109_3739_amd.profiling stats  <results.db> [regex]
    python -m paper_1109_3739_amd.profiling traffic <fetch_counter_collection.csv> <write_counter_collection.csv>
        <kernel_regex> <copy_regex> <copy_bytes> <out.json>
    python -m paper_1109_3739_amd.profiling counters <kernel_regex> <counter_collection.csv> [...]

`stats` prints per-kernel dispatch counts and durations (grouped by kernel
name and workgroup size).  `traffic` turns FETCH_SIZE / WRITE_SIZE (KiB per
dispatch) of the kernels matching kernel_regex into HBM bytes per launch,
each scaled by the ratio of the known size of a plain copy to what the same
counter reports for that copy (copy_regex), and records the digest of the
kernel sources the counters were taken on.  `counters` prints the average
per dispatch of every counter in the CSVs for the matching kernels.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1109_3739_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def kernel_stats(db: str, regex: str = ".*"):
    con = sqlite3.connect(db)
    rows = con.execute("select name, workgroup_x, lds_size, count(*), avg(duration), sum(duration), min(duration), "
                       "max(duration) from kernels group by name, workgroup_x, lds_size "
                       "order by sum(duration) desc").fetchall()
    pat = re.compile(regex)
    return [r for r in rows if pat.search(r[0])]


def print_stats(db: str, regex: str = ".*") -> None:
    print(f"{'total_ms':>10} {'calls':>6} {'avg_ms':>10} {'min_ms':>10} {'max_ms':>10} {'wg':>5} {'lds':>7}  kernel")
    for name, wg, lds, n, avg, tot, mn, mx in kernel_stats(db, regex):
        short = re.sub(r"\(.*", "", name)
        print(f"{tot / 1e6:10.3f} {n:6d} {avg / 1e6:10.4f} {mn / 1e6:10.4f} {mx / 1e6:10.4f} {wg:5d} {lds:7d}  {short}")


def pmc_per_dispatch(csv_path: str, counter: str):
    """{(kernel, workgroup size): [value per dispatch]} for one counter."""
    out = collections.defaultdict(list)
    acc = collections.defaultdict(float)
    meta = {}
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        acc[key] += float(r["Counter_Value"])
        meta[key] = (r["Kernel_Name"], int(r["Workgroup_Size"]))
    for key, v in acc.items():
        out[meta[key]].append(v)
    return out


def counters(kernel_regex: str, csv_paths) -> None:
    """Average per dispatch of every counter in the given rocprofv3 counter
    CSVs, per kernel and workgroup size, for kernels matching the regex."""
    pat = re.compile(kernel_regex)
    table = collections.defaultdict(dict)
    for path in csv_paths:
        names = sorted({r["Counter_Name"] for r in csv.DictReader(open(path))})
        for name in names:
            for (k, wg), vs in pmc_per_dispatch(path, name).items():
                if pat.search(k):
                    table[(re.sub(r"[(<].*", "", k), wg)][name] = (sum(vs) / len(vs), len(vs))
    for (k, wg), row in sorted(table.items()):
        print(f"{k} (workgroup {wg})")
        for name, (avg, n) in sorted(row.items()):
            print(f"  {name:36s} {avg:20.1f}   ({n} dispatches)")


def traffic(fetch_csv, write_csv, kernel_regex, copy_regex, copy_bytes, out_json):
    kpat, cpat = re.compile(kernel_regex), re.compile(copy_regex)
    res = {"source_digest": source_digest(), "copy_bytes": int(copy_bytes), "kernels": {}}
    scale = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = pmc_per_dispatch(path, name)
        copies = [v for (k, wg), vs in d.items() if cpat.search(k) for v in vs]
        if not copies:
            raise SystemExit(f"no copy kernel matching {copy_regex} in {path}")
        kib = max(copies)
        scale[name] = copy_bytes / (kib * 1024.0)
        res[f"{name}_copy_kib"] = kib
        for (k, wg), vs in d.items():
            if kpat.search(k):
                key = f"{re.sub(r'[(<].*', '', k)}_wg{wg}"
                e = res["kernels"].setdefault(key, {"dispatches": len(vs)})
                e[f"{name}_kib_avg"] = sum(vs) / len(vs)
    res["scale"] = scale
    for e in res["kernels"].values():
        fb = e.get("FETCH_SIZE_kib_avg", 0) * 1024 * scale["FETCH_SIZE"]
        wb = e.get("WRITE_SIZE_kib_avg", 0) * 1024 * scale["WRITE_SIZE"]
        e["hbm_read_bytes_per_launch"] = fb
        e["hbm_write_bytes_per_launch"] = wb
        e["hbm_bytes_per_launch"] = fb + wb
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "stats":
        print_stats(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ".*")
    elif len(sys.argv) >= 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3:])
    elif len(sys.argv) == 8 and sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], int(sys.argv[6]), sys.argv[7])
    else:
        print(__doc__)
        sys.exit(2)
