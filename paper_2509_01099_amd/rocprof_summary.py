"""Summaries of rocprofv3 output for the profiles/ folder.

kernel-stats:  python -m paper_2509_01099_amd.rocprof_summary stats <run_kernel_stats.csv>
traffic:       python -m paper_2509_01099_amd.rocprof_summary traffic <fetch counter csv>
                   <write counter csv> <kernel name substring> <copy bytes> <digest>
FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled by the
ratio of the known size of a plain copy kernel's transfer to what the same
counter reads for that copy (the copy is dispatched in the same run).
"""
from __future__ import annotations

import csv
import json
import sys
from collections import defaultdict


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg ns | min ns | max ns | % |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {r['Name'][:110]} | {r['Calls']} | {float(r['AverageNs']):.0f} | "
                   f"{r['MinNs']} | {r['MaxNs']} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def _per_kernel(path: str):
    agg = defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, digest: str) -> dict:
    res = {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        agg = _per_kernel(path)
        copies = [max(v) for k, v in agg.items() if "copyBuffer" in k or "elementwise" in k.lower()
                  or "copy" in k.lower()]
        copy_kib = max(copies)
        factor = copy_bytes / (copy_kib * 1024.0)
        ks = [v for k, v in agg.items() if kernel in k]
        vals = [x for v in ks for x in v]
        avg_kib = sum(vals) / len(vals)
        res[name] = {"kib_per_dispatch": avg_kib, "copy_kib": copy_kib, "factor": factor,
                     "bytes_per_launch": avg_kib * 1024.0 * factor, "dispatches": len(vals)}
    res["bytes_per_launch"] = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    res["kernel"] = kernel
    res["kernel_digest"] = digest
    return res


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    else:
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]),
                                 sys.argv[6]), indent=1))
