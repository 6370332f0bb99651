"""Summaries of rocprofv3 output for the profiles/ directory.

kernel_stats(csv): the --stats kernel table (name, calls, average ns, share).
counters(csv, names): mean value per dispatch of each requested counter for
every kernel in a --pmc counter_collection CSV (FETCH_SIZE and WRITE_SIZE are
in KiB per dispatch).
"""
from __future__ import annotations

import csv
import sys
from collections import defaultdict


def kernel_stats(path, top=20):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows[:top]:
        out.append(dict(name=r["Name"], calls=int(r["Calls"]), avg_ns=float(r["AverageNs"]),
                        total_ns=float(r["TotalDurationNs"]), percent=float(r["Percentage"])))
    return out


def counters(path):
    acc = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName")
        acc[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: (sum(v) / len(v), len(v)) for c, v in d.items()} for k, d in acc.items()}


def short(name):
    return name.split("(")[0].replace("void ", "")


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    if mode == "stats":
        for r in kernel_stats(path):
            print("| %s | %d | %.2f | %.2f |" % (short(r["name"]), r["calls"], r["avg_ns"] / 1e3, r["percent"]))
    else:
        for k, d in sorted(counters(path).items()):
            for c, (m, n) in d.items():
                print("| %s | %s | %.1f | %d |" % (short(k), c, m, n))
