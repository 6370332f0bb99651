"""Summaries of rocprofv3 output for the profiles/ directory.

kernel_stats(csv): the --stats kernel table (name, calls, average ns, share).
trace(csv, min_us): per kernel from the --kernel-trace CSV: launches, mean and
median duration of all launches and of those longer than min_us (launches
enqueued past the solver's device-side convergence test exit at once and
take about a microsecond).
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


def trace(path, min_us=2.0):
    d = defaultdict(list)
    rd = csv.DictReader(open(path))
    cols = rd.fieldnames or []
    pick = lambda *names: next((n for n in names if n in cols), None)
    kn, t0, t1 = pick("Kernel_Name", "Kernel-Name"), pick("Start_Timestamp", "BeginNs"), pick("End_Timestamp", "EndNs")
    if not (kn and t0 and t1):
        raise KeyError("unexpected kernel-trace columns: %s" % cols)
    for r in rd:
        d[r[kn]].append((int(r[t1]) - int(r[t0])) / 1e3)
    out = []
    for name, v in d.items():
        v.sort()
        w = [x for x in v if x > min_us]
        out.append(dict(name=name, launches=len(v), mean_us=sum(v) / len(v), median_us=v[len(v) // 2],
                        working=len(w), working_mean_us=sum(w) / len(w) if w else 0.0,
                        working_median_us=w[len(w) // 2] if w else 0.0, total_us=sum(v)))
    out.sort(key=lambda e: -e["total_us"])
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
    elif mode == "trace":
        for r in trace(path)[:16]:
            print("| %s | %d | %.2f | %.2f | %d | %.2f | %.2f |" % (short(r["name"]), r["launches"], r["mean_us"],
                                                               r["median_us"], r["working"], r["working_mean_us"],
                                                               r["working_median_us"]))
    else:
        for k, d in sorted(counters(path).items()):
            for c, (m, n) in d.items():
                print("| %s | %s | %.1f | %d |" % (short(k), c, m, n))
