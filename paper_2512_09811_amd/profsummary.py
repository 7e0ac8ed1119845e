"""Summarize rocprofv3 output.

  python -m paper_2512_09811_amd.profsummary <results.db>
      kernel-trace database: total/average duration per kernel, sorted by total
      time (the database's top_kernels view reports microseconds);
  python -m paper_2512_09811_amd.profsummary --counters <counter_collection.csv> [...]
      per-dispatch counters (e.g. FETCH_SIZE, WRITE_SIZE in KiB): mean per kernel,
      and the largest dispatch of the device copy kernel (the calibration copy).
"""
import csv
import sqlite3
import sys
from collections import defaultdict


def summarize(db, limit=25):
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    out = ["| kernel | calls | total s | avg ms | % of GPU time |", "|---|---|---|---|---|"]
    for name, n, tot, avg, pct in rows[:limit]:
        short = name.replace("ppw::(anonymous namespace)::", "").split("(")[0]
        out.append(f"| `{short}` | {n} | {tot / 1e6:.2f} | {avg / 1e3:.2f} | {pct:.1f} |")
    return "\n".join(out)


def _col(row, *names):
    for n in names:
        for k in row:
            if k and k.lower() == n.lower():
                return row[k]
    raise KeyError(names)


def counters(paths, limit=12):
    per = defaultdict(list)  # (kernel, counter) -> values per dispatch
    for p in paths:
        with open(p, newline="") as f:
            for row in csv.DictReader(f):
                k = _col(row, "Kernel_Name", "kernel_name")
                c = _col(row, "Counter_Name", "counter_name")
                v = float(_col(row, "Counter_Value", "counter_value"))
                per[(k, c)].append(v)
    names = sorted({c for _, c in per})
    kern = sorted({k for k, _ in per}, key=lambda k: -max(sum(per.get((k, c), [0])) for c in names))
    out = ["| kernel | dispatches | " + " | ".join(f"mean {c}" for c in names) + " |",
           "|---|---|" + "---|" * len(names)]
    for k in kern[:limit]:
        short = k.replace("ppw::(anonymous namespace)::", "").split("(")[0]
        n = max(len(per.get((k, c), [])) for c in names)
        vals = " | ".join(f"{sum(per[(k, c)]) / len(per[(k, c)]):.0f}" if per.get((k, c)) else "-" for c in names)
        out.append(f"| `{short}` | {n} | {vals} |")
    for k in kern:
        if "copyBuffer" in k:
            big = " | ".join(f"{max(per[(k, c)]):.0f}" if per.get((k, c)) else "-" for c in names)
            out.append(f"| largest `{k.split('(')[0]}` dispatch | 1 | {big} |")
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "--counters":
        print(counters(sys.argv[2:]))
    else:
        print(summarize(sys.argv[1]))
