"""Summarize a rocprofv3 results database (kernel-trace) as a per-kernel table.

Usage: python -m paper_2512_09811_amd.profsummary <results.db> [command-string]
Prints total/average duration per kernel, sorted by total time (the database's
top_kernels view reports microseconds).
"""
import sqlite3
import sys


def summarize(db, limit=25):
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    out = ["| kernel | calls | total s | avg ms | % of GPU time |", "|---|---|---|---|---|"]
    for name, n, tot, avg, pct in rows[:limit]:
        short = name.replace("ppw::(anonymous namespace)::", "").split("(")[0]
        out.append(f"| `{short}` | {n} | {tot / 1e6:.2f} | {avg / 1e3:.2f} | {pct:.1f} |")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarize(sys.argv[1]))
