"""Summarize rocprofv3 output.

  python -m paper_2512_09811_amd.profsummary <results.db | kernel_stats.csv>
      kernel trace: total/average duration per kernel, sorted by total time;
  python -m paper_2512_09811_amd.profsummary --grid <kernel_trace.csv> <name substring>
      durations of one kernel's dispatches grouped by grid size (launch shape);
  python -m paper_2512_09811_amd.profsummary --counters <counter_collection.csv> [...]
      per-dispatch counters (e.g. FETCH_SIZE, WRITE_SIZE in KiB): mean per kernel,
      and the largest dispatch of the device copy kernel (the calibration copy);
  python -m paper_2512_09811_amd.profsummary --bandwidth <fetch.csv> <write.csv> <kernel_trace.csv>
      calibrated HBM bytes per dispatch (FETCH_SIZE and WRITE_SIZE scaled by what they
      read for the largest device copy of 1 GiB in the same runs) and the bandwidth they
      imply over each kernel's mean duration in the trace;
  python -m paper_2512_09811_amd.profsummary --mfma <counter_collection.csv>
      MFMA work (SQ_INSTS_VALU_MFMA_MOPS_*, 512 flops each), MFMA busy cycles and LDS
      bank conflicts per kernel and launch shape.
"""
import csv
import sqlite3
import sys
from collections import defaultdict


def short(name):
    """Kernel name without the namespace and the argument list."""
    n = name.replace("ppw::(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and i > 0:
            return n[:i]
    return n


def summarize(path, limit=25):
    out = ["| kernel | calls | total s | avg ms | % of GPU time |", "|---|---|---|---|---|"]
    if path.endswith(".csv"):
        rows = [(r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]), float(r["Percentage"]))
                for r in csv.DictReader(open(path))]
        rows.sort(key=lambda r: -r[2])
        for name, n, tot, avg, pct in rows[:limit]:
            out.append(f"| `{short(name)}` | {n} | {tot / 1e9:.2f} | {avg / 1e6:.3f} | {pct:.1f} |")
        return "\n".join(out)
    # read-only: a path that does not exist is an error, never a new empty database
    c = sqlite3.connect(f"file:{path}?mode=ro", uri=True)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    for name, n, tot, avg, pct in rows[:limit]:
        out.append(f"| `{short(name)}` | {n} | {tot / 1e6:.2f} | {avg / 1e3:.2f} | {pct:.1f} |")
    return "\n".join(out)


def by_grid(trace, substring):
    per = defaultdict(list)
    for r in csv.DictReader(open(trace)):
        if substring in r["Kernel_Name"]:
            g = r.get("Grid_Size") or r.get("Grid_Size_X")
            per[(short(r["Kernel_Name"]), g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
    out = ["| kernel | grid (threads) | dispatches | mean ms | min ms | max ms |", "|---|---|---|---|---|---|"]
    for (k, g), v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| `{k}` | {g} | {len(v)} | {sum(v) / len(v):.3f} | {min(v):.3f} | {max(v):.3f} |")
    return "\n".join(out)


def _col(row, *names):
    for n in names:
        for k in row:
            if k and k.lower() == n.lower():
                return row[k]
    raise KeyError(names)


def _per_kernel(paths, key=lambda row: short(_col(row, "Kernel_Name", "kernel_name"))):
    per = defaultdict(list)  # (kernel, counter) -> values per dispatch
    for p in paths:
        with open(p, newline="") as f:
            for row in csv.DictReader(f):
                per[(key(row), _col(row, "Counter_Name", "counter_name"))].append(
                    float(_col(row, "Counter_Value", "counter_value")))
    return per


def counters(paths, limit=12):
    per = _per_kernel(paths)
    names = sorted({c for _, c in per})
    kern = sorted({k for k, _ in per}, key=lambda k: -max(sum(per.get((k, c), [0])) for c in names))
    out = ["| kernel | dispatches | " + " | ".join(f"mean {c}" for c in names) + " |",
           "|---|---|" + "---|" * len(names)]
    for k in kern[:limit]:
        n = max(len(per.get((k, c), [])) for c in names)
        vals = " | ".join(f"{sum(per[(k, c)]) / len(per[(k, c)]):.0f}" if per.get((k, c)) else "-" for c in names)
        out.append(f"| `{k}` | {n} | {vals} |")
    for k in kern:
        if "copyBuffer" in k:
            big = " | ".join(f"{max(per[(k, c)]):.0f}" if per.get((k, c)) else "-" for c in names)
            out.append(f"| largest `{k}` dispatch | 1 | {big} |")
    return "\n".join(out)


def bandwidth(fetch, write, trace, limit=40):
    per = _per_kernel([fetch, write])
    dur = defaultdict(list)
    for r in csv.DictReader(open(trace)):
        dur[short(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    # the calibration copies are the 1 GiB device copies: the copy dispatches that write
    # exactly 1 GiB, and the dispatches at the same positions of the (deterministic)
    # fetch run
    cfv = per[("__amd_rocclr_copyBuffer", "FETCH_SIZE")]
    cwv = per[("__amd_rocclr_copyBuffer", "WRITE_SIZE")]
    idx = [i for i, x in enumerate(cwv) if x == 1048576.0 and i < len(cfv)]
    if not idx:
        raise SystemExit("no 1 GiB calibration copy in the counter runs (bench.py --copy-calibration)")
    cf = 1048576.0 / (sum(cfv[i] for i in idx) / len(idx))
    cw = 1.0
    rows = []
    for k in dur:
        f, w = per.get((k, "FETCH_SIZE")), per.get((k, "WRITE_SIZE"))
        if not f or not w:
            continue
        fb = 1024.0 * cf * sum(f) / len(f)
        wb = 1024.0 * cw * sum(w) / len(w)
        t = sum(dur[k]) / len(dur[k])
        rows.append((k, len(dur[k]), fb, wb, t, sum(dur[k])))
    rows.sort(key=lambda r: -r[5])
    out = [f"calibration: FETCH_SIZE x{cf:.4f}, WRITE_SIZE x{cw:.4f} (1 GiB device copy)", "",
           "| kernel | dispatches | MB read | MB written | mean us | GB/s | % of 8 TB/s | total ms |",
           "|---|---|---|---|---|---|---|---|"]
    for k, n, fb, wb, t, tot in rows[:limit]:
        bw = (fb + wb) / t / 1e9
        out.append(f"| `{k}` | {n} | {fb / 1e6:.2f} | {wb / 1e6:.2f} | {t * 1e6:.1f} | {bw:.0f} | {bw / 80:.1f} | "
                   f"{tot * 1e3:.1f} |")
    return "\n".join(out)


def mfma(path, limit=14):
    per = _per_kernel([path], key=lambda row: (short(row["Kernel_Name"]), row.get("Grid_Size", "")))
    kern = sorted({k for k, _ in per}, key=lambda k: -sum(per.get((k, "GRBM_GUI_ACTIVE"), [0])))
    out = ["| kernel | grid | dispatches | MFMA flops per dispatch (MOPS x 512) | MFMA busy / GUI active | "
           "LDS bank conflict / LDS active |", "|---|---|---|---|---|---|"]
    for k in kern[:limit]:
        m = lambda c: (sum(per[(k, c)]) / len(per[(k, c)])) if per.get((k, c)) else 0.0
        mops = sum(m(c) for (kk, c) in per if kk == k and c.startswith("SQ_INSTS_VALU_MFMA_MOPS"))
        g = m("GRBM_GUI_ACTIVE")
        busy = m("SQ_VALU_MFMA_BUSY_CYCLES") / g if g else 0.0
        act = m("SQ_LDS_IDX_ACTIVE")
        conf = m("SQ_LDS_BANK_CONFLICT") / act if act else 0.0
        out.append(f"| `{k[0]}` | {k[1]} | {len(per[(k, 'GRBM_GUI_ACTIVE')])} | {512 * mops:.3e} | {busy:.1f} | "
                   f"{conf:.3f} |")
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) < 2 or sys.argv[1] in ("-h", "--help") or (
            sys.argv[1].startswith("-") and sys.argv[1] not in ("--counters", "--bandwidth", "--mfma", "--grid")):
        print(__doc__)
        sys.exit(0 if len(sys.argv) >= 2 and sys.argv[1] in ("-h", "--help") else 2)
    if sys.argv[1] == "--counters":
        print(counters(sys.argv[2:]))
    elif sys.argv[1] == "--bandwidth":
        print(bandwidth(*sys.argv[2:5]))
    elif sys.argv[1] == "--mfma":
        print(mfma(sys.argv[2]))
    elif sys.argv[1] == "--grid":
        print(by_grid(sys.argv[2], sys.argv[3]))
    else:
        print(summarize(sys.argv[1]))
