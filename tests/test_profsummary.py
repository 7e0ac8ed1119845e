"""The rocprofv3 summary helper (paper_2512_09811_amd/profsummary.py) on synthetic counter
files: the HBM-traffic calibration takes the 1 GiB device copies (the copy dispatches
that write exactly 1 GiB), not the largest copy of the run, and scales a kernel's
per-dispatch counters by it."""
import csv

import pytest

from paper_2512_09811_amd import profsummary


def _counters(path, name, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (kernel, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": name, "Counter_Value": value})


def _trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 0
        for kernel, ns in rows:
            w.writerow({"Kernel_Name": kernel, "Start_Timestamp": t, "End_Timestamp": t + ns})
            t += ns + 1000


def test_calibration_uses_the_1gib_copies(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    kern = "void ppw::(anonymous namespace)::some_kernel(long, double*)"
    gib = 1048576.0  # KiB in a GiB
    # a 14 GiB setup copy first, then the kernel twice, then three 1 GiB calibration copies;
    # fetch counters read half the bytes (as on the device), write counters all of them
    fetch = [(copy, 7.0 * gib), (kern, 1000.0), (kern, 3000.0)] + [(copy, 0.5 * gib)] * 3
    write = [(copy, 14.0 * gib), (kern, 500.0), (kern, 500.0)] + [(copy, gib)] * 3
    _counters(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _counters(tmp_path / "w.csv", "WRITE_SIZE", write)
    _trace(tmp_path / "t.csv", [(copy, 10), (kern, 1_000_000), (kern, 1_000_000)] + [(copy, 10)] * 3)
    out = profsummary.bandwidth(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "t.csv"))
    assert out.splitlines()[0].startswith("calibration: FETCH_SIZE x2.0000, WRITE_SIZE x1.0000")
    row = next(line for line in out.splitlines() if "some_kernel" in line)
    cells = [c.strip() for c in row.strip("|").split("|")]
    # mean fetch 2000 KiB x 2 = 4000 KiB = 4.096 MB read; 500 KiB = 0.512 MB written; 1 ms each
    assert cells[2] == "4.10" and cells[3] == "0.51"
    assert cells[5] == "5"  # (4.096 + 0.512) MB per 1 ms = 4.6 GB/s, printed rounded


def test_missing_calibration_is_an_error(tmp_path):
    kern = "void ppw::(anonymous namespace)::some_kernel(long, double*)"
    _counters(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 100.0), (kern, 1.0)])
    _counters(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 200.0), (kern, 1.0)])
    _trace(tmp_path / "t.csv", [(kern, 100)])
    with pytest.raises(SystemExit):
        profsummary.bandwidth(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "t.csv"))
