"""The profile summaries' reductions (CPU): the window between two marker dispatches, per-kernel
averages, and the FETCH_SIZE / WRITE_SIZE calibration against the 256 MiB copy, on small synthetic
rocprofv3 CSV files."""
import csv
import os

import pytest

from paper_1502_00858_amd import prof_summary as ps

TRACE_FIELDS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
PMC_FIELDS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Counter_Name", "Counter_Value"]


def _write(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(fields, r)))


# (name, start ns, end ns): k_a twice and k_b once between the markers, one k_a before and after
TRACE = [
    ("void k_a(int)", 0, 4_000),
    ("at::cuda::spin_kernel(long)", 10_000, 12_000),
    ("void k_a(int)", 20_000, 30_000),
    ("k_b(double*)", 40_000, 46_000),
    ("void k_a(int)", 50_000, 64_000),
    ("at::cuda::spin_kernel(long)", 100_000, 102_000),
    ("void k_a(int)", 120_000, 220_000),
]


def _table(out):
    rows = {}
    for line in out.splitlines():
        cells = [c.strip() for c in line.strip("|").split("|")]
        if line.startswith("| ") and cells[0] not in ("kernel", "---"):
            rows[cells[0]] = cells[1:]
    return rows


def test_trace_window_and_averages(tmp_path, capsys):
    _write(str(tmp_path / "t" / "run_kernel_trace.csv"), TRACE_FIELDS, TRACE)
    ps.trace(str(tmp_path / "t"), "spin_kernel")
    out = capsys.readouterr().out
    assert "Window: 3 dispatches over 0.09 ms" in out   # from 12 us to 100 us
    rows = _table(out)
    assert set(rows) == {"void k_a", "k_b"}
    calls, total_ms, avg_us, share, full, full_avg = rows["void k_a"]
    assert (calls, avg_us, full, full_avg) == ("2", "12.0", "2", "12.0")
    assert rows["k_b"][:3] == ["1", "0.01", "6.0"]
    assert share == "80.0%"                            # 24 of 30 us
    ps.trace(str(tmp_path / "t"))                      # whole run: every dispatch
    rows = _table(capsys.readouterr().out)
    assert rows["void k_a"][0] == "4" and rows["at::cuda::spin_kernel"][0] == "2"


def test_window_needs_two_markers(tmp_path):
    _write(str(tmp_path / "t" / "run_kernel_trace.csv"), TRACE_FIELDS, TRACE[:3])
    with pytest.raises(SystemExit):
        ps.trace(str(tmp_path / "t"), "spin_kernel")


def test_pmc_calibration_and_window(tmp_path, capsys):
    copy = "__amd_rocclr_copyBuffer"
    # the copy reads 131072 KiB for FETCH (scale 2) and 262144 KiB for WRITE (scale 1)
    fetch = [(copy, 200_000, 210_000, "FETCH_SIZE", 131072.0)]
    write = [(copy, 200_000, 210_000, "WRITE_SIZE", 262144.0)]
    for name, s, e, fv, wv in (("spin_kernel", 0, 10, 0.0, 0.0), ("k_x", 20, 30, 1000.0, 500.0),
                               ("k_x", 40, 50, 3000.0, 1500.0), ("spin_kernel", 60, 70, 0.0, 0.0),
                               ("k_x", 80, 90, 1e6, 1e6)):
        fetch.append((name, s, e, "FETCH_SIZE", fv))
        write.append((name, s, e, "WRITE_SIZE", wv))
    _write(str(tmp_path / "f" / "run_counter_collection.csv"), PMC_FIELDS, fetch)
    _write(str(tmp_path / "w" / "run_counter_collection.csv"), PMC_FIELDS, write)
    ps.pmc(str(tmp_path / "f"), str(tmp_path / "w"), "spin_kernel")
    out = capsys.readouterr().out
    assert "(x2.0000)" in out and "(x1.0000)" in out
    rows = _table(out)
    assert set(rows) == {"k_x"}                        # markers and the late dispatch left out
    n, f_mb, w_mb = rows["k_x"]
    assert n == "2"
    assert float(f_mb) == pytest.approx(2000.0 * 1024 * 2 / 1e6, abs=0.01)
    assert float(w_mb) == pytest.approx(1000.0 * 1024 / 1e6, abs=0.01)
