"""Host-only checks of the rocprofv3 summary tool on small synthetic CSV
files laid out as rocprofv3 writes them: per-kernel stats, the window of
the last dispatches, HBM traffic scaled by a copy probe, device-busy
fractions of builds, and per-counter sums."""
import csv
import os

import pytest

from paper_1304_4661_amd import rocprof_summary as rs


def _write(d, name, header, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, name), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_stats_and_window(tmp_path):
    d = str(tmp_path / "trace")
    _write(d, "run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
           [["k_a", 3, 300, 100, 75.0], ["k_b", 1, 100, 100, 25.0]])
    assert rs.stats(d) == [("k_a", 3, 300.0, 100.0, 75.0), ("k_b", 1, 100.0, 100.0, 25.0)]
    # dispatches out of start order; the window takes the last two k_a ones
    _write(d, "run_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [["k_a<64>", 500, 560], ["k_a<64>", 100, 110], ["k_b", 200, 900], ["k_a<8>", 300, 330]])
    assert rs.window(d, "k_a", 2) == (2, 90.0, 45.0)
    assert rs.window(d, "k_a", 10) == (3, 100.0, 100 / 3)
    assert rs.window(d, "k_c", 2) == (0, 0.0, None)


def test_traffic_scales_by_the_copy_probe(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _write(str(tmp_path / "f"), "run_counter_collection.csv", hdr,
           [[1, "k_x", "FETCH_SIZE", 100], [2, "k_y", "FETCH_SIZE", 7], [3, "k_x", "FETCH_SIZE", 300]])
    _write(str(tmp_path / "w"), "run_counter_collection.csv", hdr,
           [[1, "k_x", "WRITE_SIZE", 10], [3, "k_x", "WRITE_SIZE", 30]])
    # the copy of 1 MiB read 512 KiB and wrote 1024 KiB by the counters
    _write(str(tmp_path / "cf"), "run_counter_collection.csv", hdr,
           [[1, "copy", "FETCH_SIZE", 512], [2, "fill", "FETCH_SIZE", 1]])
    _write(str(tmp_path / "cw"), "run_counter_collection.csv", hdr, [[1, "copy", "WRITE_SIZE", 1024]])
    t = rs.traffic("k_x", str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                   str(tmp_path / "cw"), float(1 << 20))
    assert t["dispatches"] == 2 and t["fetch_kib_per_dispatch"] == 200 and t["write_kib_per_dispatch"] == 20
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["bytes_per_launch"] == 200 * 1024 * 2 + 20 * 1024
    last = rs.traffic("k_x", str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                      str(tmp_path / "cw"), float(1 << 20), last=1)
    assert last["fetch_kib_per_dispatch"] == 300 and last["dispatches"] == 1


def test_busy_merges_overlapping_kernels_per_build(tmp_path):
    d = str(tmp_path / "trace")
    rows = [
        # build 1: span 0..100, kernels 0..30 and 20..50 overlap, 60..100
        ["k_validate_graph", 0, 10], ["k_a", 10, 30], ["k_b", 20, 50], ["k_final_copy", 60, 100],
        ["k_query", 120, 200],  # after the build's end: not counted
        # build 2: span 300..400, kernels back to back
        ["k_validate_graph", 300, 320], ["k_a", 320, 350], ["k_final_copy", 350, 400],
    ]
    _write(d, "run_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    got = rs.busy(d)
    assert got == [(100, 90), (100, 100)]


def test_busy_skips_a_build_without_its_end(tmp_path):
    d = str(tmp_path / "trace")
    _write(d, "run_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [["k_validate_graph", 0, 10], ["k_a", 10, 30]])
    assert rs.busy(d) == []


def test_counters_sum_per_counter(tmp_path):
    d = str(tmp_path / "sq")
    _write(d, "run_counter_collection.csv", ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
           [[1, "k", "SQ_WAVES", 4], [2, "k", "SQ_WAVES", 6], [1, "k", "SQ_INSTS_VALU", 2.5]])
    assert rs.counters(d) == {"SQ_INSTS_VALU": (2.5, 1), "SQ_WAVES": (10.0, 2)}


def test_missing_files_are_reported(tmp_path):
    with pytest.raises(FileNotFoundError):
        rs.stats(str(tmp_path))
