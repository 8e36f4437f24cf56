"""Host-only checks of bench.py's contract: it refuses more than one GPU
with a message before touching a device, and its byte models are the sums
stated in their docstrings (so the roofline figures it prints can be
recomputed from the counters)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_level_kernel_byte_model():
    st = {"visited": 10, "roots": 3, "bp_checks": 3, "normal_tests": 4, "label_scanned": 100,
          "candidates": 2}
    assert bench.level_kernel_bytes(st, 50) == 7 * 58 + 32 * 3 + 12 * 4 + 5 * 100 + 18 * 2


def test_weighted_step_byte_model():
    st = {"visited": 10, "normal_tests": 4, "label_scanned": 100, "edges": 50,
          "land_checks": 40, "filtered": 30, "improved": 7}
    assert bench.weighted_step_bytes(st) == (16 * 10 + 12 * 4 + 8 * 100 + 12 * 50 + 32 * 40
                                             - 4 * 30 + 16 * 7)


def test_expand_kernel_byte_model():
    # a reached neighbour's row: 32 B from the 4-bit copy of a 64-slot row
    # (t_bp = 50 pads to 64), t_bp B from the 8-bit rows (knob off, or a
    # 48-slot row)
    from paper_1304_4661_amd import binding
    st = {"candidates": 5, "edges": 100, "expand_earlier": 40, "expand_direct": 30,
          "expand_claims": 20}
    old = binding.get_tuning("packed_rows")
    try:
        binding.set_tuning("packed_rows", 1)
        assert bench.expand_kernel_bytes(st, 50) == (5 * 66 + 4 * 100 + 60 * 32 + 4 * 30
                                                     + 8 * 20)
        assert bench.expand_kernel_bytes(st, 40) == (5 * 56 + 4 * 100 + 60 * 40 + 4 * 30
                                                     + 8 * 20)
        binding.set_tuning("packed_rows", 0)
        assert bench.expand_kernel_bytes(st, 50) == (5 * 66 + 4 * 100 + 60 * 50 + 4 * 30
                                                     + 8 * 20)
    finally:
        binding.set_tuning("packed_rows", old)


def test_method_byte_model():
    c = {"bp_reached": 10, "bp_edges": 40, "bp_e0": 7, "bp_e1": 9, "root_staged": 11,
         "roots": 3, "visited": 20, "label_scanned": 100, "labeled": 6, "edges": 30,
         "entries": 6}
    bp, pr, fi = bench.s8d_bytes(c, 12, 4)
    assert bp == 10 * (8 + 17) + 40 * 5 + 16 * 16
    assert pr == 5 * 11 + 17 * 4 * 3 + 20 * (16 + 17 * 4) + 5 * 100 + 6 * (8 + 5) + 5 * 30
    assert fi == 2 * (5 * 6 + 8 * 12)


def test_query_pair_byte_model():
    import numpy as np
    ls, lt = np.array([3, 0]), np.array([5, 1])
    # per pair 9 B, per side 16 + t + 5 (entries + sentinel)
    assert bench.query_pair_bytes(4, ls, lt) == 2 * 9 + 4 * (16 + 4) + 5 * (4 + 1 + 6 + 2)
