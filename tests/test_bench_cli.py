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
    st = {"candidates": 5, "edges": 100, "expand_earlier": 40, "expand_direct": 30,
          "expand_claims": 20}
    assert bench.expand_kernel_bytes(st, 50) == (5 * 66 + 4 * 100 + 60 * 50 + 4 * 30
                                                 + 8 * 20)
