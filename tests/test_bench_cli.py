"""Host-side contract of bench.py (no GPU): the one-GPU refusal and the roofline peaks."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    # exits with status 2 and a message before anything touches torch or a GPU
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_point_cost_alu_peak():
    import bench

    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-slots per second over 8 + d slots per element
    slots = 256 * 4 * 16 * 2.4e9
    assert bench.points_alu_peak_gexps(2) == pytest.approx(slots / 10 / 1e9)
    assert bench.points_alu_peak_gexps(3) == pytest.approx(slots / 11 / 1e9)
    assert bench.points_alu_peak_gexps(2) == pytest.approx(3932.16)
    assert bench.HBM_PEAK_GBPS == 8000.0
