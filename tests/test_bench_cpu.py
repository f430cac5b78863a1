"""Host logic of the benchmark: the issue-limited VALU peak, the counter-based
figures it reports only for the kernel sources they were taken on, and the
one-GPU guard.  No GPU needed."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("update,precision,n2,n4", [("metropolis", "fp32", 23, 13), ("metropolis", "fp64", 17, 40),
                                                     ("heatbath", "fp32", 21, 20), ("heatbath", "fp64", 7, 56)])
def test_valu_peak_is_the_issue_limited_rate(update, precision, n2, n4):
    # 256 CUs x 4 SIMDs x 2.4 GHz; a 2-cycle wave64 instruction gives 32 lane
    # operations per SIMD-cycle, a 4-cycle one 16
    simd_cycles_per_s = 256 * 4 * 2.4e9
    seconds_per_attempt = n2 / (32 * simd_cycles_per_s) + n4 / (16 * simd_cycles_per_s)
    peak, ops = bench.valu_peak(update, precision)
    assert ops == n2 + n4
    assert peak == pytest.approx((n2 + n4) / seconds_per_attempt, rel=1e-12)
    # between the all-4-cycle and the all-2-cycle rates
    assert 16 * simd_cycles_per_s < peak < 32 * simd_cycles_per_s


def test_counter_figures_only_for_their_workload_and_sources():
    assert bench.sweep_traffic_bytes("l8_fp64") is None
    assert bench.houdayer_utilisation("l16_fp32", "single") is None
    assert bench.houdayer_utilisation("l12_fp32", "acu") is None
    traffic = bench.sweep_traffic_bytes("l16_fp32")
    if bench.kernel_sources_sha256() != bench.SWEEP_TRAFFIC["sources_sha256"]:
        assert traffic is None
        return
    # algorithmic bytes of one sweep launch at L=16: 1024 samples, 4096 sites,
    # 6 spin words per site read and written, 3 float couplings per site,
    # 160 float clone factors per sample
    S, V = 1024, 4096
    algorithmic = S * (2 * 6 * V * 4 + 3 * V * 4 + 160 * 4)
    assert algorithmic <= traffic <= 1.02 * algorithmic
    u = bench.houdayer_utilisation("l16_fp32", "acu")
    assert 0.0 < u["valu_issue"] < 1.0 and 0.0 < u["lds_pipe_busy"] < 1.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
