"""The FP32 form's error against the FP64 form, stated per observable as the
precision criteria require (mean energy per spin within 1e-4 absolute and
within 3 standard errors at every temperature; P(q) no farther from the FP64
runs of other seeds than an FP64 run is, within 3 standard errors), on a
reduced run of the L=8
workload's shape.  The FP64 form is bit-identical to the FP64 oracle (the
parity tests), so this compares the FP32 form with the oracle's statistics.
Both forms use counter-based random numbers, so the run and its verdict are
reproducible bit for bit."""
from __future__ import annotations

import sys

import pytest

from paper_2605_25872_amd import analysis, inputs

pytestmark = pytest.mark.gpu


def test_fp32_form_within_the_stated_tolerances_l8():
    w = inputs.WORKLOADS["l8_fp64"]
    print("[gpu-precision] L=8, 512 samples, 1536 EMCS, 4 seeds per form", file=sys.stderr, flush=True)
    res = analysis.compare_precisions(w, 512, 1536, [1, 2, 3, 4],
                                      progress=lambda m: print(f"[gpu-precision] {m}", file=sys.stderr, flush=True))
    assert res["e_within_tolerance"], (res["max_abs_e_diff"], res["e_diff_fp32_minus_fp64"])
    assert res["e_within_n_sigma"], (res["max_abs_z"], res["e_diff_fp32_minus_fp64"], res["e_diff_sigma"])
    assert res["pq_within_fp64_spread"], (res["pq_tv_gap"], res["pq_tv_gap_se"], res["pq_tv_mean_over_T"])
