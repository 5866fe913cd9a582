"""Host-side checks of bench.py's reporting (no GPU): the per-variant error
against the FP64 run of the same workload and window."""
import pytest

import bench


def _run(v, a, steps=100, us=1.0):
    return {"cell_steps_per_s": 1.0, "us_per_step": us, "achieved_GBs": 1.0, "avg_launch_us": us,
            "kernel": "k", "tuning": {}, "window_steps": steps, "v_avg": v, "absorption": a}


def test_variant_errors_against_the_fp64_run_of_the_same_workload():
    main = _run(0.5, 0.2)
    variants = {
        "large_fp32": _run(0.5 * (1 + 1e-8), 0.2 + 3e-9),
        "large_fp64_fused2": _run(0.5, 0.2),
        "crossed_fp64": _run(0.1, 0.01, steps=200),
        "crossed_fp32": _run(0.1 * (1 - 2e-8), 0.01 - 1e-9, steps=200),
        "other_fp32": _run(1.0, 1.0),                      # no FP64 run of its workload
        "large_fp64_window": _run(0.5, 0.2, steps=50),     # different window: not compared
    }
    rep = bench.variant_report(main, variants, "large", 0)
    assert rep["large_fp32"]["vs_fp64"]["rel_v_avg"] == pytest.approx(1e-8, rel=1e-6)
    assert rep["large_fp32"]["vs_fp64"]["abs_absorption"] == pytest.approx(3e-9, rel=1e-6)
    assert rep["large_fp64_fused2"]["vs_fp64"] == {"rel_v_avg": 0.0, "abs_absorption": 0.0}
    assert "vs_fp64" not in rep["crossed_fp64"]                # the reference itself
    assert rep["crossed_fp32"]["vs_fp64"]["rel_v_avg"] == pytest.approx(2e-8, rel=1e-6)
    assert "vs_fp64" not in rep["other_fp32"]
    assert "vs_fp64" not in rep["large_fp64_window"]
    assert rep["crossed_fp32"]["window"] == {"steps": 200, "v_avg": 0.1 * (1 - 2e-8),
                                             "absorption": 0.01 - 1e-9}


def test_fp32_main_run_compares_against_the_fp64_variant():
    main = _run(0.5 * (1 + 4e-8), 0.2)                          # FP32 main run
    variants = {"large_fp64": _run(0.5, 0.2), "large_fp32_fused3": _run(0.5 * (1 + 4e-8), 0.2)}
    rep = bench.variant_report(main, variants, "large", 1)
    assert "vs_fp64" not in rep["large_fp64"]
    assert rep["large_fp32_fused3"]["vs_fp64"]["rel_v_avg"] == pytest.approx(4e-8, rel=1e-6)
