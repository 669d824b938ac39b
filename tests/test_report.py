"""The benchmark's compact result line (no GPU): bounded size, the required
keys, the full detail in its own file, and the compact line last."""
import io
import json

import pytest

from paper_2608_15764_amd import report


def _curve(base):
    ks = range(1, 17)
    return {"median_gbps": {k: base + k for k in ks}, "min_gbps": {k: base for k in ks},
            "best_gbps": {k: base + 2 * k for k in ks},
            "pct_of_best_cell": {k: 90.0 for k in ks},
            "in_flight_mib": {k: 0.5 * k for k in ks},
            "littles_law_latency_ns": {k: 500.0 for k in ks},
            "peak_K": 7, "knee_K": 2, "regime": "saturating", "decline_2_8": -0.01,
            "paired_declines_2_8": [-0.01] * 10,
            "by_order": {"asc": {"decline_2_8": -0.01, "peak_K": 7},
                         "rev": {"decline_2_8": -0.02, "peak_K": 8}}}


def full_result():
    """A result shaped like a whole benchmark run, every row included."""
    curves = {4 * w: _curve(6000.0 + w) for w in range(1, 9)}
    regime = {f"full_V{v}_w{w}": {"regime": "saturating", "peak_K": 8,
                                   "peak_gbps": 7000.0, "decline_2_8": -0.01}
              for v in (4, 8, 16) for w in range(4, 33, 4)}
    return {
        "metric": "attained HBM GB/s vs offered loads/thread K; % of HBM peak; "
                  "K=2→8 decline %",
        "value": 6635.1, "unit": "GB/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 40.78, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (SplitMix64-seeded uint32 buffer, resident in HBM)",
        "config": {"workload": "fixed-work plain-load K sweep: 1 GiB seeded u32 buffer, "
                               "16-byte loads, K=1..16, 2^26 logical loads per cell, "
                               "1..8 waves/SIMD, ascending then reversed K",
                   "buffer_bytes": 1 << 30, "vec_width": 16, "L": 1 << 26,
                   "Ks": list(range(1, 17)), "waves_per_cu": list(range(4, 33, 4)),
                   "orders": ["asc", "rev"], "cache_policy": "bypass_l1_nt",
                   "cells_per_step": 252,
                   "infeasible_cells": [{"waves_per_cu": 32, "K": 16}] * 4},
        "curve_peak_gbps": 7250.3, "curve_peak_frac_of_hbm": 0.9063,
        "best_waves_per_cu": 4, "peak_K_at_best": 8, "decline_2_8_at_best": 0.0123,
        "paper_like_cell": {"waves_per_cu": 16, "median_gbps": {2: 6900.0, 8: 6800.0},
                            "peak_K": 3, "decline_2_8": -0.0145, "regime": "saturating",
                            "by_order": {"asc": {"decline_2_8": -0.014},
                                         "rev": {"decline_2_8": -0.015}}},
        "curves": curves,
        "strict_cg": {"policy": "bypass_l1", "value": 6100.0, "ms_per_step": 44.1,
                      "curve_peak_gbps": 6800.0, "curve_peak_frac_of_hbm": 0.85,
                      "best_waves_per_cu": 8, "peak_K_at_best": 4,
                      "paper_like_decline_2_8": -0.05, "paper_like_decline_2_8_asc": -0.05,
                      "paper_like_decline_2_8_rev": -0.06,
                      "paper_like_paired_decline_median": -0.05, "curves": curves},
        "roofline": {"bound": "hbm", "achieved": 6641.2, "peak": 8000.0, "unit": "GB/s",
                     "frac": 0.8302, "traffic": 1073908535.0,
                     "kernel": "ilp::plain_kload<K,16,policy>", "launches": 5040,
                     "mean_launch_us": 161.7, "timing": "hipEvent pair per replay",
                     "algorithmic_bytes_per_launch": 1073739296},
        "gap": {"kernel_frac": 0.84, "ceiling_frac_of_peak": 0.98,
                "frac_of_ceiling": 0.857, "tail_loss": 0.12, "residual_frac": 0.974,
                "hbm_latency_ns": 360.1, "by_waves_per_cu": {w: {} for w in curves}},
        "fabric_by_xcd": {8: {"by_class": {"all": [6900.0, 6900.0]}, "masks": {}},
                          4: {"by_class": {"one": [1340.0, 1350.0], "all": [7000.0, 7000.0]},
                              "masks": {}}},
        "xcd_weighting": {4: {"gain": 0.001, "even_over_odd_share": 0.98, "rounds": []},
                          16: {"gain": 0.05, "even_over_odd_share": 1.17, "rounds": []}},
        "eager_sweep": {"step_ms": 42.0, "aggregate_gbps": 6442.0,
                        "dispatch_event_gbps": 6678.0},
        "streaming_gate": {"median_gbps": 3900.0, "median_frac": 0.4875,
                           "littles_law_ceiling_gbps": 5825.0, "frac_of_ceiling": 0.67,
                           "verdict": "latency-bound"},
        "cpu_baseline": {"value": 1.56, "unit": "GB/s", "cores": 1, "kind": "oracle",
                         "sample": "16 full cells of the sweep (K=1..16 at 4 waves/CU, "
                                   "1024 waves): per-wave sum/xor checksums of 15 GiB "
                                   "issued, NumPy, one process; buffer generation 1.7 s "
                                   "excluded",
                         "checksum_s": 10.9, "host_cpu": "AMD EPYC 9575F 64-Core Processor",
                         "matches_gpu": True,
                         "multi_process": {"value": 17.7, "cores": 16, "matches_gpu": True}},
        "rows": {
            "c5a_batched": {"batched_aggregate_gbps": 6800.0, "batched_aggregate_frac": 0.85,
                            "hbm_aggregate_gbps": 6900.0, "hbm_aggregate_frac": 0.8625,
                            "batched_best_point_gbps": 7300.0, "matches_oracle": True,
                            "points_checked": 64, "sizes": 64,
                            "points": [{"bytes": 1 << 20, "batched_gbps": 100.0}] * 64},
            "c5b_precision": {k: {"median_gbps": 7200.0, "frac_of_hbm_peak": 0.9,
                                  "abs_err": 1e-10, "rel_err": 1e-16, "within_bound": True}
                              for k in ("f32", "bf16", "fp8_e4m3")},
            "f4_regime_map": {"counts": {"saturating": 30}, "curves": regime,
                              "backends": {b: {"counts": {"saturating": 20,
                                                          "rising-censored": 4,
                                                          "peak-decline": 24},
                                               "curves": regime,
                                               "fixed_iters": {
                                                   "counts": {"saturating": 8,
                                                              "rising-censored": 10,
                                                              "peak-decline": 30},
                                                   "curves": regime}}
                                           for b in ("hbm", "infinity_cache", "l2")}},
        },
    }


def test_headline_line_fits_and_keeps_everything():
    r = full_result()
    assert len(json.dumps(r)) > 8000          # the detail alone would not fit
    line = report.headline_line(r, "results/bench_detail.json")
    assert len(line.encode()) <= report.LINE_LIMIT
    d = json.loads(line)
    for k in report.REQUIRED:
        assert k in d, k
    assert "dropped" not in d
    assert d["value"] == 6635.1 and d["ms_per_step"] == 40.78
    assert d["config"]["workload"].startswith("fixed-work plain-load K sweep")
    rl = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
              "algorithmic_bytes_per_launch", "mean_launch_us"):
        assert k in rl, k
    cb = d["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample", "host_cpu", "matches_gpu"):
        assert k in cb, k
    assert cb["multi_process"] == {"value": 17.7, "cores": 16, "matches_gpu": True}
    assert d["paper_like"]["decline_2_8"] == -0.0145
    assert d["paper_like"]["decline_2_8_rev"] == -0.015
    assert d["strict_cg"]["paper_like_decline_2_8"] == -0.05
    assert d["c5a"]["matches_oracle"] is True
    assert set(d["c5b"]) == {"f32", "bf16", "fp8_e4m3"}
    assert d["gap"]["tail_loss"] == 0.12
    assert d["fabric"] == {"one": [1340.0, 1350.0], "all": [7000.0, 7000.0]}   # lowest w
    assert d["xcd_weighting"] == {"4": [0.001, 0.98], "16": [0.05, 1.17]}   # JSON keys
    assert d["streaming_gate"]["verdict"] == "latency-bound"
    assert d["f4"] == {b: [20, 4, 24] for b in ("hbm", "infinity_cache", "l2")}
    assert d["f4_fixed_iters"] == {b: [8, 10, 30] for b in ("hbm", "infinity_cache", "l2")}
    assert d["detail"] == "results/bench_detail.json"


def test_optional_sections_give_way_to_the_limit():
    r = full_result()
    line = report.headline_line(r, "x.json", limit=1800)
    d = json.loads(line)
    assert len(line.encode()) <= 1800
    for k in report.REQUIRED:
        assert k in d, k
    assert d["dropped"] and all(k in report.OPTIONAL for k in d["dropped"])
    with pytest.raises(ValueError):
        report.headline_line(r, "x.json", limit=200)


def test_emit_writes_the_detail_and_ends_with_the_line(tmp_path):
    out = io.StringIO()
    out.write("earlier output\n")
    r = full_result()
    path = str(tmp_path / "sub" / "detail.json")
    line = report.emit(r, path, out)
    text = out.getvalue()
    assert text.endswith(line + "\n")
    assert text.splitlines()[-1] == line
    with open(path) as f:
        detail = json.load(f)
    assert detail["rows"]["f4_regime_map"]["counts"] == {"saturating": 30}
    assert json.loads(line)["detail"] == path


def test_missing_sections_are_tolerated():
    r = full_result()
    for k in ("strict_cg", "gap", "rows", "streaming_gate", "eager_sweep", "cpu_baseline"):
        del r[k]
    d = json.loads(report.headline_line(r))
    assert d["cpu_baseline"] is None and "c5a" not in d and "detail" not in d


def test_summarize_reads_a_full_result(tmp_path):
    r = full_result()
    r["fabric_by_xcd_error"] = "sweep_xcd_subset: no usable gfx950 device (-6): ..."
    text = report.summarize(r)
    assert text.splitlines()[0].startswith(r["metric"])
    assert "roofline:" in text and "gap:" in text and "batched sweep:" in text
    assert "fabric by XCD subset" in text and "fabric_by_xcd_error" in text
    p = tmp_path / "d.json"
    report.write_detail(r, str(p))
    assert report.main([str(p)]) == 0
