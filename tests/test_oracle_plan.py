"""Pins for the fixed-work control (Section 3; Section 4.2)."""
import json
import os

import pytest

from conftest import GOLDEN
from oracle import plan


def _fw():
    with open(os.path.join(GOLDEN, "fixed_work.json")) as f:
        return json.load(f)


def _threads(cell):
    return cell["ctas"] * cell["warps_per_cta"] * cell["threads_per_warp"]


def test_paper_mismatch_is_reproduced():
    g = _fw()
    T = _threads(g["primary_cell"])
    issued = [plan.per_thread_floor(g["L"], T, K)["issued"] for K in g["K_set"]]
    pct = 100 * plan.kset_mismatch(issued)
    assert f"{pct:.6f}" == g["printed"]["max_mismatch_percent"]
    # the printed bound "<= 0.0246 %" holds
    assert pct <= 0.0246


def test_half_cell_has_the_same_mismatch():
    g = _fw()
    c = dict(g["half_cell"])
    c["threads_per_warp"] = 32
    T = _threads(c)
    issued = [plan.per_thread_floor(g["L"], T, K)["issued"] for K in g["K_set"]]
    assert f"{100 * plan.kset_mismatch(issued):.6f}" == g["printed"]["max_mismatch_percent"]


def test_issued_volume_and_ratios():
    g = _fw()
    T = _threads(g["primary_cell"])
    V = g["primary_cell"]["vector_bytes"]
    vol = max(plan.per_thread_floor(g["L"], T, K)["issued"] for K in g["K_set"]) * V
    mib = vol / 2**20
    assert round(mib) == g["printed"]["issued_volume_MiB"]
    assert f"{vol / 1e9:.1f}" == g["printed"]["issued_volume_GB"]
    # printed ratios use the rounded MiB figure over 512 MiB and 20,000 MiB
    assert f"{round(mib) / 512:.0f}" == g["printed"]["volume_to_allocation_512MiB"]
    assert f"{round(mib) / 20000:.2f}" == g["printed"]["volume_to_allocation_20000MiB"]
    assert f"{100 * round(mib) / 20000:.0f}" == g["printed"]["unique_coverage_bound_percent_20000MiB"]


@pytest.mark.parametrize("K", range(1, 17))
@pytest.mark.parametrize("n_waves", [1, 7, 1024, 8192])
def test_wave_group_plan_by_enumeration(K, n_waves):
    L = 2**26 + 12345
    p = plan.wave_group(L, K, n_waves)
    # brute-force: deal groups one by one
    count = [0] * n_waves
    q = 0
    while (q + 1) * 64 * K <= L:
        count[q % n_waves] += 1
        q += 1
    assert p["Q"] == q
    assert p["iters"] == count
    assert p["issued"] == 64 * K * q <= L
    assert p["iters_max"] - p["iters_min"] <= 1


def test_wave_group_meets_the_paper_bound_for_K_1_to_16():
    L = 2**26
    issued = [plan.wave_group(L, K, 8192)["issued"] for K in range(1, 17)]
    m = plan.kset_mismatch(issued)
    assert m <= 0.0246 / 100
    # the worst K is 13 and the figure is about 0.00086 %
    assert abs(100 * m - 0.000858) < 5e-6
    # power-of-two K issue exactly one full pass of 2**26 loads
    for K in (1, 2, 4, 8, 16):
        assert plan.wave_group(L, K, 8192)["issued"] == L


def test_per_thread_floor_cannot_meet_the_bound_at_2_26():
    # why the library does not use the paper's per-thread floor for K=1..16
    L = 2**26
    for w in (1, 4, 8):
        T = 256 * 4 * w * 64
        issued = [plan.per_thread_floor(L, T, K)["issued"] for K in range(1, 17)]
        assert plan.kset_mismatch(issued) > 0.0246 / 100


def test_fixed_iters_grows_with_K():
    a = plan.fixed_iters(10, 2, 100)["issued"]
    b = plan.fixed_iters(10, 8, 100)["issued"]
    assert b == 4 * a
