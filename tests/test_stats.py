"""Pins for the sweep statistics against the paper's printed numbers."""
import json
import os

import pytest

from conftest import GOLDEN
from paper_2608_15764_amd import stats


def _t1():
    with open(os.path.join(GOLDEN, "table1_decline.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("row", _t1()["rows"], ids=lambda r: r["arm"])
def test_table1_changes(row):
    # the medians are printed to 0.1 GB/s and the change to 0.1 %, so the
    # change computed from any medians that round to the printed ones must
    # round-overlap the printed change
    b2, b8, h = row["K2"], row["K8"], 0.05
    lo = 100 * stats.decline(b2 + h, b8 - h)
    hi = 100 * stats.decline(b2 - h, b8 + h)
    p = float(row["change_percent"])
    assert lo - 1e-9 <= p + 0.05 and p - 0.05 <= hi + 1e-9
    # and the point value is within one printed step
    assert abs(100 * stats.decline(b2, b8) - p) <= 0.1
    # the other plausible denominator (B8) is far off
    assert abs(100 * (b8 - b2) / b8 - p) > 10


def test_decline_sign_and_zero():
    assert stats.decline(100.0, 100.0) == 0.0
    assert stats.decline(100.0, 50.0) == -0.5
    with pytest.raises(ValueError):
        stats.decline(0.0, 1.0)


def test_medians_resist_two_anomalous_launches():
    # ten launches shaped like the Repeatability paragraph: eight agree to
    # 0.6 %, launch 9 runs up to 8 % slow, launch 10 at about half speed
    spread = [-0.002, -0.001, -0.0005, 0.0, 0.0, 0.0005, 0.001, 0.002]
    base = {1: 2200.0, 2: 3050.0, 4: 2500.0, 8: 1980.0}
    samples = {k: [b * (1 + d) for d in spread] for k, b in base.items()}
    # launch 9: slow, paired change -32.9 %; launch 10: half speed, -43.0 %
    for k in base:
        samples[k].append(base[k] * 0.92)
        samples[k].append(base[k] * 0.5)
    samples[8][8] = samples[2][8] * (1 - 0.329)
    samples[8][9] = samples[2][9] * (1 - 0.430)
    full = stats.decline(stats.median(samples[2]), stats.median(samples[8]))
    kept = {k: v[:8] for k, v in samples.items()}
    trimmed = stats.decline(stats.median(kept[2]), stats.median(kept[8]))
    lim = _t1()["repeatability"]["max_median_shift_pp"]
    assert abs(100 * (full - trimmed)) < lim
    # whereas a mean would move by far more
    mean = lambda v: sum(v) / len(v)
    md = stats.decline(mean(samples[2]), mean(samples[8]))
    assert abs(100 * (md - trimmed)) > lim


def test_peak_knee_and_regimes():
    rising = {k: float(k) for k in range(1, 9)}
    assert stats.classify(rising) == "rising-censored"
    assert stats.peak_k(rising) == 8
    flat = {1: 50.0, 2: 99.0, 3: 100.0, 4: 100.0, 5: 99.5, 6: 98.0}
    assert stats.classify(flat) == "saturating"
    assert stats.knee(flat) == 2
    peak = {1: 80.0, 2: 100.0, 3: 90.0, 4: 80.0, 5: 70.0, 6: 65.0}
    assert stats.classify(peak) == "peak-decline"
    assert stats.peak_k(peak) == 2
    tie = {1: 1.0, 2: 5.0, 3: 5.0, 4: 1.0}
    assert stats.peak_k(tie) == 2


def test_residency_screen():
    big = 1 << 30
    assert stats.residency_flag(8500.0, big)
    assert not stats.residency_flag(7000.0, big)
    assert not stats.residency_flag(20000.0, 64 << 20)   # cache-resident cell


def test_littles_law():
    # the paper's H100 figures: 3,350 GB/s x 353 ns ~ 1.18 MB in flight
    assert abs(3350 * 353 - 1.18e6) / 1.18e6 < 0.01
    fl = stats.in_flight_bytes(n_waves=1024, K=2, vec_bytes=16)
    assert fl == 1024 * 64 * 2 * 16
    assert stats.implied_latency_ns(fl, 2097.152) == pytest.approx(1000.0)


def test_summary_curve():
    s = {1: [1.0, 1.1], 2: [3.0, 3.2], 4: [2.5, 2.4], 8: [2.0, 2.1]}
    out = stats.summarize_curve(s)
    assert out["peak_K"] == 2
    assert out["decline_2_8"] == pytest.approx((2.05 - 3.1) / 3.1)
    assert len(out["paired_declines_2_8"]) == 2


def test_anomalous_launches_are_disclosed():
    # ten launches per cell, one at half speed and one 8 % slow (the shape of
    # the two disclosed primary launches); only the first crosses the 10 % rule
    s = {2: [100.0] * 8 + [50.0, 92.0], 8: [80.0] * 10}
    a = stats.anomalous_launches(s)
    assert a == [(2, 50.0, 0.5)]
    c = stats.summarize_curve(s)
    assert c["launches"] == 20 and c["anomalous"] == [(2, 50.0, 0.5)]
    assert c["median_gbps"][2] == 100.0            # medians are insensitive
    assert stats.anomalous_launches({4: [10.0, 10.0, 8.0]}, frac=0.85) == [(4, 8.0, 0.8)]


def test_front_duplicates_closed_forms():
    # round robin: the front of one iteration is contiguous, n_waves groups;
    # no sharing while it fits the allocation
    assert stats.front_duplicates(0, 2, 8, 64, 64 * 2 * 16) == 0.0
    # blocked over 4 passes: wave w reads groups 4w..4w+3 of a 4-group
    # allocation, so in every iteration all four waves read the same group
    assert stats.front_duplicates(1, 1, 4, 16, 64 * 4) == 0.75
    # round robin with a front of 8 groups over a 4-group allocation: each
    # segment is read twice per iteration
    assert stats.front_duplicates(0, 1, 8, 64, 64 * 4) == 0.5
    # strided, Q a multiple of the allocation's 16 segments: the K loads of
    # a group all read segment q mod 16, so K - 1 of every K repeat
    for K in (1, 2, 4, 8):
        assert stats.front_duplicates(2, K, 4, 64, 64 * 16) == (K - 1) / K
    # strided without a wrap (K Q segments in the allocation): all distinct
    assert stats.front_duplicates(2, 4, 8, 64, 64 * 4 * 64) == 0.0
    # strided, Q = S / 2: loads j and j + 2 of a group meet
    assert stats.front_duplicates(2, 4, 2, 8, 64 * 16) == 0.5
    with pytest.raises(ValueError):
        stats.front_duplicates(3, 1, 1, 1, 64)


def _front_brute(order, K, nw, Q, nv):
    from oracle import checksums, plan as oplan
    lists = [list(oplan.groups_of_wave(w, Q, nw, order)) for w in range(nw)]
    n_it = max(len(x) for x in lists)
    total = dup = 0
    for i in range(n_it):
        segs = [checksums.vector_index(x[i], j, 0, K, nv, Q=Q, order=order) // 64
                for x in lists if i < len(x) for j in range(K)]
        total += len(segs)
        dup += len(segs) - len(set(segs))
    return dup / total


@pytest.mark.parametrize("order", [0, 1, 2])
def test_front_duplicates_matches_brute_force(order):
    """Against the oracle's own owners and vector map, load by load."""
    for K, nw, Q, nv in [(3, 5, 47, 64 * 3 * 4), (2, 6, 100, 64 * 2 * 10),
                         (1, 16, 40, 64 * 7), (4, 3, 20, 64 * 16), (3, 4, 9, 64 * 5)]:
        assert stats.front_duplicates(order, K, nw, Q, nv, max_iters=10**6) == \
            pytest.approx(_front_brute(order, K, nw, Q, nv), abs=0), (order, K, nw, Q, nv)


def test_idle_slots():
    # every wave runs the whole window: nothing idle
    assert stats.idle_slots([0, 0, 0, 0], [100, 100, 100, 100]) == 0.0
    # three of four waves stop at half time: 3 x 50 idle of 4 x 100
    assert abs(stats.idle_slots([0, 0, 0, 0], [50, 50, 50, 100]) - 150 / 400) < 1e-12
    assert stats.idle_slots([], []) == 0.0


def test_active_ceiling():
    """Four waves of 1 MiB in flight each, latency 1000 ns (1 MiB / 1000 ns
    = 1048.576 GB/s per wave).  All running all the time: the design
    ceiling.  Three stopping at half time: half the window at 4 waves'
    rate, half at one wave's."""
    mib = float(1 << 20)
    per = mib / 1000.0
    full = stats.active_ceiling_gbps([0] * 4, [100] * 4, mib, 1000.0)
    assert abs(full - 4 * per) < 1e-9
    tail = stats.active_ceiling_gbps([0] * 4, [50, 50, 50, 100], mib, 1000.0)
    assert abs(tail - (0.5 * 4 * per + 0.5 * per)) < 1e-9
    # the datasheet caps every moment: a large offer loses nothing to the tail
    # until too few waves remain to cover the bandwidth-delay product
    capped = stats.active_ceiling_gbps([0] * 4, [50, 50, 50, 100], 64 * mib, 1000.0)
    assert capped == stats.HBM_PEAK_GBPS
    # a late start counts from the first start
    late = stats.active_ceiling_gbps([0, 0, 0, 50], [100] * 4, mib, 1000.0)
    assert abs(late - (0.5 * 3 * per + 0.5 * 4 * per)) < 1e-9
    assert stats.active_ceiling_gbps([], [], mib, 1000.0) == 0.0


def test_littles_ceiling():
    assert stats.littles_ceiling_gbps(2 << 20, 360.0) == (2 << 20) / 360.0
    assert stats.littles_ceiling_gbps(64 << 20, 360.0) == stats.HBM_PEAK_GBPS
    with pytest.raises(ValueError):
        stats.littles_ceiling_gbps(1, 0.0)


def test_gap_split_factors_multiply_to_the_kernel_fraction():
    cells = [{"bytes": 1e9, "gbps": 2000.0, "ceiling_gbps": 2900.0,
              "active_ceiling_gbps": 2700.0},
             {"bytes": 1e9, "gbps": 7000.0, "ceiling_gbps": 8000.0,
              "active_ceiling_gbps": 8000.0},
             {"bytes": 2e9, "gbps": 6800.0, "ceiling_gbps": 8000.0,
              "active_ceiling_gbps": 7600.0}]
    g = stats.gap_split(cells)
    t_meas = 1e9 / 2000 + 1e9 / 7000 + 2e9 / 6800
    assert abs(g["kernel_frac"] - (4e9 / 8000) / t_meas) < 1e-12
    prod = g["ceiling_frac_of_peak"] * (1 - g["tail_loss"]) * g["residual_frac"]
    assert abs(prod - g["kernel_frac"]) < 1e-12
    t_ceil = 1e9 / 2900 + 1e9 / 8000 + 2e9 / 8000
    t_act = 1e9 / 2700 + 1e9 / 8000 + 2e9 / 7600
    assert abs(g["tail_loss"] - (1 - t_ceil / t_act)) < 1e-12
    assert abs(g["residual_frac"] - t_act / t_meas) < 1e-12
    # every cell at its ceiling with no tail: only the design factor is left
    flat = [dict(c, gbps=c["ceiling_gbps"], active_ceiling_gbps=c["ceiling_gbps"])
            for c in cells]
    g = stats.gap_split(flat)
    assert abs(g["residual_frac"] - 1) < 1e-12 and abs(g["tail_loss"]) < 1e-12
    assert abs(g["kernel_frac"] - g["ceiling_frac_of_peak"]) < 1e-12
    with pytest.raises(ValueError):
        stats.gap_split([])


def test_front_duplicates_random_cells():
    """The same brute force over random small cells of every order."""
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=120, deadline=None, derandomize=not os.environ.get("ILPSWEEP_HYPOTHESIS_RANDOM"))
    @given(order=st.integers(0, 2), K=st.integers(1, 6), nw=st.integers(1, 12),
           Q=st.integers(1, 60), segs=st.integers(1, 40))
    def check(order, K, nw, Q, segs):
        nv = 64 * segs
        assert stats.front_duplicates(order, K, nw, Q, nv, max_iters=10**6) == \
            pytest.approx(_front_brute(order, K, nw, Q, nv), abs=0), (order, K, nw, Q, nv)

    check()
