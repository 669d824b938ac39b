"""Line coverage of a cell: the oracle's walk of the address map against a
lane-by-lane brute force, the paper's printed bound, and the product's
closed form against the oracle (no GPU)."""
import os

import pytest

from oracle import coverage, plan
from paper_2608_15764_amd import stats


TINY = [  # (alloc bytes, V, K, Q, n_waves)
    (64 * 16 * 8, 16, 3, 7, 2),      # wraps, K does not divide the segments
    (64 * 4 * 6, 4, 4, 5, 3),        # 4-byte vectors: two lines per segment
    (64 * 8 * 5, 8, 7, 2, 4),        # K larger than the segment count
    (64 * 16 * 16, 16, 2, 3, 2),     # less than one pass
    (64 * 16 * 4, 16, 1, 4, 4),      # exactly one pass
]


@pytest.mark.parametrize("order", [plan.ROUND_ROBIN, plan.BLOCKED, plan.STRIDED])
@pytest.mark.parametrize("alloc,V,K,Q,n_waves", TINY)
def test_walk_matches_lane_brute_force(alloc, V, K, Q, n_waves, order):
    brute = coverage.lane_line_reads(alloc, V, K, Q, n_waves, order)
    seg = coverage.segment_reads(alloc, V, K, Q, n_waves, order)
    lines = [int(c) for c in seg for _ in range(64 * V // 128)]
    assert lines == brute
    c = coverage.line_coverage(alloc, V, K, Q, n_waves, order)
    assert c["unique_lines"] == sum(1 for x in brute if x)
    assert c["line_reads"] == sum(brute) and c["max_reads"] == max(brute)
    # every load reads 64 V bytes, i.e. V/2 lines
    assert c["line_reads"] == 64 * K * Q * V // 128


def test_paper_bound_for_the_largest_allocation():
    """16,785 MiB issued over a 20,000 MiB allocation (Section 4.2): the
    walk finds unique coverage 16,785 / 20,000 = 0.839..., within the
    paper's 'at most 84 %', and no line read twice."""
    MiB = 1 << 20
    alloc, V, K = 20000 * MiB, 16, 8
    Q = 16785 * MiB // (64 * K * V)
    assert 64 * K * V * Q == 16785 * MiB
    c = coverage.line_coverage(alloc, V, K, Q, 64, plan.ROUND_ROBIN)
    assert c["coverage"] == 16785 / 20000 and c["coverage"] <= 0.84
    assert c["re_reads"] == 0 and c["max_reads"] == 1
    # the 512 MiB allocation takes the same volume about 33 times over
    small = coverage.line_coverage(512 * MiB, V, K, Q, 64, plan.ROUND_ROBIN)
    assert small["coverage"] == 1.0 and small["max_reads"] == 33


@pytest.mark.parametrize("order", [plan.ROUND_ROBIN, plan.BLOCKED, plan.STRIDED])
@pytest.mark.parametrize("alloc,V,K,L,n_waves", [
    (1 << 20, 16, 3, 1 << 17, 96), (1 << 20, 4, 5, 1 << 20, 64),
    (2 << 20, 8, 16, 1 << 16, 256), (3 << 20, 16, 7, 1 << 20, 1024),
    (1 << 22, 16, 1, 1 << 18, 512)])
def test_product_closed_form_matches_the_walk(alloc, V, K, L, n_waves, order):
    Q = L // (64 * K)
    want = coverage.line_coverage(alloc, V, K, Q, n_waves, order)
    got = stats.line_coverage(alloc, V, 64 * K * Q)
    assert got == want


def test_walk_and_closed_form_on_random_cells():
    """The walk against the lane brute force, and the product's closed
    form against the walk, over random small cells of every order."""
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=150, deadline=None, derandomize=not os.environ.get("ILPSWEEP_HYPOTHESIS_RANDOM"))
    @given(order=st.sampled_from([plan.ROUND_ROBIN, plan.BLOCKED, plan.STRIDED]),
           V=st.sampled_from([4, 8, 16]), K=st.integers(1, 9), Q=st.integers(1, 30),
           n_waves=st.integers(1, 9), segs=st.integers(1, 24))
    def check(order, V, K, Q, n_waves, segs):
        alloc = 64 * V * segs
        brute = coverage.lane_line_reads(alloc, V, K, Q, n_waves, order)
        c = coverage.line_coverage(alloc, V, K, Q, n_waves, order)
        assert c["unique_lines"] == sum(1 for x in brute if x)
        assert c["line_reads"] == sum(brute) and c["max_reads"] == max(brute)
        assert stats.line_coverage(alloc, V, 64 * K * Q) == c

    check()
