"""Pins for the streaming sum's error bound (``oracle.fpsum.sum2_bound``)
through a binary32 model of the whole accumulation scheme: per-lane Sum2,
the depth-8 merge tree of a workgroup and the binary64 final combine.

Each of the bound's three terms is pinned on its own: adversarial inputs
stay within the whole bound; an input whose error only the merge-tree term
can cover exceeds the bound without it; an input whose error comes from
the final combine alone reaches most of that term.  A plain binary32 sum in
the same layout exceeds the bound on the absorbed-terms inputs, so the
tolerance the GPU tests use can tell compensated from uncompensated
summation."""
from fractions import Fraction

import numpy as np
import pytest

import fp_scheme as fs
from oracle import fpsum

f32 = np.float32


def _exact(lane_terms):
    flat = np.concatenate([np.asarray(t, dtype=np.float32) for wg in lane_terms
                           for t in wg]).astype(np.float64)
    return fpsum.exact_sum_rational(flat), float(np.abs(flat).sum())


def _family(name, n_wg, n_lane, seed):
    rng = np.random.default_rng(seed)
    wgs = []
    for _ in range(n_wg):
        lanes = []
        for _ in range(256):
            if name == "absorbed":
                # a large leading term, then ones that a binary32 running sum
                # of that size cannot hold, then the large term taken back
                t = [2.0**30] + [1.0] * (n_lane - 2) + [-(2.0**30)]
            elif name == "heavy_leading":
                big = np.ldexp(1.0 + rng.random(), int(rng.integers(24, 40)))
                small = np.ldexp(rng.random(n_lane - 1) + 1.0,
                                 rng.integers(-10, 8, n_lane - 1))
                t = [big * rng.choice([-1, 1])] + list(small)
            elif name == "wide":
                t = np.ldexp(1.0 + rng.random(n_lane), rng.integers(-60, 60, n_lane)) \
                    * rng.choice([-1, 1], n_lane)
            elif name == "cancelling":
                x = np.ldexp(1.0 + rng.random(n_lane // 2), rng.integers(0, 30, n_lane // 2))
                y = -(x * (1.0 - np.ldexp(rng.random(n_lane // 2), -20)))
                t = np.empty(2 * (n_lane // 2))
                t[0::2], t[1::2] = x, y
            elif name == "normal":
                t = rng.standard_normal(n_lane)
            else:
                raise ValueError(name)
            lanes.append(np.asarray(t, dtype=np.float32))
        wgs.append(lanes)
    return wgs


@pytest.mark.parametrize("name", ["absorbed", "heavy_leading", "wide", "cancelling",
                                  "normal"])
def test_scheme_error_within_the_whole_bound(name):
    n_wg, n_lane = 3, 16
    lanes = _family(name, n_wg, n_lane, seed=len(name))
    exact, abs_sum = _exact(lanes)
    got = fs.scheme(lanes)
    err = abs(Fraction(got) - exact)
    assert float(err) <= fpsum.sum2_bound(abs_sum, n_lane, 8, n_wg)


@pytest.mark.parametrize("name", ["absorbed", "heavy_leading"])
def test_plain_fp32_in_the_same_layout_breaks_the_bound(name):
    n_wg, n_lane = 3, 16
    lanes = _family(name, n_wg, n_lane, seed=len(name))
    exact, abs_sum = _exact(lanes)
    plain = fs.scheme(lanes, compensated=False)
    err = abs(Fraction(plain) - exact)
    assert float(err) > 100 * fpsum.sum2_bound(abs_sum, n_lane, 8, n_wg)


def _tree_adversary(k=40):
    """One term per lane, so every lane is exact.  In each quad of lanes,
    lanes 0 and 2 hold 2**k and lanes 1 and 3 small terms B1 and B2 below
    half a unit of 2**k: the first merge level keeps them whole as c parts
    (exact TwoSum errors), and the second adds B1 + B2 in binary32, where B2
    is laid out to lose just under half a unit of B1's last place.  Every
    later merge adds two equal pairs, which is exact."""
    B1 = f32(np.ldexp(2**23 + 1, k - 48))
    N = 2**23 + 2**11 - 1                  # low 12 bits just under half of 2**12
    B2 = f32(np.ldexp(N, k - 60))
    A = f32(np.ldexp(1.0, k))
    assert float(B1) < 2.0 ** (k - 24) and float(B2) < 2.0 ** (k - 24)
    quad = [A, B1, A, B2]
    return [[np.array([quad[i % 4]], dtype=np.float32) for i in range(256)]], k


def test_merge_tree_term_is_exercised():
    lanes, k = _tree_adversary()
    exact, abs_sum = _exact(lanes)
    got = fs.scheme(lanes)
    err = abs(Fraction(got) - exact)
    # 64 quads, each losing (2**11 - 1) * 2**(k - 60) in the second level
    assert err == 64 * (2**11 - 1) * Fraction(2) ** (k - 60)
    without_tree = fpsum.sum2_bound(abs_sum, 1, 0, 1)
    assert float(err) > 2 * without_tree
    assert float(err) <= fpsum.sum2_bound(abs_sum, 1, 8, 1)


def test_final_combine_term_is_pinned():
    """Pairs straight into the binary64 combine (no lanes, no tree): each of
    the 256 threads first takes 1.0, then m - 1 terms of 2**-53, each a tie
    that rounds back to 1.0.  The loss is (m - 1) units of 2**-53 per
    thread, close to the bound's final term for chains of m."""
    m = 64
    pairs = [(f32(1.0), f32(0.0))] * 256 + [(f32(2.0**-53), f32(0.0))] * (256 * (m - 1))
    got = fs.final_combine(pairs)
    exact = Fraction(256) + 256 * (m - 1) * Fraction(2) ** -53
    err = abs(Fraction(got) - exact)
    assert err == 256 * (m - 1) * Fraction(2) ** -53
    abs_sum = float(exact)
    bound = fpsum.sum2_bound(abs_sum, 1, 0, len(pairs))
    assert 0.8 * bound <= float(err) <= bound


def test_bound_terms_vanish_where_the_scheme_is_exact():
    # one term per lane, no merges, one group: only the binary64 roundings
    b = fpsum.sum2_bound(1.0, 1, 0, 1)
    assert b == fpsum.U64 + fpsum.gamma(2, fpsum.U64) * 1.001
    # no groups at all: the rounding of the reference only
    assert fpsum.sum2_bound(1.0, 0, 0, 0) == fpsum.U64
    # more terms per lane, deeper trees and more groups only loosen it
    assert fpsum.sum2_bound(1.0, 2, 0, 1) > b
    assert fpsum.sum2_bound(1.0, 1, 1, 1) > b
    assert fpsum.sum2_bound(1.0, 1, 0, 257) > b


def test_lane_term_is_reached_within_a_factor_of_four():
    """One lane of three terms: 2**(p+24), then 2**p (a tie that leaves the
    running sum unchanged, so c takes it whole), then a term whose binary32
    sum with c loses just under half a unit of c's last place.  The error is
    about a quarter of gamma_2**2 sum|x|."""
    p = -30
    A = f32(np.ldexp(1.0, p + 24))
    beta = f32(np.ldexp(1.0, p))
    N = 2**23 + 2**11 - 1
    b2 = f32(np.ldexp(N, p - 35))
    s, c = fs.lane_sum2([A, beta, b2])
    exact = Fraction(float(A)) + Fraction(float(beta)) + Fraction(float(b2))
    err = abs(Fraction(float(s)) + Fraction(float(c)) - exact)
    abs_sum = float(A) + float(beta) + float(b2)
    lane_term = fpsum.gamma(2) ** 2 * abs_sum
    assert err == (2**11 - 1) * Fraction(2) ** (p - 35)
    assert 0.2 * lane_term <= float(err) <= fpsum.sum2_bound(abs_sum, 3, 0, 0)
