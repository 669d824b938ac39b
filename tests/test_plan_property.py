"""The C planner against the oracle's fixed-work accounting on random
inputs (hypothesis): every mode, every address order, full and explicit
grids, sizes from one vector segment to 2**40 loads.  Host only."""
import os

import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st

from oracle import plan as oplan

WAVE = 64
# a fixed example sequence, so that a run of the suite is reproducible;
# set ILPSWEEP_HYPOTHESIS_RANDOM=1 to draw fresh examples
DERANDOMIZE = not os.environ.get("ILPSWEEP_HYPOTHESIS_RANDOM")


@pytest.fixture(scope="module")
def isw():
    from paper_2608_15764_amd import ilpsweep
    return ilpsweep


def _want(mode, order, K, n_waves, L, iters):
    if mode == 0:
        Q = L // (WAVE * K)
    elif mode == 1:
        Q = n_waves * iters
    else:
        Q = n_waves * (L // (n_waves * WAVE * K))
    per_wave = [len(oplan.groups_of_wave(w, Q, n_waves, order)) for w in range(n_waves)]
    return Q, per_wave


@settings(max_examples=300, deadline=None, derandomize=DERANDOMIZE)
@given(V=st.sampled_from([4, 8, 16]), K=st.integers(1, 16),
       w=st.sampled_from([4, 8, 12, 16, 20, 24, 28, 32]),
       cus=st.integers(1, 256), grid=st.one_of(st.just(0), st.integers(1, 2048)),
       segs=st.integers(1, 1 << 22), L=st.integers(1, 1 << 40),
       mode=st.integers(0, 2), order=st.integers(0, 2), iters=st.integers(1, 5000))
def test_planner_matches_oracle(isw, V, K, w, cus, grid, segs, L, mode, order, iters):
    nbytes = segs * WAVE * V
    n_waves = (grid or cus * w // 4) * 4
    Q, per_wave = _want(mode, order, K, n_waves, L, iters)
    args = dict(mode=mode, fixed_iters=iters if mode == 1 else 0, num_cus=cus,
                grid_wgs=grid, order=order)
    if Q == 0 or max(per_wave) > 2**32 - 1:
        # no work, or a per-wave iteration count beyond the 32-bit fields
        with pytest.raises(isw.SweepError) as e:
            isw.sweep_plan(nbytes, K, V, w, L, **args)
        assert e.value.code == isw.EINVAL
        return
    p = isw.sweep_plan(nbytes, K, V, w, L, **args)
    assert p["waves"] == n_waves and p["wg_threads"] == 256
    assert p["n_vec"] == nbytes // V
    assert p["Q"] == Q and p["issued_loads"] == WAVE * K * Q
    assert p["issued_bytes"] == V * WAVE * K * Q
    assert (p["iters_min"], p["iters_max"]) == (min(per_wave), max(per_wave))
    if mode == 1:
        assert p["mismatch"] == 0.0
    else:
        assert p["mismatch"] == pytest.approx(oplan.target_mismatch(L, WAVE * K * Q),
                                              rel=1e-12, abs=1e-15)


def test_planner_rejects_more_than_32_bit_iterations(isw):
    """2^40 - 64 loads of 4 bytes at K = 1 on one CU of 4 waves: each wave
    would run 2^32 iterations, which the 32-bit counts cannot report."""
    with pytest.raises(isw.SweepError) as e:
        isw.sweep_plan(64 * 4, 1, 4, 4, (1 << 40) - 64, num_cus=1)
    assert e.value.code == isw.EINVAL
    p = isw.sweep_plan(64 * 4, 1, 4, 4, (1 << 40) - 64 - 4 * 64, num_cus=1)
    assert p["iters_max"] == 2**32 - 1
