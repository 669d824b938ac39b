"""Pins for the oracle's address map and checksum sinks."""
import itertools
import os

import numpy as np
import pytest

from oracle import brute, checksums, plan, splitmix


def _buf(nbytes, seed=11):
    return splitmix.buffer_words(seed, nbytes)


CASES = [
    # V, K, Q, n_waves, buffer bytes (n_vec * V); includes wrap-around
    (4, 1, 5, 2, 4 * 64 * 4),
    (4, 3, 7, 3, 4 * 64 * 5),       # ragged: Q not a multiple of n_waves
    (8, 2, 6, 4, 8 * 64 * 3),       # issued 768 vectors over 192: 4 passes
    (16, 5, 3, 2, 16 * 64 * 7),     # 960 of 448 vectors: wraps mid-group
    (16, 16, 2, 1, 16 * 64 * 4),
    (16, 1, 9, 4, 16 * 64 * 64),    # less than one pass
    (8, 7, 4, 3, 8 * 64 * 2),       # group larger than the buffer
]


@pytest.mark.parametrize("V,K,Q,nw,nbytes", CASES)
def test_vectorised_lanes_match_brute_force(V, K, Q, nw, nbytes):
    w = _buf(nbytes)
    lanes = brute.simulate(w, V, K, Q, nw)
    s, x = checksums.per_lane(w, V, K, Q, nw)
    for (wave, lane), (ls, lx) in lanes.items():
        assert s[wave, lane] == ls and x[wave, lane] == lx


@pytest.mark.parametrize("V,K,Q,nw,nbytes", CASES)
def test_vectorised_waves_match_brute_force(V, K, Q, nw, nbytes):
    w = _buf(nbytes, seed=12)
    bs, bx = brute.per_wave(brute.simulate(w, V, K, Q, nw), nw)
    s, x = checksums.per_wave(w, V, K, Q, nw, chunk_groups=2)
    assert s.tolist() == bs and x.tolist() == bx


@pytest.mark.parametrize("V,K,Q,nw,nbytes", CASES)
def test_seeded_single_wave_and_lane(V, K, Q, nw, nbytes):
    seed = 12345
    w = _buf(nbytes, seed=seed)
    s, x = checksums.per_wave(w, V, K, Q, nw)
    ls, lx = checksums.per_lane(w, V, K, Q, nw)
    for wave in range(nw):
        assert checksums.wave_from_seed(seed, V, K, Q, nw, wave,
                                        buffer_bytes=nbytes) == (s[wave], x[wave])
        for lane in (0, 17, 63):
            assert checksums.lane_from_seed(seed, V, K, Q, nw, wave, lane,
                                            nbytes // V) == (ls[wave, lane], lx[wave, lane])


def test_region_offset_matches_brute_force():
    V, K, Q, nw = 16, 3, 5, 2
    w = _buf(16 * 64 * 8)
    base, n_vec = 192, 128
    lanes = brute.simulate(w, V, K, Q, nw, base=base, n_vec=n_vec)
    s, x = checksums.per_lane(w, V, K, Q, nw, base=base, n_vec=n_vec)
    for (wave, lane), (ls, lx) in lanes.items():
        assert (s[wave, lane], x[wave, lane]) == (ls, lx)


def test_closed_form_passes_plus_prefix():
    # global sinks over m full passes plus a prefix of r vectors:
    # sum = m * S + S_prefix (mod 2**32); xor = (X if m odd) ^ X_prefix
    V, K, nw = 16, 4, 3
    n_vec = 64 * 9
    w = _buf(n_vec * V, seed=3)
    S, X = checksums.whole_buffer(w)
    for Q in (1, 2, 8, 9, 20, 21, 33):
        issued = 64 * K * Q
        m, r = divmod(issued, n_vec)
        ps, px = checksums.whole_buffer(w[:r * V // 4])
        want_s = (m * S + ps) & 0xFFFFFFFF
        want_x = (X if m % 2 else 0) ^ px
        s, x = checksums.per_wave(w, V, K, Q, nw)
        assert checksums.combine(s, x) == (want_s, want_x)


def test_xor_cancels_on_even_passes_but_sum_does_not():
    V, K, nw = 4, 2, 2
    n_vec = 64 * 4
    w = _buf(n_vec * V, seed=4)
    S, X = checksums.whole_buffer(w)
    Q = 2 * n_vec // (64 * K)
    s, x = checksums.combine(*checksums.per_wave(w, V, K, Q, nw))
    assert x == 0 and s == (2 * S) & 0xFFFFFFFF and s != 0


def test_one_full_pass_is_independent_of_K_and_grid():
    # the invariant the GPU sweep relies on: every power-of-two K at fixed
    # work issues one full pass, so the global sinks equal the whole buffer
    V = 16
    n_vec = 64 * 64
    w = _buf(n_vec * V, seed=5)
    want = checksums.whole_buffer(w)
    for K, nw in itertools.product((1, 2, 4, 8, 16), (1, 3, 16)):
        p = plan.wave_group(n_vec, K, nw)
        assert p["issued"] == n_vec
        got = checksums.combine(*checksums.per_wave(w, V, K, p["Q"], nw))
        assert got == want


def test_lanes_fold_into_waves():
    V, K, Q, nw = 8, 3, 11, 4
    w = _buf(8 * 64 * 10, seed=6)
    ls, lx = checksums.per_lane(w, V, K, Q, nw)
    s, x = checksums.per_wave(w, V, K, Q, nw)
    assert ((ls.astype(np.uint64).sum(axis=1) & 0xFFFFFFFF) == s).all()
    assert (np.bitwise_xor.reduce(lx, axis=1) == x).all()


def test_every_instruction_is_one_coalesced_segment():
    # lane l of a load reads vector base + l: 64 consecutive vectors
    K, n_vec = 5, 64 * 7
    for q in range(6):
        for j in range(K):
            v = [checksums.vector_index(q, j, l, K, n_vec) for l in range(64)]
            assert v == list(range(v[0], v[0] + 64))


def test_two_stream_regions_partition_the_buffer():
    V, nw = 16, 2
    n_vec = 64 * 10
    w = _buf(n_vec * V, seed=8)
    (a0, an), (b0, bn) = checksums.two_stream_regions(n_vec)
    assert a0 == 0 and a0 + an == b0 and b0 + bn == n_vec
    K = 1
    sa, xa = checksums.per_wave(w, V, K, an // 64, nw, base=a0, n_vec=an)
    sb, xb = checksums.per_wave(w, V, K, bn // 64, nw, base=b0, n_vec=bn)
    s = (checksums.combine(sa, xa)[0] + checksums.combine(sb, xb)[0]) & 0xFFFFFFFF
    x = checksums.combine(sa, xa)[1] ^ checksums.combine(sb, xb)[1]
    assert (s, x) == checksums.whole_buffer(w)


@pytest.mark.parametrize("V,K,Q,nw,nbytes", CASES)
def test_blocked_order_matches_brute_force(V, K, Q, nw, nbytes):
    w = _buf(nbytes, seed=21)
    lanes = brute.simulate(w, V, K, Q, nw, blocked=True)
    s, x = checksums.per_lane(w, V, K, Q, nw, order=plan.BLOCKED)
    for (wave, lane), (ls, lx) in lanes.items():
        assert (s[wave, lane], x[wave, lane]) == (ls, lx)
    ws, wx = checksums.per_wave(w, V, K, Q, nw, order=plan.BLOCKED, chunk_groups=3)
    for wave in range(nw):
        assert checksums.wave_from_seed(21, V, K, Q, nw, wave, buffer_bytes=nbytes,
                                        order=plan.BLOCKED) == (ws[wave], wx[wave])


@pytest.mark.parametrize("V,K,Q,nw,nbytes", CASES)
def test_strided_layout_matches_brute_force(V, K, Q, nw, nbytes):
    """The strided layout (load j of group q reads segment j*Q + q): the
    vectorised oracle equals the lane-by-lane simulation, per lane, per
    wave and from the seed; the cell's global sinks equal the adjacent
    layout's, since both read the stream 0 .. 64 K Q - 1 modulo the
    region."""
    w = _buf(nbytes, seed=23)
    lanes = brute.simulate(w, V, K, Q, nw, strided=True)
    s, x = checksums.per_lane(w, V, K, Q, nw, order=plan.STRIDED)
    for (wave, lane), (ls, lx) in lanes.items():
        assert (s[wave, lane], x[wave, lane]) == (ls, lx)
    ws, wx = checksums.per_wave(w, V, K, Q, nw, order=plan.STRIDED, chunk_groups=3)
    for wave in range(nw):
        assert checksums.wave_from_seed(23, V, K, Q, nw, wave, buffer_bytes=nbytes,
                                        order=plan.STRIDED) == (ws[wave], wx[wave])
        lane = (7 * wave) % 64
        assert checksums.lane_from_seed(23, V, K, Q, nw, wave, lane, nbytes // V,
                                        order=plan.STRIDED) == (s[wave, lane], x[wave, lane])
    rs, rx = checksums.per_wave(w, V, K, Q, nw)
    assert checksums.combine(ws, wx) == checksums.combine(rs, rx)


def test_strided_vector_index_spreads_a_groups_loads():
    # Q = 5 groups of K = 3 loads over 15 segments: group 2 reads 2, 7, 12
    n_vec = 15 * 64
    got = [checksums.vector_index(2, j, 0, 3, n_vec, Q=5, order=plan.STRIDED) // 64
           for j in range(3)]
    assert got == [2, 7, 12]
    assert [checksums.vector_index(2, j, 0, 3, n_vec) // 64 for j in range(3)] == [6, 7, 8]


def test_orders_partition_the_same_groups():
    for Q, nw in [(0, 3), (1, 4), (7, 3), (12, 4), (13, 4), (100, 7)]:
        for order in (plan.ROUND_ROBIN, plan.BLOCKED, plan.STRIDED):
            seen = sorted(q for w in range(nw) for q in plan.groups_of_wave(w, Q, nw, order))
            assert seen == list(range(Q))
            for w in range(nw):
                for q in plan.groups_of_wave(w, Q, nw, order):
                    assert plan.owner(q, Q, nw, order) == w
    # global sinks do not depend on the order
    V, K, nw = 16, 3, 5
    w = _buf(16 * 64 * 16, seed=22)
    Q = 23
    a = checksums.combine(*checksums.per_wave(w, V, K, Q, nw))
    b = checksums.combine(*checksums.per_wave(w, V, K, Q, nw, order=plan.BLOCKED))
    assert a == b


@pytest.mark.parametrize("V,K", [(16, 1), (16, 7), (8, 3), (4, 13), (16, 16)])
def test_range_sinks_equal_a_one_pass_cell(V, K):
    """A one-pass cell over a region (no wrap) reads exactly its issued
    prefix once: the per-wave oracle's global sinks equal the range sums of
    that prefix, for K that do not divide the region too."""
    seed, base_words = 77, 1000
    n_vec = (48 << 10) // V
    words = splitmix.words(seed, 0, base_words + n_vec * V // 4)
    region = words[base_words:]
    Q = n_vec // (64 * K)
    s, x = checksums.per_wave(region, V, K, Q, 24, n_vec=n_vec)
    want = checksums.combine(s, x)
    issued_words = Q * 64 * K * V // 4
    assert checksums.range_sinks(seed, base_words, issued_words, chunk=999) == want


def test_range_sinks_brute_force_and_empty():
    seed = 3
    got = checksums.range_sinks(seed, 17, 50, chunk=7)
    s = sum(splitmix.word_int(seed, i) for i in range(17, 67)) & 0xFFFFFFFF
    x = 0
    for i in range(17, 67):
        x ^= splitmix.word_int(seed, i)
    assert got == (s, x)
    assert checksums.range_sinks(seed, 5, 0) == (0, 0)


def test_range_sinks_many_combines_pieces():
    ranges = [(9, 0, 10000), (9, 123, 4567), (10, 5, 1), (9, 0, 10000), (9, 40, 0)]
    want = [checksums.range_sinks(*r) for r in ranges]
    assert checksums.range_sinks_many(ranges, threads=3, piece=1000) == want
    assert checksums.range_sinks_many(ranges, threads=1, piece=333) == want


def test_vectorised_oracle_matches_brute_force_on_random_cells():
    """Per-lane and per-wave sinks of the vectorised oracle against the
    lane-by-lane simulation, over random small cells of every order (random
    words, wrap, ragged deals, groups larger than the buffer)."""
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=60, deadline=None, derandomize=not os.environ.get("ILPSWEEP_HYPOTHESIS_RANDOM"))
    @given(order=st.sampled_from([plan.ROUND_ROBIN, plan.BLOCKED, plan.STRIDED]),
           V=st.sampled_from([4, 8, 16]), K=st.integers(1, 6), Q=st.integers(1, 12),
           nw=st.integers(1, 5), segs=st.integers(1, 9), seed=st.integers(0, 2**32 - 1))
    def check(order, V, K, Q, nw, segs, seed):
        nbytes = V * 64 * segs
        w = splitmix.buffer_words(seed, nbytes)
        lanes = brute.simulate(w, V, K, Q, nw, blocked=order == plan.BLOCKED,
                               strided=order == plan.STRIDED)
        s, x = checksums.per_lane(w, V, K, Q, nw, order=order)
        for (wave, lane), (ls, lx) in lanes.items():
            assert (s[wave, lane], x[wave, lane]) == (ls, lx)
        bs, bx = brute.per_wave(lanes, nw)
        ws, wx = checksums.per_wave(w, V, K, Q, nw, order=order, chunk_groups=2)
        assert ws.tolist() == bs and wx.tolist() == bx

    check()
