"""Pointer-chase oracle and chain generator (no GPU)."""
import numpy as np
import pytest

from oracle import chase
import synth


@pytest.mark.parametrize("footprint,stride", [(8192, 128), (65536, 64), (4096, 4)])
def test_chain_is_one_cycle_over_every_node(footprint, stride):
    t, start = synth.chase_chain(footprint, stride, seed=3)
    words = t.numpy().view(np.uint32)
    n = footprint // stride
    assert chase.cycle_length(words, start, n + 1) == n
    # every node visited once, all on stride boundaries
    seen = set()
    idx = start
    for _ in range(n):
        assert idx % (stride // 4) == 0 and idx not in seen
        seen.add(idx)
        idx = int(words[idx])
    assert len(seen) == n


def test_follow_by_hand():
    words = np.array([2, 0, 3, 1], dtype=np.uint32)   # 0 -> 2 -> 3 -> 1 -> 0
    assert [chase.follow(words, 0, h) for h in range(6)] == [0, 2, 3, 1, 0, 2]
    assert chase.cycle_length(words, 0, 10) == 4
    assert chase.cycle_length(np.array([1, 1], dtype=np.uint32), 0, 5) is None


@pytest.mark.parametrize("n_starts", [1, 3, 8, 64])
def test_chain_starts_are_evenly_spaced_along_the_cycle(n_starts):
    """Start i is i * nodes / n_starts hops from start 0 along the cycle,
    and the chain is the one chase_chain builds from the same seed."""
    t, s0 = synth.chase_chain(8192, 128, seed=9)
    t2, starts = synth.chase_chain_starts(8192, 128, 9, n_starts)
    words = t.numpy().view(np.uint32)
    assert np.array_equal(words, t2.numpy().view(np.uint32)) and starts[0] == s0
    n = 8192 // 128
    for i, s in enumerate(starts):
        assert chase.follow(words, s0, (i * n) // n_starts) == s
    with pytest.raises(ValueError):
        synth.chase_chain_starts(8192, 128, 9, n + 1)
