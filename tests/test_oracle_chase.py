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
