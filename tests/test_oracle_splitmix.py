"""Pins for the oracle's SplitMix64 buffer generator."""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN
from oracle import splitmix


def _golden():
    with open(os.path.join(GOLDEN, "splitmix64_vectors.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden())
def test_published_outputs(case):
    want = [int(v, 0) for v in case["outputs"]]
    got = [splitmix.output_int(case["seed"], i) for i in range(len(want))]
    assert got == want


@pytest.mark.parametrize("case", _golden())
def test_words_are_low_halves_of_published_outputs(case):
    want = [int(v, 0) & 0xFFFFFFFF for v in case["outputs"]]
    got = splitmix.words(case["seed"], 0, len(want)).tolist()
    assert got == want


def test_vectorised_matches_scalar_at_large_indices():
    rng = np.random.default_rng(7)
    seed = 0x1D5EED01
    for start in [0, 1, 2**31 - 3, 2**32 - 2, 5 * 2**30 + 17, 2**40 + 5]:
        n = int(rng.integers(1, 40))
        got = splitmix.words(seed, start, n).tolist()
        want = [splitmix.word_int(seed, start + i) for i in range(n)]
        assert got == want


def test_buffer_chunking_is_invisible():
    a = splitmix.buffer_words(99, 4 * 10007, chunk_words=1000)
    b = splitmix.words(99, 0, 10007)
    assert np.array_equal(a, b)


def test_seed_wraps_modulo_2_64():
    assert splitmix.words(2**64 + 5, 3, 4).tolist() == splitmix.words(5, 3, 4).tolist()
