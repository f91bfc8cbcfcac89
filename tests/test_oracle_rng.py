"""Pins of the oracle's counter-based generator (no GPU): its Philox-4x64-10
outputs equal those of numpy's independent Philox bit generator with the
same key, and its doubles equal numpy's Generator.random on that stream."""
import numpy as np
import pytest

from oracle.rng import philox4x64_10, raw_stream, uniform01


@pytest.mark.parametrize("seed", [0, 1, 12345, 2**63 + 17, 2**64 - 1])
def test_raw_stream_matches_numpy_philox(seed):
    ref = np.random.Philox(key=seed).random_raw(37)
    assert [int(x) for x in ref] == raw_stream(seed, 37)


@pytest.mark.parametrize("seed", [0, 7, 10000])
def test_uniform01_matches_numpy_generator(seed):
    ref = np.random.Generator(np.random.Philox(key=seed)).random(101)
    got = uniform01(seed, 101)
    assert np.array_equal(got, ref)
    assert got.min() >= 0.0 and got.max() < 1.0


def test_counter_block_is_the_cipher_of_b_plus_one():
    out = raw_stream(99, 12)
    for b in range(3):
        assert list(philox4x64_10((b + 1, 0, 0, 0), (99, 0))) == out[4 * b:4 * b + 4]
