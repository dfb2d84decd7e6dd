"""Checks of the seeded input generators (not the oracle): SplitMix64 against
its published first output and a pure-Python form, the Thearling-Smith bands
against the paper's Table 1, and the segmented and sweep workload recipes."""
import math

import numpy as np
import pytest

import workload as W
from conftest import read_golden


def test_splitmix64_published_first_output():
    # SplitMix64 started from state 0 returns mix64(gamma) first.
    assert int(W.mix64(np.array([W.GAMMA], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF
    assert W.mix64_int(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF


def test_vectorised_equals_scalar():
    w = W.words_numpy(3, 1, 100, start=5)
    b = int(W.base(3, 1))
    for i in range(100):
        z = (b + (i + 6) * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
        assert int(w[i]) == W.mix64_int(z)


def test_chunked_generation_is_seamless():
    a = W.words(7, 2, (1 << 22) + 10)
    b = W.words(7, 2, 20, start=(1 << 22) - 10)
    assert np.array_equal(a[(1 << 22) - 10:], b)


def test_determinism_and_streams():
    assert np.array_equal(W.uniform(1, 1000), W.uniform(1, 1000))
    assert not np.array_equal(W.uniform(1, 1000), W.uniform(2, 1000))
    assert not np.array_equal(W.words(1, 1, 100), W.words(1, 2, 100))
    assert W.uniform(1, 10, 64).dtype == np.uint64
    assert np.array_equal(W.uniform(1, 10, 32), (W.uniform(1, 10, 64) >> np.uint64(32)).astype(np.uint32))


def test_table1_closed_form():
    g = read_golden("entropy_table1.txt")
    for q, h in zip(g["q"], g["entropy_per_bit"]):
        # the table prints 6 significant digits at most
        assert abs(W.binary_entropy(2.0 ** -q) - h) <= 5e-6 + 1e-4 * h, q


@pytest.mark.parametrize("q", [1, 2, 3, 4, 8])
def test_entropy_bands_match_table1(q):
    g = read_golden("entropy_table1.txt")
    want = dict(zip(g["q"], g["entropy_per_bit"]))[q]
    keys = W.and_of_q(11, q, 1 << 20)
    got = W.per_bit_entropy(keys)
    assert abs(got - want) < max(3e-3, 0.05 * want), (q, got, want)


def test_all_equal():
    k = W.all_equal(2, 1000)
    assert np.all(k == k[0])


def test_lognormal_segments():
    L = W.lognormal_segment_lengths()
    assert L.size == 20000 and int(L.sum()) == 1 << 26 and L.min() >= 0
    raw = W.lognormal_segment_lengths(total=None)
    # median 2000 and sigma 1.5 before scaling; the sum is near E = S*m*exp(s^2/2)
    assert abs(np.median(raw) / 2000.0 - 1.0) < 0.05
    expect = 20000 * 2000 * math.exp(1.5 ** 2 / 2)
    assert abs(raw.sum() / expect - 1.0) < 0.1
    z = np.log(raw[raw > 0] / 2000.0)
    assert abs(z.std() - 1.5) < 0.05
    off = W.offsets_from_lengths(L)
    assert off[0] == 0 and off[-1] == 1 << 26


def test_zipf_head_probability():
    k = W.zipf_keys(5, 1 << 18)
    h = np.sum(1.0 / np.arange(1, (1 << 20) + 1) ** 1.1)
    p0 = 1.0 / h
    assert abs(np.mean(k == 0) - p0) < 0.01
    assert k.max() < 1 << 20


def test_sweep_cases():
    seen = set()
    for s in range(1000, 1200):
        n, kb, dist = W.sweep_case(s)
        assert (1 << 17) <= n <= (1 << 28)
        assert kb in (32, 64) and dist in W.DISTRIBUTIONS
        seen.add((kb, dist))
    assert len(seen) == 16


def test_other_distributions():
    assert np.all(np.diff(W.presorted(1, 1000).astype(np.int64)) >= 0)
    assert np.all(np.diff(W.reverse_sorted(1, 1000).astype(np.int64)) <= 0)
    assert len(np.unique(W.distinct16(1, 10000))) <= 16


def test_fast_generator_equals_numpy_definition():
    for seed, stream, start, n in [(1, 1, 0, 5000), (3, 7, 123456, 999), (2, 200, 1 << 33, 64)]:
        assert np.array_equal(W.words(seed, stream, n, start), W.words_numpy(seed, stream, n, start))
    w = [W.words_numpy(4, k, 4097) for k in (1, 2, 3)]
    acc = w[0] & w[1] & w[2]
    assert np.array_equal(W.and_of_q(4, 3, 4097, 64), acc)
    assert np.array_equal(W.and_of_q(4, 3, 4097, 32), (acc >> np.uint64(32)).astype(np.uint32))
    assert np.array_equal(W.uniform(4, 4097, 32), (w[0] >> np.uint64(32)).astype(np.uint32))
