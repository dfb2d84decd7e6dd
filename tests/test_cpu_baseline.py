"""The multithreaded CPU baseline sort (cpu_baseline/) against the oracle:
keys only and pairs, 32- and 64-bit keys, empty, tiny, ragged and
low-entropy inputs (skipped places), one to eight threads."""
import numpy as np
import pytest

import cpu_baseline
import oracle
import workload as W


@pytest.mark.parametrize("key_bits", [32, 64])
@pytest.mark.parametrize("n", [0, 1, 7, 1000, 100_003])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_matches_oracle(key_bits, n, threads):
    keys = W.uniform(5, n, key_bits)
    vals = np.arange(n, dtype=np.uint32)
    k, v = cpu_baseline.sort(keys, vals, threads=threads)
    wk, wv = oracle.sort(keys, vals)
    assert np.array_equal(k, wk) and np.array_equal(v, wv)
    k, v = cpu_baseline.sort(keys, threads=threads)
    assert v is None and np.array_equal(k, wk)


@pytest.mark.parametrize("dist", ["and4", "and16", "equal", "zipf", "distinct16", "presorted"])
def test_skewed_inputs_and_skipped_places(dist):
    keys = W.make_keys(dist, 6, 200_001)
    vals = np.arange(keys.size, dtype=np.uint32)
    k, v = cpu_baseline.sort(keys, vals, threads=5)
    wk, wv = oracle.sort(keys, vals)
    assert np.array_equal(k, wk) and np.array_equal(v, wv)


def test_default_threads_reported():
    assert cpu_baseline.threads_used() >= 1
    assert cpu_baseline.threads_used(3) == 3
