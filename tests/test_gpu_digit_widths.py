"""Digit places narrower than 8 bits (Section 4, Table 2 varies the digit
width d): whole sorts, the histogram entry, the reduce-then-scan baseline,
strips and segmented sorts with d = 4..7 against the oracle at the same d.
Bit-exact everywhere; expected values come only from `oracle`."""
import numpy as np
import pytest
import torch

import oracle
import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ow():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2206_01784_amd as mod
    return mod


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def sort_and_check(ow, keys, vals, begin, end, d, cfg, key_type=0, descending=False):
    kb = keys.dtype.itemsize * 8
    tk = dev(keys)
    if key_type:
        cfg.key_type = key_type
        cfg.descending = int(descending)
    if vals is None:
        got_k, got_v = host(ow.sort_keys(tk, begin, end, config=cfg)), None
    else:
        rk, rv = ow.sort_pairs(tk, dev(vals), begin, end, config=cfg)
        got_k, got_v = host(rk), host(rv)
    want_k, want_v = oracle.sort(keys, vals, begin, end, d, key_type=key_type,
                                 descending=descending)
    assert np.array_equal(got_k, want_k), (kb, d, begin, end)
    if vals is not None:
        assert np.array_equal(got_v, want_v), (kb, d, begin, end)


@pytest.mark.parametrize("d", [4, 5, 6, 7])
@pytest.mark.parametrize("vals", [False, True])
def test_plain_sorts_at_every_digit_width(ow, d, vals):
    """32-bit keys over the full width (ceil(32 / d) passes, the last one
    narrower unless d divides 32) and over partial ranges; ragged sizes."""
    for n in (1, 4097, 300001):
        keys = W.uniform(40 + d, n)
        v = np.arange(n, dtype=np.uint32) if vals else None
        sort_and_check(ow, keys, v, 0, 32, d, ow.make_config(digit_bits=d))
        sort_and_check(ow, keys, v, 3, 29, d, ow.make_config(digit_bits=d))


@pytest.mark.parametrize("d", [5, 7])
def test_digit_widths_with_typed_keys_and_64_bit_ranges(ow, d):
    """Signed and floating-point keys, descending, and 64-bit keys over a
    range of at most 8 places."""
    n = 200003
    sort_and_check(ow, W.signed_ints(51, n), None, 0, 32, d, ow.make_config(digit_bits=d),
                   key_type=oracle.KEY_SIGNED, descending=True)
    sort_and_check(ow, W.float_bits(52, n), np.arange(n, dtype=np.uint32), 0, 32, d,
                   ow.make_config(digit_bits=d), key_type=oracle.KEY_FLOAT)
    keys64 = W.uniform(53, n, 64)
    span = 8 * d
    sort_and_check(ow, keys64, np.arange(n, dtype=np.uint32), 64 - span, 64, d,
                   ow.make_config(digit_bits=d))


def test_too_many_places_are_refused(ow):
    """A sort covers at most 8 places: 64-bit keys over all 64 bits need 8-bit
    digits."""
    keys = dev(W.uniform(54, 1000, 64))
    with pytest.raises(ow.OnesweepError):
        ow.sort_keys(keys, config=ow.make_config(digit_bits=7))


@pytest.mark.parametrize("d", [4, 6, 7])
def test_histogram_entry_at_narrow_digits(ow, d):
    """Phase 1 with d-bit places (one launch per group of at most one place
    per key byte): counts equal the oracle's, bins from 2^d on stay 0."""
    for kb in (32, 64):
        keys = W.uniform(60 + d, 123457, kb)
        end = kb if kb == 32 else 8 * d
        got = host(ow.histogram(dev(keys), 0, end, config=ow.make_config(digit_bits=d)))
        want = oracle.histograms(keys, 0, end, d)
        assert got.shape == (want.shape[0], 256)
        assert np.array_equal(got[:, :1 << d].astype(np.uint64), want), (kb, d)
        assert not got[:, 1 << d:].any()


def test_reduce_then_scan_and_strips_at_7_bit_digits(ow):
    n = 9 * 8192 + 1234
    keys = W.uniform(70, n)
    v = np.arange(n, dtype=np.uint32)
    cfg = ow.make_config(1024, 8, digit_bits=7, algorithm=ow.ALGORITHM_REDUCE_THEN_SCAN)
    sort_and_check(ow, keys, v, 0, 32, 7, cfg)
    cfg = ow.make_config(1024, 8, digit_bits=7, strip_log2=15)
    sort_and_check(ow, keys, v, 0, 32, 7, cfg)


@pytest.mark.parametrize("d", [5, 7])
@pytest.mark.parametrize("kb", [32, 64])
def test_segmented_sorts_at_narrow_digits(ow, d, kb):
    """Every class (LDS sorts and binned segments, whose first launch counts
    the d-bit places per segment) at d-bit digits."""
    lengths = W.lognormal_segment_lengths(num_segments=600, total=1 << 20, seed=d + kb)
    off = W.offsets_from_lengths(lengths)
    n = int(off[-1])
    keys = W.uniform(80 + d, n, kb)
    vals = np.arange(n, dtype=np.uint32)
    end = 32 if kb == 32 else 8 * d
    cfg = ow.make_config(digit_bits=d)
    rk, rv = ow.sort_segments(dev(keys), dev(off.astype(np.uint32)), dev(vals), 0, end,
                              config=cfg)
    want_k, want_v = oracle.sort_segments(keys, off, vals, 0, end, d)
    assert np.array_equal(host(rk), want_k)
    assert np.array_equal(host(rv), want_v)


def test_segment_tuner_may_pick_7_bit_digits(ow):
    """The autotuner times 8- and 7-bit digits; its pick sorts bit-exactly."""
    lengths = W.lognormal_segment_lengths(num_segments=500, total=1 << 20, seed=90)
    off = W.offsets_from_lengths(lengths)
    n = int(off[-1])
    keys = W.uniform(90, n)
    vals = np.arange(n, dtype=np.uint32)
    tk, tv, to = dev(keys), dev(vals), dev(off.astype(np.uint32))
    ko, vo = torch.empty_like(tk), torch.empty_like(tv)
    cfg = ow.tune_segments(tk, to, tv, keys_out=ko, values_out=vo, repetitions=1)
    torch.cuda.synchronize()
    assert cfg.digit_bits in (7, 8)
    want_k, want_v = oracle.sort_segments(keys, off, vals, 0, 32, cfg.digit_bits)
    assert np.array_equal(host(ko), want_k) and np.array_equal(host(vo), want_v)
