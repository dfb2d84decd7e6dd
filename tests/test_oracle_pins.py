"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests reuses the oracle's own code to produce an expected value:
expectations come from the paper's printed worked examples (tests/golden/),
closed forms, brute force written here independently (Python's stable
`sorted`), invariants, or library routines (numpy.sort) in the cases where the
definition reduces to them.
"""
import itertools
import random

import numpy as np
import pytest

import oracle
from conftest import read_golden


def field(k, begin, end):
    return (int(k) >> begin) & ((1 << (end - begin)) - 1)


def brute_sort(keys, vals, begin, end):
    """Stable comparison sort by the bit field [begin, end): Python's sorted is stable."""
    order = sorted(range(len(keys)), key=lambda i: field(keys[i], begin, end))
    ko = np.array([keys[i] for i in order], dtype=keys.dtype)
    vo = None if vals is None else np.array([vals[i] for i in order], dtype=np.uint32)
    return ko, vo


# --------------------------------------------------------------- paper examples

def test_prefix_sum_worked_example():
    """Section 2: exclusive sum of <8,6,7,5,3,0,9,2> is <0,8,14,21,26,29,29,38>."""
    g = read_golden("prefix_sum_example.txt")
    hist = np.array([g["histogram"]], dtype=np.uint64)
    assert hist.shape[1] == g["radix"][0]
    off = oracle.exclusive_sums(hist)
    assert off[0].tolist() == g["offsets"]


def test_digit_flags_worked_example():
    """Section 2: keys <17,8,24,5>, low 3-bit place, flags and flag prefix for digit 0."""
    g = read_golden("digit_flags_example.txt")
    keys = np.array(g["keys"], dtype=np.uint32)
    d = g["digit_bits"][0]
    digits = [oracle.digit(k, 0, 32, d, 0) for k in keys]
    flags = [1 if x == g["digit"][0] else 0 for x in digits]
    assert flags == g["flags"]
    # The exclusive prefix of the flags, computed by the oracle's scan.
    pref = oracle.exclusive_sums(np.array([flags], dtype=np.uint64))[0].tolist()
    assert pref == g["flag_prefix"]
    # In one binning iteration each flagged key lands at bin start + its prefix.
    hist = oracle.histograms(keys, 0, d, d)
    off = oracle.exclusive_sums(hist)
    out, _ = oracle.binning_pass(keys, 0, d, off[0])
    base = int(off[0][g["digit"][0]])
    for i, f in enumerate(flags):
        if f:
            assert out[base + g["flag_prefix"][i]] == keys[i]


def test_lookback_figure7():
    """Figure 7: local counts -> inclusive prefixes 11, 26, 35, 45, 53."""
    g = read_golden("lookback_fig7.txt")
    incl = oracle.inclusive_scan(g["local_counts"]).tolist()
    assert incl == g["inclusive"]
    assert incl[3] == g["exclusive_of_tile_4"][0]


def test_lookback_figure7_status_words():
    """The final chained-scan state of Figure 7f through the status-word oracle.

    Five tiles of 16 keys each; tile t holds local_counts[t] keys whose 4-bit
    digit is 0 and the rest with digit 1. Every counter of digit 0 must end as
    status G holding the inclusive prefixes the paper prints.
    """
    g = read_golden("lookback_fig7.txt")
    tile = 16
    keys = []
    for c in g["local_counts"]:
        keys += [0] * c + [1] * (tile - c)
    keys = np.array(keys, dtype=np.uint32)
    st = oracle.pass_status(keys, 0, 4, tile)
    for t, want in enumerate(g["inclusive"]):
        s, v = oracle.status_unpack(int(st[t, 0]))
        assert s == oracle.STATUS_G and v == want
    # digit 1 is the complement within each tile
    ones = np.cumsum([tile - c for c in g["local_counts"]])
    for t in range(5):
        assert oracle.status_unpack(int(st[t, 1])) == (oracle.STATUS_G, int(ones[t]))


def test_status_word_layout():
    """Figure 6: two high bits status, 30 low bits value."""
    assert oracle.status_pack(oracle.STATUS_G, 35) == (2 << 30) | 35
    assert oracle.status_pack(oracle.STATUS_L, (1 << 30) - 1) == 0x7FFFFFFF
    assert oracle.status_unpack(0x80000023) == (2, 35)
    assert oracle.status_unpack(0x40000000) == (1, 0)
    assert oracle.status_unpack(0) == (0, 0)


def test_num_places_closed_form():
    """Section 1: p = ceil(k/d)."""
    for k in (32, 64):
        for d in range(1, 17):
            assert oracle.num_places(0, k, d) == -(-k // d)
    assert oracle.num_places(0, 32, 8) == 4
    assert oracle.num_places(0, 32, 7) == 5  # Table 2 prints 4 here; see the reading of p
    assert oracle.num_places(0, 64, 8) == 8
    assert oracle.num_places(5, 5, 8) == 0


def test_memory_operation_model():
    """Section 3: (2p+1)n vs 3pn operations; 1.33x at p = 4, 1.5x ceiling."""
    g = read_golden("memory_ops_model.txt")
    p = g["p"][0]
    assert round(3 * p / (2 * p + 1), 2) == g["reduction"][0]
    assert abs(3 * 10**6 / (2 * 10**6 + 1) - g["ceiling"][0]) < 1e-5


# --------------------------------------------------------------- brute force

@pytest.mark.parametrize("key_bits", [32, 64])
def test_sort_matches_brute_force_random(key_bits):
    rng = random.Random(1234 + key_bits)
    dt = np.uint32 if key_bits == 32 else np.uint64
    for _ in range(300):
        n = rng.randint(0, 70)
        begin = rng.randint(0, key_bits)
        end = rng.randint(begin, key_bits)
        d = rng.randint(1, 11)
        span = rng.choice([2, 7, 1 << 12, (1 << key_bits) - 1])
        keys = np.array([rng.randint(0, span) for _ in range(n)], dtype=dt)
        keys <<= dt(rng.randint(0, 3))
        vals = np.arange(n, dtype=np.uint32)
        ko, vo = oracle.sort(keys, vals, begin, end, d)
        bk, bv = brute_sort(keys, vals, begin, end)
        assert np.array_equal(ko, bk), (n, begin, end, d)
        assert np.array_equal(vo, bv), (n, begin, end, d)


def test_exhaustive_small_sequences():
    """Every sequence of length <= 5 over 3-bit keys, for d = 1, 2, 3 and
    several bit ranges, against brute force. All sequences go through the
    segmented oracle at once (one segment each), which also pins it."""
    seqs = []
    for length in range(0, 6):
        seqs.extend(itertools.product(range(8), repeat=length))
    lengths = np.array([len(s) for s in seqs], dtype=np.int64)
    off = np.zeros(len(seqs) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lengths)
    keys = np.array([x for s in seqs for x in s], dtype=np.uint32)
    vals = np.arange(keys.size, dtype=np.uint32)
    for (begin, end) in [(0, 3), (1, 3), (0, 2), (2, 3), (0, 32)]:
        for d in (1, 2, 3):
            ko, vo = oracle.sort_segments(keys, off, vals, begin, end, d)
            for s in range(len(seqs)):
                a, b = int(off[s]), int(off[s + 1])
                if b - a < 2:
                    assert np.array_equal(ko[a:b], keys[a:b])
                    continue
                bk, bv = brute_sort(keys[a:b], vals[a:b], begin, end)
                assert np.array_equal(ko[a:b], bk)
                assert np.array_equal(vo[a:b], bv)


@pytest.mark.parametrize("key_bits,d", [(32, 8), (32, 5), (64, 8), (64, 7)])
def test_each_pass_is_stable_sort_by_its_digit(key_bits, d):
    """Pass j output = stable sort, by digit j alone, of pass j-1 output."""
    dt = np.uint32 if key_bits == 32 else np.uint64
    rng = np.random.default_rng(7)
    keys = rng.integers(0, 1 << 62, 3000, dtype=np.uint64).astype(dt)
    begin, end = 3, key_bits - 2
    ko, _, passes = oracle.sort(keys, None, begin, end, d, return_passes=True)
    p = oracle.num_places(begin, end, d)
    assert passes.shape == (p, keys.size)
    prev = keys
    for j in range(p):
        lo = begin + j * d
        hi = min(lo + d, end)
        order = sorted(range(prev.size), key=lambda i: field(prev[i], lo, hi))
        assert np.array_equal(passes[j], prev[order]), j
        prev = passes[j]
    assert np.array_equal(ko, prev)


# --------------------------------------------------------------- invariants

@pytest.mark.parametrize("key_bits", [32, 64])
def test_histogram_invariants(key_bits):
    dt = np.uint32 if key_bits == 32 else np.uint64
    rng = np.random.default_rng(11)
    keys = rng.integers(0, 1 << 63, 20000, dtype=np.uint64).astype(dt)
    for d in (4, 8, 11):
        hist = oracle.histograms(keys, 0, key_bits, d)
        off = oracle.exclusive_sums(hist)
        p = oracle.num_places(0, key_bits, d)
        assert hist.shape == (p, 1 << d)
        assert np.all(hist.sum(axis=1) == keys.size)  # totals equal n at every place
        assert np.all(off[:, -1] + hist[:, -1] == keys.size)
        # order independence (Section 3: counts depend only on the multiset)
        perm = rng.permutation(keys.size)
        assert np.array_equal(oracle.histograms(keys[perm], 0, key_bits, d), hist)
        # independent count with numpy for every place
        for j in range(p):
            lo = j * d
            w = min(d, key_bits - lo)
            dig = ((keys.astype(np.uint64) >> np.uint64(lo)) & np.uint64((1 << w) - 1))
            assert np.array_equal(np.bincount(dig.astype(np.int64), minlength=1 << d), hist[j])


@pytest.mark.parametrize("key_bits", [32, 64])
def test_full_width_keys_only_equals_numpy_sort(key_bits):
    """Special case: full width and no values reduces to an ordinary sort."""
    dt = np.uint32 if key_bits == 32 else np.uint64
    rng = np.random.default_rng(5)
    for n in (0, 1, 2, 1000, 65537):
        keys = rng.integers(0, 1 << 64, n, dtype=np.uint64).astype(dt)
        ko, _ = oracle.sort(keys, None, 0, key_bits, 8)
        assert np.array_equal(ko, np.sort(keys))


def test_pairs_permutation_sorted_stable():
    rng = np.random.default_rng(3)
    n = 50000
    keys = (rng.integers(0, 1 << 32, n, dtype=np.uint64) & np.uint64(0xF0F0)).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = oracle.sort(keys, vals, 0, 32, 8)
    assert np.array_equal(np.sort(vo), vals)  # a permutation
    assert np.array_equal(ko, keys[vo])  # keys travel with their values
    assert np.all(ko[1:] >= ko[:-1])  # sorted
    same = ko[1:] == ko[:-1]
    assert np.all(vo[1:][same] > vo[:-1][same])  # stable


def test_partial_bit_range_carries_whole_keys():
    rng = np.random.default_rng(9)
    keys = rng.integers(0, 1 << 32, 5000, dtype=np.uint64).astype(np.uint32)
    ko, _ = oracle.sort(keys, None, 8, 20, 8)
    assert np.array_equal(np.sort(ko), np.sort(keys))
    f = (ko >> np.uint32(8)) & np.uint32(0xFFF)
    assert np.all(f[1:] >= f[:-1])
    # a stable sort by the field equals numpy's stable argsort of the field
    fi = (keys >> np.uint32(8)) & np.uint32(0xFFF)
    assert np.array_equal(ko, keys[np.argsort(fi, kind="stable")])


def test_begin_equals_end_copies():
    keys = np.array([5, 3, 9], dtype=np.uint32)
    ko, vo = oracle.sort(keys, np.array([0, 1, 2], dtype=np.uint32), 7, 7, 8)
    assert ko.tolist() == [5, 3, 9] and vo.tolist() == [0, 1, 2]


def test_segments_independent():
    rng = np.random.default_rng(21)
    lengths = rng.integers(0, 300, 60)
    off = np.zeros(61, dtype=np.uint64)
    off[1:] = np.cumsum(lengths)
    n = int(off[-1])
    keys = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = oracle.sort_segments(keys, off, vals, 0, 32, 8)
    for s in range(60):
        a, b = int(off[s]), int(off[s + 1])
        assert np.all((vo[a:b] >= a) & (vo[a:b] < b))  # no element crosses a boundary
        assert np.array_equal(ko[a:b], keys[a:b][np.argsort(keys[a:b], kind="stable")])
    with pytest.raises(ValueError):
        bad = off.copy()
        bad[-1] += 1
        oracle.sort_segments(keys, bad, vals)


def test_pass_status_invariants():
    """Final chained-scan state: all G; consecutive differences are the
    tile's own digit counts (np.bincount); the last tile holds the totals."""
    rng = np.random.default_rng(13)
    tile = 96
    keys = rng.integers(0, 1 << 32, 96 * 7 + 13, dtype=np.uint64).astype(np.uint32)
    lo, width = 4, 6
    st = oracle.pass_status(keys, lo, width, tile)
    g = -(-keys.size // tile)
    assert st.shape == (g, 1 << width)
    assert np.all(st >> np.uint32(30) == oracle.STATUS_G)
    vals = (st & np.uint32(0x3FFFFFFF)).astype(np.int64)
    dig = ((keys >> np.uint32(lo)) & np.uint32((1 << width) - 1)).astype(np.int64)
    prev = np.zeros(1 << width, dtype=np.int64)
    for t in range(g):
        cnt = np.bincount(dig[t * tile:(t + 1) * tile], minlength=1 << width)
        assert np.array_equal(vals[t] - prev, cnt)
        prev = vals[t]
    assert np.array_equal(vals[-1], np.bincount(dig, minlength=1 << width))


# ---------------------------------------------------------------- key order

def _float_class_key(bits: int, kb: int):
    """Rank of an IEEE 754 bit pattern in the order the sort promises
    (-NaN < -inf < negative < -0 < +0 < positive < +inf < +NaN, NaNs by their
    magnitude bits), computed from the decoded value, not from the bit
    transform under test."""
    ftype, itype = (np.float32, np.uint32) if kb == 32 else (np.float64, np.uint64)
    x = float(np.array([bits], dtype=itype).view(ftype)[0])
    negative = bits >> (kb - 1)
    magnitude = bits & ((1 << (kb - 1)) - 1)
    if x != x:
        return (0, -magnitude) if negative else (7, magnitude)
    if x == float("-inf"):
        return (1, 0)
    if x == float("inf"):
        return (6, 0)
    if x == 0.0:
        return (3, 0) if negative else (4, 0)
    return (2, x) if x < 0 else (5, x)


SPECIAL_F32 = [0x00000000, 0x80000000, 0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00000,
               0x7F800001, 0xFF800001, 0x00000001, 0x80000001, 0x3F800000, 0xBF800000,
               0x7F7FFFFF, 0xFF7FFFFF, 0x00800000, 0x80800000]
SPECIAL_F64 = [0x0, 0x8000000000000000, 0x7FF0000000000000, 0xFFF0000000000000,
               0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001,
               0xFFF0000000000001, 0x1, 0x8000000000000001, 0x3FF0000000000000,
               0xBFF0000000000000, 0x7FEFFFFFFFFFFFFF, 0xFFEFFFFFFFFFFFFF]


def test_signed_ordered_bits_closed_form():
    """Two's complement: the ordered bits are x + 2^(w-1) as an unsigned number."""
    for kb, st, ut in ((32, np.int32, np.uint32), (64, np.int64, np.uint64)):
        x = np.array([-(1 << (kb - 1)), -2, -1, 0, 1, 7, (1 << (kb - 1)) - 1], dtype=st)
        got = oracle.ordered_bits(x.view(ut), oracle.KEY_SIGNED)
        want = [int(v) + (1 << (kb - 1)) for v in x]
        assert [int(g) for g in got] == want
        desc = oracle.ordered_bits(x.view(ut), oracle.KEY_SIGNED, descending=True)
        assert [int(g) for g in desc] == [(1 << kb) - 1 - w for w in want]


def test_float_ordered_bits_follow_the_total_order():
    for kb, specials, ut in ((32, SPECIAL_F32, np.uint32), (64, SPECIAL_F64, np.uint64)):
        ranked = sorted(specials, key=lambda b: _float_class_key(b, kb))
        got = oracle.ordered_bits(np.array(ranked, dtype=ut), oracle.KEY_FLOAT)
        assert all(int(a) < int(b) for a, b in zip(got[:-1], got[1:])), kb
        down = oracle.ordered_bits(np.array(ranked, dtype=ut), oracle.KEY_FLOAT, descending=True)
        assert all(int(a) > int(b) for a, b in zip(down[:-1], down[1:])), kb


@pytest.mark.parametrize("kb", [32, 64])
def test_signed_sort_matches_numpy(kb):
    st, ut = (np.int32, np.uint32) if kb == 32 else (np.int64, np.uint64)
    rng = np.random.default_rng(71)
    x = rng.integers(-600, 600, 6000).astype(st)  # both signs, many ties
    x[:4] = [np.iinfo(st).min, np.iinfo(st).max, -1, 0]
    v = np.arange(x.size, dtype=np.uint32)
    ko, vo = oracle.sort(x.view(ut), v, key_type=oracle.KEY_SIGNED)
    order = np.argsort(x, kind="stable")
    assert np.array_equal(vo, order)
    assert np.array_equal(ko.view(st), x[order])
    ko, vo = oracle.sort(x.view(ut), v, key_type=oracle.KEY_SIGNED, descending=True)
    down = np.argsort(-x.astype(np.float64), kind="stable")  # exact: |x| < 2^53
    assert np.array_equal(vo, down)


@pytest.mark.parametrize("kb", [32, 64])
def test_float_sort_matches_numpy_on_finite_nonzero_values(kb):
    ft, ut = (np.float32, np.uint32) if kb == 32 else (np.float64, np.uint64)
    rng = np.random.default_rng(73)
    ints = rng.integers(1, 400, 5000) * rng.choice([-1, 1], 5000)
    x = (ints * 0.37).astype(ft) * ft(10.0) ** rng.integers(-3, 4, 5000).astype(ft)
    v = np.arange(x.size, dtype=np.uint32)
    ko, vo = oracle.sort(x.view(ut), v, key_type=oracle.KEY_FLOAT)
    order = np.argsort(x, kind="stable")
    assert np.array_equal(vo, order)
    assert np.array_equal(ko, x.view(ut)[order])


@pytest.mark.parametrize("kb", [32, 64])
def test_float_sort_of_special_values_brute_force(kb):
    specials = SPECIAL_F32 if kb == 32 else SPECIAL_F64
    ut = np.uint32 if kb == 32 else np.uint64
    rng = np.random.default_rng(79)
    bits = np.array([specials[i] for i in rng.integers(0, len(specials), 700)], dtype=ut)
    v = np.arange(bits.size, dtype=np.uint32)
    for descending in (False, True):
        sign = -1 if descending else 1
        want = sorted(range(bits.size),
                      key=lambda i: (tuple(sign * c for c in _float_class_key(int(bits[i]), kb)),
                                     i))
        ko, vo = oracle.sort(bits, v, key_type=oracle.KEY_FLOAT, descending=descending)
        assert list(vo) == want, descending
        assert np.array_equal(ko, bits[want])


@pytest.mark.parametrize("kb", [32, 64])
def test_descending_unsigned_sort_brute_force(kb):
    ut = np.uint32 if kb == 32 else np.uint64
    rng = np.random.default_rng(83)
    k = rng.integers(0, 1 << 20, 3000, dtype=np.uint64).astype(ut) << ut(kb - 20)
    k[::7] = k[3]  # ties
    v = np.arange(k.size, dtype=np.uint32)
    ko, vo = oracle.sort(k, v, descending=True)
    assert list(vo) == sorted(range(k.size), key=lambda i: (-int(k[i]), i))
    # a bit range: descending by the field, ties (equal fields) in input order
    b, e = 3, kb - 9
    field = lambda i: (int(k[i]) >> b) & ((1 << (e - b)) - 1)  # noqa: E731
    ko, vo = oracle.sort(k, v, b, e, descending=True)
    assert list(vo) == sorted(range(k.size), key=lambda i: (-field(i), i))


# ------------------------------------------------- typed keys, per segment

SEG_LENGTHS = [0, 1, 37, 500, 0, 1200, 3, 2, 900]


def _seg_offsets(lengths):
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint64)


@pytest.mark.parametrize("kb", [32, 64])
def test_segments_typed_signed_and_float_match_numpy_per_segment(kb):
    """Each segment of a typed segmented sort equals numpy's stable argsort of
    that segment's decoded values (signed integers, finite non-zero floats),
    ascending and descending; values carry the global input index."""
    st, ft, ut = ((np.int32, np.float32, np.uint32) if kb == 32
                  else (np.int64, np.float64, np.uint64))
    off = _seg_offsets(SEG_LENGTHS)
    n = int(off[-1])
    rng = np.random.default_rng(211)
    v = np.arange(n, dtype=np.uint32)
    xi = rng.integers(-300, 300, n).astype(st)  # both signs, many ties per segment
    ints = rng.integers(1, 400, n) * rng.choice([-1, 1], n)
    xf = (ints * 0.37).astype(ft) * ft(10.0) ** rng.integers(-3, 4, n).astype(ft)
    for x, key_type in ((xi, oracle.KEY_SIGNED), (xf, oracle.KEY_FLOAT)):
        for descending in (False, True):
            ko, vo = oracle.sort_segments(x.view(ut), off, v, key_type=key_type,
                                          descending=descending)
            for s in range(len(SEG_LENGTHS)):
                a, b = int(off[s]), int(off[s + 1])
                seg = x[a:b].astype(np.float64)  # exact: |x| < 2^53 or already float
                order = np.argsort(-seg if descending else seg, kind="stable")
                assert np.array_equal(vo[a:b], a + order), (kb, key_type, descending, s)
                assert np.array_equal(ko[a:b], x.view(ut)[a:b][order])


@pytest.mark.parametrize("kb", [32, 64])
def test_segments_typed_special_floats_and_bit_ranges_brute_force(kb):
    """Float special values (NaN payloads, signed zeros, infinities) ranked from
    decoded values, and descending unsigned sorts of a bit field, per segment,
    against Python's stable sorted()."""
    specials = SPECIAL_F32 if kb == 32 else SPECIAL_F64
    ut = np.uint32 if kb == 32 else np.uint64
    off = _seg_offsets(SEG_LENGTHS)
    n = int(off[-1])
    rng = np.random.default_rng(223)
    v = np.arange(n, dtype=np.uint32)
    bits = np.array([specials[i] for i in rng.integers(0, len(specials), n)], dtype=ut)
    for descending in (False, True):
        sign = -1 if descending else 1
        ko, vo = oracle.sort_segments(bits, off, v, key_type=oracle.KEY_FLOAT,
                                      descending=descending)
        for s in range(len(SEG_LENGTHS)):
            a, b = int(off[s]), int(off[s + 1])
            want = sorted(range(a, b), key=lambda i: (
                tuple(sign * c for c in _float_class_key(int(bits[i]), kb)), i))
            assert list(vo[a:b]) == want, (descending, s)
            assert np.array_equal(ko[a:b], bits[want])
    k = rng.integers(0, 1 << 20, n, dtype=np.uint64).astype(ut) << ut(kb - 20)
    k[::5] = k[2]  # ties across and within segments
    lo, hi = 3, kb - 9
    fld = lambda i: (int(k[i]) >> lo) & ((1 << (hi - lo)) - 1)  # noqa: E731
    ko, vo = oracle.sort_segments(k, off, v, lo, hi, descending=True)
    for s in range(len(SEG_LENGTHS)):
        a, b = int(off[s]), int(off[s + 1])
        want = sorted(range(a, b), key=lambda i: (-fld(i), i))
        assert list(vo[a:b]) == want, s
        assert np.array_equal(ko[a:b], k[want])
