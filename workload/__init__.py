"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only produces input data. It holds none of the sorting method's
arithmetic, so both the CPU oracle and the GPU path may consume what it makes
without sharing any code with each other.

Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator::

    mix64(z)      = the SplitMix64 finaliser
    base(s, k)    = mix64((s << 8) | k)
    word(s, k, i) = mix64(base(s, k) + (i + 1) * 0x9E3779B97F4A7C15)

A 32-bit key is the high half of a word, a 64-bit key is the whole word.

Key distributions follow the Thearling-Smith entropy bands the paper uses
(Section 4: each key is the bitwise AND of q independent uniform words, so the
entropy per bit is H(2^-q), Table 1), plus the extra shapes the learned-config
sweep needs (Zipf, presorted, reverse-sorted, 16 distinct values) and the
log-normal segment lengths of the batched segmented workload.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Elements generated per numpy chunk; bounds temporary memory to ~100 MiB.
_CHUNK = 1 << 22


def mix64(z):
    """SplitMix64 finaliser on a numpy uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def mix64_int(z: int) -> int:
    """Pure-Python SplitMix64 finaliser (reference for the vectorised form)."""
    mask = (1 << 64) - 1
    z &= mask
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
    return z ^ (z >> 31)


def base(seed: int, stream: int) -> np.uint64:
    return np.uint64(mix64_int(((seed << 8) | stream) & ((1 << 64) - 1)))


_HERE = os.path.dirname(os.path.abspath(__file__))
_GEN_SRC = os.path.join(_HERE, "gen.c")
_GEN_LIB = os.path.join(_HERE, "libgen.so")
_gen = None


def build(force: bool = True) -> str:
    """Compile gen.c (the fast form of the same generator) with gcc."""
    if force or not os.path.exists(_GEN_LIB) or \
            os.path.getmtime(_GEN_LIB) < os.path.getmtime(_GEN_SRC):
        tmp = _GEN_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _GEN_SRC, "-o", tmp])
        os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _fast():
    global _gen
    if _gen is None:
        L = ctypes.CDLL(build(force=False))
        for f in ("gen_words", "gen_and_words", "gen_words_hi32", "gen_and_words_hi32"):
            getattr(L, f).argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_size_t,
                                      ctypes.c_void_p]
            getattr(L, f).restype = None
        _gen = L
    return _gen


def words_numpy(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """word(seed, stream, i) for i in [start, start + n): the numpy definition."""
    out = np.empty(n, dtype=np.uint64)
    b = base(seed, stream)
    for c0 in range(0, n, _CHUNK):
        c1 = min(n, c0 + _CHUNK)
        i = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            out[c0:c1] = mix64(b + i * GAMMA)
    return out


def words(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """word(seed, stream, i) for i in [start, start + n) as uint64 (C fast path)."""
    out = np.empty(n, dtype=np.uint64)
    if n:
        _fast().gen_words(int(base(seed, stream)), start, n, out.ctypes.data)
    return out


def _narrow(w: np.ndarray, key_bits: int) -> np.ndarray:
    if key_bits == 64:
        return w
    if key_bits == 32:
        return (w >> np.uint64(32)).astype(np.uint32)
    raise ValueError("key_bits must be 32 or 64")


def uniform(seed: int, n: int, key_bits: int = 32, stream: int = 1) -> np.ndarray:
    """Uniform keys: the entropy band q = 1."""
    if key_bits == 32:
        out = np.empty(n, dtype=np.uint32)
        if n:
            _fast().gen_words_hi32(int(base(seed, stream)), 0, n, out.ctypes.data)
        return out
    return _narrow(words(seed, stream, n), key_bits)


def and_of_q(seed: int, q: int, n: int, key_bits: int = 32) -> np.ndarray:
    """Bitwise AND of q independent uniform words (streams 1..q).

    Each bit is set with probability 2^-q, so the entropy per bit is
    H(2^-q) with H the binary entropy (Section 4 and Table 1).
    """
    if q < 1:
        raise ValueError("q >= 1")
    out = uniform(seed, n, key_bits, stream=1)
    if n:
        f = _fast().gen_and_words_hi32 if key_bits == 32 else _fast().gen_and_words
        for k in range(2, q + 1):
            f(int(base(seed, k)), 0, n, out.ctypes.data)
    return out


def all_equal(seed: int, n: int, key_bits: int = 32) -> np.ndarray:
    """Every key equal to word(seed, 9, 0)."""
    v = _narrow(words(seed, 9, 1), key_bits)[0]
    return np.full(n, v, dtype=v.dtype)


def unit_doubles(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Doubles in (0, 1): the top 53 bits of each word, offset by half an ulp."""
    w = words(seed, stream, n, start)
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / (1 << 53))


def zipf_keys(seed: int, n: int, key_bits: int = 32, s: float = 1.1,
              support: int = 1 << 20) -> np.ndarray:
    """Zipf(s) over ranks 1..support; key = rank - 1 (inverse CDF, binary search)."""
    ranks = np.arange(1, support + 1, dtype=np.float64)
    cdf = np.cumsum(ranks ** (-s))
    cdf /= cdf[-1]
    u = unit_doubles(seed, 1, n)
    k = np.searchsorted(cdf, u, side="left")
    k = np.minimum(k, support - 1)
    return k.astype(np.uint32 if key_bits == 32 else np.uint64)


def presorted(seed: int, n: int, key_bits: int = 32) -> np.ndarray:
    return np.sort(uniform(seed, n, key_bits))


def reverse_sorted(seed: int, n: int, key_bits: int = 32) -> np.ndarray:
    return np.sort(uniform(seed, n, key_bits))[::-1].copy()


def distinct16(seed: int, n: int, key_bits: int = 32) -> np.ndarray:
    """16 distinct values word(seed, 100, 0..15); index = top 4 bits of word(seed, 1, i)."""
    table = _narrow(words(seed, 100, 16), key_bits)
    idx = (words(seed, 1, n) >> np.uint64(60)).astype(np.int64)
    return table[idx]


def runs(seed: int, n: int, key_bits: int = 32, run: int = 1 << 16, low_bits: int = 8,
         last_high_ones: bool = False) -> np.ndarray:
    """Keys whose bits above `low_bits` are constant over runs of `run`
    consecutive indices (drawn once per run from stream 2); the low bits are
    uniform (stream 1). With `last_high_ones` the last, possibly partial, run
    has every high bit set."""
    w = uniform(seed, n, key_bits, stream=1)
    runs_n = -(-n // run) if n else 0
    high = uniform(seed, runs_n, key_bits, stream=2)
    if last_high_ones and runs_n:
        high[-1] = np.iinfo(high.dtype).max
    one = np.array(1, dtype=w.dtype)
    low = (one << np.array(low_bits, dtype=w.dtype)) - one
    return (np.repeat(high, run)[:n] & ~low) | (w & low)


def signed_ints(seed: int, n: int, key_bits: int = 32, span_bits: int = 12) -> np.ndarray:
    """Raw bits of two's-complement integers in [-2^(span_bits-1), 2^(span_bits-1)):
    the top span_bits of a uniform word, sign-extended (ties and both signs)."""
    w = uniform(seed, n, key_bits)
    st = np.int32 if key_bits == 32 else np.int64
    return (w.view(st) >> (key_bits - span_bits)).view(w.dtype)


def float_bits(seed: int, n: int, key_bits: int = 32) -> np.ndarray:
    """Raw bits of IEEE 754 values: finite values of both signs over many
    magnitudes, with one key in 16 drawn from the special values (signed
    zeros, infinities, NaNs of both signs, smallest subnormals, extremes)."""
    ft = np.float32 if key_bits == 32 else np.float64
    u = unit_doubles(seed, 1, n)
    e = (words(seed, 2, n) >> np.uint64(59)).astype(np.int64) - 16  # decades -16..15
    x = ((u * 2.0 - 1.0) * 10.0 ** e).astype(ft)
    out = x.view(np.uint32 if key_bits == 32 else np.uint64).copy()
    if key_bits == 32:
        specials = np.array([0x00000000, 0x80000000, 0x7F800000, 0xFF800000, 0x7FC00000,
                             0xFFC00000, 0x00000001, 0x80000001, 0x7F7FFFFF, 0xFF7FFFFF,
                             0x3F800000, 0xBF800000, 0x7F800001, 0xFF800123, 0x00800000,
                             0x80800000], dtype=np.uint32)
    else:
        specials = np.array([0x0, 0x8000000000000000, 0x7FF0000000000000, 0xFFF0000000000000,
                             0x7FF8000000000000, 0xFFF8000000000000, 0x1, 0x8000000000000001,
                             0x7FEFFFFFFFFFFFFF, 0xFFEFFFFFFFFFFFFF, 0x3FF0000000000000,
                             0xBFF0000000000000, 0x7FF0000000000001, 0xFFF0000000000123,
                             0x0010000000000000, 0x8010000000000000], dtype=np.uint64)
    pick = words(seed, 3, n)
    special = (pick & np.uint64(15)) == np.uint64(0)
    out[special] = specials[((pick[special] >> np.uint64(4)) & np.uint64(15)).astype(np.int64)]
    return out


DISTRIBUTIONS = ("and1", "and2", "and3", "and4", "zipf", "presorted", "reverse", "distinct16")


def make_keys(dist: str, seed: int, n: int, key_bits: int = 32) -> np.ndarray:
    """Keys of one named distribution of the learned-config sweep."""
    if dist.startswith("and"):
        return and_of_q(seed, int(dist[3:]), n, key_bits)
    if dist == "uniform":
        return uniform(seed, n, key_bits)
    if dist == "zipf":
        return zipf_keys(seed, n, key_bits)
    if dist == "presorted":
        return presorted(seed, n, key_bits)
    if dist == "reverse":
        return reverse_sorted(seed, n, key_bits)
    if dist == "distinct16":
        return distinct16(seed, n, key_bits)
    if dist == "equal":
        return all_equal(seed, n, key_bits)
    raise ValueError(f"unknown distribution {dist!r}")


def sweep_case(seed: int):
    """(n, key_bits, dist) of one learned-config sweep input.

    n = round(2^(17 + 11 u)) with u from word(seed, 300, 0); key widths alternate
    between 32 and 64 bits and distributions cycle over DISTRIBUTIONS by seed.
    """
    u = float(unit_doubles(seed, 300, 1)[0])
    n = int(round(2.0 ** (17.0 + 11.0 * u)))
    key_bits = 32 if seed % 2 == 0 else 64
    dist = DISTRIBUTIONS[(seed // 2) % len(DISTRIBUTIONS)]
    return n, key_bits, dist


def lognormal_segment_lengths(num_segments: int = 20000, median: float = 2000.0,
                              sigma: float = 1.5, cap: int = 1 << 22, seed: int = 4,
                              total: int | None = 1 << 26) -> np.ndarray:
    """Segment lengths L_s = min(cap, round(exp(ln(median) + sigma * z_s))).

    z_s is a standard normal from Box-Muller on consecutive unit doubles of
    stream 200. When `total` is given, every length is scaled by one common
    factor and rounded so that the lengths add up to `total` exactly (largest
    remainders receive the leftover units, ties broken by lower index).
    """
    u = unit_doubles(seed, 200, 2 * num_segments)
    u1, u2 = u[0::2], u[1::2]
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    raw = np.minimum(float(cap), np.rint(np.exp(math.log(median) + sigma * z)))
    if total is None:
        return raw.astype(np.int64)
    scaled = raw * (float(total) / raw.sum())
    base_len = np.floor(scaled).astype(np.int64)
    short = int(total - base_len.sum())
    if short > 0:
        frac = scaled - base_len
        order = np.lexsort((np.arange(num_segments), -frac))
        base_len[order[:short]] += 1
    return base_len


def offsets_from_lengths(lengths: np.ndarray) -> np.ndarray:
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return off


def binary_entropy(p: float) -> float:
    if p <= 0.0 or p >= 1.0:
        return 0.0
    return -(p * math.log2(p) + (1 - p) * math.log2(1 - p))


def per_bit_entropy(keys: np.ndarray) -> float:
    """Mean over bit positions of the empirical binary entropy of that bit."""
    bits = keys.dtype.itemsize * 8
    ks = keys.astype(np.uint64)
    h = 0.0
    for b in range(bits):
        p1 = float(np.count_nonzero((ks >> np.uint64(b)) & np.uint64(1))) / len(ks)
        h += binary_entropy(p1)
    return h / bits
