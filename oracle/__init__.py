"""CPU oracle for the Onesweep LSD radix sort: TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's CPU-baseline leg
may import this package. The product path (the HIP library and its binding)
never imports, links or calls it, and it imports nothing from the product.

The arithmetic lives in plain C (`oracle.c`, built with gcc into
`liboracle.so`); this module only marshals numpy arrays through ctypes.

Parity pins: every function here is checked by `tests/test_oracle_*.py`
against values the paper prints, closed forms, brute force and library
routines; see the test modules for which pin covers which function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS_N, STATUS_L, STATUS_G = 0, 1, 2
KEY_UNSIGNED, KEY_SIGNED, KEY_FLOAT = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Werror", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # The mutation tests point this at a deliberately broken build of
        # oracle.c to show that the pins catch planted mistakes.
        path = os.environ.get("ONESWEEP_ORACLE_LIB")
        if not path:
            path = build(force=False)
        L = ctypes.CDLL(path)
        vp, sz, i32, u64p = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p
        L.oracle_num_places.argtypes = [i32, i32, i32]
        L.oracle_num_places.restype = i32
        L.oracle_digit.argtypes = [ctypes.c_uint64, i32, i32, i32, i32]
        L.oracle_digit.restype = ctypes.c_uint64
        L.oracle_histograms.argtypes = [vp, i32, sz, i32, i32, i32, u64p]
        L.oracle_histograms.restype = i32
        L.oracle_exclusive_sums.argtypes = [u64p, i32, i32, u64p]
        L.oracle_exclusive_sums.restype = None
        L.oracle_inclusive_scan.argtypes = [u64p, sz, u64p]
        L.oracle_inclusive_scan.restype = None
        L.oracle_binning_pass.argtypes = [vp, vp, vp, vp, i32, sz, i32, i32, u64p]
        L.oracle_binning_pass.restype = i32
        L.oracle_sort.argtypes = [vp, vp, vp, vp, i32, sz, i32, i32, i32, vp]
        L.oracle_sort.restype = i32
        L.oracle_sort_segments.argtypes = [vp, vp, vp, vp, i32, sz, u64p, sz, i32, i32, i32]
        L.oracle_sort_segments.restype = i32
        L.oracle_ordered_bits.argtypes = [ctypes.c_uint64, i32, i32, i32]
        L.oracle_ordered_bits.restype = ctypes.c_uint64
        L.oracle_ordered_keys.argtypes = [vp, i32, sz, i32, i32, vp]
        L.oracle_ordered_keys.restype = i32
        L.oracle_sort_typed.argtypes = [vp, vp, vp, vp, i32, sz, i32, i32, i32, i32, i32]
        L.oracle_sort_typed.restype = i32
        L.oracle_sort_segments_typed.argtypes = [vp, vp, vp, vp, i32, sz, u64p, sz, i32, i32,
                                                 i32, i32, i32]
        L.oracle_sort_segments_typed.restype = i32
        L.oracle_pass_status.argtypes = [vp, i32, sz, i32, i32, sz, vp]
        L.oracle_pass_status.restype = i32
        L.oracle_status_pack.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.oracle_status_pack.restype = ctypes.c_uint32
        L.oracle_status_unpack.argtypes = [ctypes.c_uint32, vp, vp]
        L.oracle_status_unpack.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _key_bits(keys: np.ndarray) -> int:
    if keys.dtype == np.uint32:
        return 32
    if keys.dtype == np.uint64:
        return 64
    raise TypeError("keys must be uint32 or uint64")


def _check(rc: int):
    if rc != 0:
        raise ValueError(f"oracle error {rc}")


def num_places(begin_bit: int, end_bit: int, d: int) -> int:
    """p = ceil((end - begin) / d)."""
    return lib().oracle_num_places(begin_bit, end_bit, d)


def place_bits(begin_bit: int, end_bit: int, d: int, j: int):
    lo = begin_bit + j * d
    return lo, min(lo + d, end_bit) - lo


def digit(key: int, begin_bit: int, end_bit: int, d: int, j: int) -> int:
    return int(lib().oracle_digit(int(key), begin_bit, end_bit, d, j))


def histograms(keys: np.ndarray, begin_bit: int = 0, end_bit: int | None = None,
               d: int = 8) -> np.ndarray:
    """hist[j, v]: count of keys whose digit at place j is v (uint64, shape p x 2^d)."""
    keys = np.ascontiguousarray(keys)
    kb = _key_bits(keys)
    end_bit = kb if end_bit is None else end_bit
    p = num_places(begin_bit, end_bit, d)
    out = np.zeros((max(p, 0), 1 << d), dtype=np.uint64)
    if p > 0:
        _check(lib().oracle_histograms(_ptr(keys), kb, keys.size, begin_bit, end_bit, d,
                                       _ptr(out)))
    return out


def exclusive_sums(hist: np.ndarray) -> np.ndarray:
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    p, r = hist.shape
    d = int(r).bit_length() - 1
    out = np.zeros_like(hist)
    if p > 0:
        lib().oracle_exclusive_sums(_ptr(hist), p, d, _ptr(out))
    return out


def inclusive_scan(counts) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64))
    out = np.zeros_like(c)
    lib().oracle_inclusive_scan(_ptr(c), c.size, _ptr(out))
    return out


def binning_pass(keys: np.ndarray, lo: int, width: int, off_j: np.ndarray,
                 vals: np.ndarray | None = None):
    """One stable digit-binning iteration at bits [lo, lo + width)."""
    keys = np.ascontiguousarray(keys)
    kb = _key_bits(keys)
    off_j = np.ascontiguousarray(off_j, dtype=np.uint64)
    out_k = np.empty_like(keys)
    out_v = None
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
        out_v = np.empty_like(vals)
    _check(lib().oracle_binning_pass(_ptr(keys), _ptr(vals), _ptr(out_k), _ptr(out_v), kb,
                                     keys.size, lo, width, _ptr(off_j)))
    return out_k, out_v


def ordered_bits(keys: np.ndarray, key_type: int = KEY_UNSIGNED,
                 descending: bool = False) -> np.ndarray:
    """The order-preserving transform of raw key bits (uint32/uint64 arrays)."""
    keys = np.ascontiguousarray(keys)
    kb = _key_bits(keys)
    out = np.empty_like(keys)
    _check(lib().oracle_ordered_keys(_ptr(keys), kb, keys.size, key_type, int(descending),
                                     _ptr(out)))
    return out


def sort(keys: np.ndarray, vals: np.ndarray | None = None, begin_bit: int = 0,
         end_bit: int | None = None, d: int = 8, return_passes: bool = False,
         key_type: int = KEY_UNSIGNED, descending: bool = False):
    """Stable LSD radix sort of `keys` (and `vals`) by bits [begin_bit, end_bit).

    Keys are raw uint32/uint64 bits; key_type (unsigned, signed, IEEE float)
    and descending select the order through oracle_ordered_bits. Returns
    (keys_out, vals_out) or, with return_passes (unsigned ascending only),
    also the p per-pass outputs as an array of shape (p, n).
    """
    keys = np.ascontiguousarray(keys)
    kb = _key_bits(keys)
    end_bit = kb if end_bit is None else end_bit
    n = keys.size
    out_k = keys.copy()
    out_v = None
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
        out_v = vals.copy()
    if key_type != KEY_UNSIGNED or descending:
        if return_passes:
            raise ValueError("return_passes covers unsigned ascending sorts only")
        _check(lib().oracle_sort_typed(_ptr(keys), _ptr(vals), _ptr(out_k), _ptr(out_v), kb, n,
                                       begin_bit, end_bit, d, key_type, int(descending)))
        return out_k, out_v
    p = num_places(begin_bit, end_bit, d)
    passes = np.zeros((max(p, 0), n), dtype=keys.dtype) if return_passes else None
    _check(lib().oracle_sort(_ptr(keys), _ptr(vals), _ptr(out_k), _ptr(out_v), kb, n,
                             begin_bit, end_bit, d, _ptr(passes)))
    if return_passes:
        return out_k, out_v, passes
    return out_k, out_v


def sort_segments(keys: np.ndarray, seg_offsets: np.ndarray, vals: np.ndarray | None = None,
                  begin_bit: int = 0, end_bit: int | None = None, d: int = 8,
                  key_type: int = KEY_UNSIGNED, descending: bool = False):
    keys = np.ascontiguousarray(keys)
    kb = _key_bits(keys)
    end_bit = kb if end_bit is None else end_bit
    off = np.ascontiguousarray(seg_offsets, dtype=np.uint64)
    out_k = keys.copy()
    out_v = None
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
        out_v = vals.copy()
    if key_type != KEY_UNSIGNED or descending:
        _check(lib().oracle_sort_segments_typed(_ptr(keys), _ptr(vals), _ptr(out_k), _ptr(out_v),
                                                kb, keys.size, _ptr(off), off.size - 1,
                                                begin_bit, end_bit, d, key_type,
                                                int(descending)))
        return out_k, out_v
    _check(lib().oracle_sort_segments(_ptr(keys), _ptr(vals), _ptr(out_k), _ptr(out_v), kb,
                                      keys.size, _ptr(off), off.size - 1, begin_bit, end_bit,
                                      d))
    return out_k, out_v


def pass_status(keys: np.ndarray, lo: int, width: int, tile: int) -> np.ndarray:
    """Final status words of one chained-scan pass over `keys` (shape g x 2^width)."""
    keys = np.ascontiguousarray(keys)
    kb = _key_bits(keys)
    g = (keys.size + tile - 1) // tile
    out = np.zeros((g, 1 << width), dtype=np.uint32)
    _check(lib().oracle_pass_status(_ptr(keys), kb, keys.size, lo, width, tile, _ptr(out)))
    return out


def status_pack(status: int, value: int) -> int:
    return int(lib().oracle_status_pack(status, value))


def status_unpack(word: int):
    s, v = ctypes.c_uint32(), ctypes.c_uint32()
    lib().oracle_status_unpack(word, ctypes.byref(s), ctypes.byref(v))
    return int(s.value), int(v.value)
