"""Multithreaded CPU LSD radix sort (OpenMP, all host cores): the benchmark's
secondary CPU baseline. Benchmark infrastructure only: the HIP library and its
binding never import it. It is checked against the oracle in
tests/test_cpu_baseline.py.

The sort itself is plain C (`lsd_omp.c`, gcc -O3 -fopenmp, `liblsd_omp.so`);
this module marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsd_omp.c")
_LIB = os.path.join(_HERE, "liblsd_omp.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
                               "-Werror", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build(force=False))
        vp = ctypes.c_void_p
        L.cpu_lsd_sort.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_size_t, ctypes.c_int]
        L.cpu_lsd_sort.restype = ctypes.c_int
        L.cpu_lsd_default_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def sort(keys: np.ndarray, vals: np.ndarray | None = None, threads: int = 0):
    """Stable ascending sort of uint32/uint64 keys (and uint32 values) on
    `threads` host threads (0 = all). Returns (keys, values or None)."""
    keys = np.ascontiguousarray(keys)
    assert keys.dtype in (np.uint32, np.uint64)
    out_k = np.empty_like(keys)
    out_v = None
    vp = None
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
        assert vals.shape == keys.shape
        out_v = np.empty_like(vals)
        vp = vals.ctypes.data
    rc = lib().cpu_lsd_sort(keys.ctypes.data, out_k.ctypes.data, vp,
                            None if out_v is None else out_v.ctypes.data,
                            8 * keys.itemsize, keys.size, threads)
    if rc:
        raise RuntimeError(f"cpu_lsd_sort failed with code {rc}")
    return out_k, out_v


def threads_used(threads: int = 0) -> int:
    """Threads a call with `threads` runs on (OpenMP's default when 0)."""
    return threads if threads > 0 else int(lib().cpu_lsd_default_threads())
