"""Host model of the chained scan with decoupled look-back: TEST INFRASTRUCTURE ONLY.

The model (`lookback_model.c`, plain C11 with POSIX threads) runs the
status-word protocol of the digit-binning kernel (Section 3, Figures 6 and 7)
on the CPU under chosen, seeded-random and truly concurrent schedules, so the
tests can check that every tile's exclusive prefix equals a sequential scan of
the tile counts whatever order the tiles run in. Like the rest of `oracle/`,
only tests import it, and it shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "lookback_model.c")
_LIB = os.path.join(_HERE, "liblookback.so")

PROGRESS, BLOCKED, DONE = 0, 1, 2
STATUS_N, STATUS_L, STATUS_G = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile lookback_model.c into liblookback.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Werror",
                               SRC, "-o", tmp, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def build_tsan(out_path: str) -> str:
    """The stand-alone driver built with the thread sanitizer (host code only)."""
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-fsanitize=thread",
                           "-DLOOKBACK_MODEL_MAIN", SRC, "-o", out_path, "-lpthread"])
    return out_path


_lib = None


def lib():
    global _lib
    if _lib is None:
        # The mutation tests point this at a deliberately broken build.
        path = os.environ.get("ONESWEEP_LOOKBACK_LIB") or build(force=False)
        L = ctypes.CDLL(path)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_uint64
        L.lookback_model_schedule.argtypes = [vp, i32, i32, i32, vp, i32, vp, vp, vp, vp]
        L.lookback_model_schedule.restype = i32
        L.lookback_model_random.argtypes = [vp, i32, i32, i32, i32, i32, u64, i32, i64, i64, vp,
                                            vp, vp]
        L.lookback_model_random.restype = i32
        L.lookback_model_threads.argtypes = [vp, i32, i32, i32, i32, i32, u64, i32, i32, i32, i64,
                                             vp, vp, vp]
        L.lookback_model_threads.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def unpack(words: np.ndarray):
    """(status, value) arrays of packed 32-bit words (Figure 6)."""
    words = np.asarray(words, dtype=np.uint32)
    return words >> np.uint32(30), words & np.uint32((1 << 30) - 1)


def schedule(counts, steps, window: int = 1, first_publishes_g: bool = False):
    """Replay single steps of one digit's chained scan; `steps` lists the tile
    that moves at each step. Returns (snapshots [steps, tiles] of status words,
    results [steps], partial sums [steps, tiles], exclusive prefixes [tiles];
    a tile that never finished has exclusive 2^64 - 1)."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    g, s = counts.size, steps.size
    snaps = np.zeros((s, g), dtype=np.uint32)
    results = np.zeros(s, dtype=np.int32)
    partial = np.zeros((s, g), dtype=np.uint64)
    excl = np.zeros(g, dtype=np.uint64)
    rc = lib().lookback_model_schedule(_p(counts), g, window, int(first_publishes_g), _p(steps), s,
                                       _p(snaps), _p(results), _p(partial), _p(excl))
    if rc != 0:
        raise ValueError(f"lookback_model_schedule returned {rc}")
    return snaps, results, partial, excl


def random_interleaving(counts, window: int = 4, first_publishes_g: bool = True,
                        in_flight: int = 8, seed: int = 1, stalled_tile: int = -1,
                        stall_steps: int = 0, spin_limit: int = 1 << 40):
    """Seeded random interleaving of the tiles of counts[tiles, digits].
    Returns (rc, final words, exclusive prefixes, stats[steps, blocked, longest walk])."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    tiles, digits = counts.shape
    words = np.zeros_like(counts)
    excl = np.zeros(counts.shape, dtype=np.uint64)
    stats = np.zeros(3, dtype=np.uint64)
    rc = lib().lookback_model_random(_p(counts), tiles, digits, window, int(first_publishes_g),
                                     in_flight, seed, stalled_tile, stall_steps, spin_limit,
                                     _p(words), _p(excl), _p(stats))
    if rc < 0:
        raise ValueError(f"lookback_model_random returned {rc}")
    return rc, words, excl, stats


def threads(counts, n_threads: int = 8, window: int = 4, first_publishes_g: bool = True,
            seed: int = 1, max_delay_us: int = 20, stalled_tile: int = -1, stall_us: int = 0,
            spin_limit: int = 1 << 40):
    """Host threads as workgroups over counts[tiles, digits].
    Returns (rc, final words, exclusive prefixes, not-ready reads)."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    tiles, digits = counts.shape
    words = np.zeros_like(counts)
    excl = np.zeros(counts.shape, dtype=np.uint64)
    stats = np.zeros(1, dtype=np.uint64)
    rc = lib().lookback_model_threads(_p(counts), tiles, digits, n_threads, window,
                                      int(first_publishes_g), seed, max_delay_us, stalled_tile,
                                      stall_us, spin_limit, _p(words), _p(excl), _p(stats))
    if rc < 0 or rc == 2:
        raise ValueError(f"lookback_model_threads returned {rc}")
    return rc, words, excl, int(stats[0])
