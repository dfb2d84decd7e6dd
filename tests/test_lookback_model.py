"""The chained scan's status-word protocol, run on the host.

The host model (`oracle/lookback_model.c`) plays the decoupled look-back of
the digit-binning kernel (Section 3, Figures 6 and 7) with tiles as steps of a
chosen schedule, as a seeded random interleaving, and as real threads with
random delays and a stalled tile (also under the thread sanitizer). Whatever
the order, every tile's exclusive prefix must equal a sequential exclusive scan
of the tile counts, and every final word must be G with the inclusive prefix.
Nothing here runs on a GPU.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from conftest import read_golden
from oracle import lookback as LB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _want(counts):
    counts = np.asarray(counts, dtype=np.uint64)
    incl = np.cumsum(counts, axis=0, dtype=np.uint64)
    return incl - counts, incl


def _check_final(counts, words, excl):
    want_ex, want_in = _want(counts)
    st, val = LB.unpack(words)
    assert np.array_equal(excl, want_ex)
    assert np.all(st == LB.STATUS_G)
    assert np.array_equal(val.astype(np.uint64), want_in)


def test_figure7_timeline():
    """Section 3, Figure 7 (b)-(f): one digit over five tiles, each tile
    reading one predecessor word per step; tile 0 first shows its local count."""
    g = read_golden("lookback_fig7.txt")
    counts = g["local_counts"]
    steps = [0, 1, 3, 4, 3,      # (b): #0, #1, #3, #4 publish L; #3 finds #2 not ready
             0, 1, 2, 3, 4,      # (c): #0, #1 reach G; #2 publishes L; #3, #4 add one L each
             2, 3,               # (d): #2 and #3 meet G at #1
             4]                  # (e): #4 meets G at #2
    snaps, results, partial, excl = LB.schedule(counts, steps, window=1, first_publishes_g=False)
    assert results[4] == LB.BLOCKED  # tile 3 waits on tile 2
    for label, at in (("b", 4), ("c", 9), ("d", 11), ("e", 12)):
        st, val = LB.unpack(snaps[at])
        assert st.tolist() == g[f"{label}_status"], label
        assert val.tolist() == g[f"{label}_value"], label
    assert partial[9, 3:5].tolist() == g["c_partial_tile3_tile4"]
    assert excl[4] == g["exclusive_of_tile_4"][0]
    assert LB.unpack(snaps[-1])[1].tolist() == g["inclusive"]
    assert excl.tolist() == [0, 11, 26, 35, 45]


def test_figure7_values_with_a_window_and_first_tile_shortcut():
    """Reading four predecessors per round trip and letting tile 0 publish G at
    once (what the kernel does) reach the same final state."""
    g = read_golden("lookback_fig7.txt")
    counts = g["local_counts"]
    steps = [4, 3, 2, 1, 0] + [4, 3, 2, 1] * 6
    snaps, _, _, excl = LB.schedule(counts, steps, window=4, first_publishes_g=True)
    st, val = LB.unpack(snaps[-1])
    assert st.tolist() == [2] * 5
    assert val.tolist() == g["inclusive"]
    assert excl[4] == g["exclusive_of_tile_4"][0]


def test_sequential_tiles_never_wait():
    """One tile in flight at a time: every walk finds G at its predecessor."""
    counts = np.random.default_rng(5).integers(0, 300, size=(40, 6), dtype=np.uint32)
    rc, words, excl, stats = LB.random_interleaving(counts, window=1, in_flight=1, seed=3)
    assert rc == 0 and stats[1] == 0 and stats[2] == 1
    _check_final(counts, words, excl)


@pytest.mark.parametrize("window", [1, 2, 4, 7])
@pytest.mark.parametrize("first_g", [False, True])
def test_random_interleavings(window, first_g):
    rng = np.random.default_rng(100 + window)
    for seed in range(12):
        tiles = int(rng.choice([1, 2, 5, 33, 200]))
        digits = int(rng.choice([1, 3, 8]))
        counts = rng.integers(0, 1000, size=(tiles, digits), dtype=np.uint32)
        counts[rng.random(counts.shape) < 0.3] = 0  # empty digits are common
        in_flight = int(rng.choice([2, 8, 64]))
        stalled = int(rng.integers(0, tiles)) if seed % 2 else -1
        rc, words, excl, stats = LB.random_interleaving(
            counts, window=window, first_publishes_g=first_g, in_flight=in_flight, seed=seed,
            stalled_tile=stalled, stall_steps=5000)
        assert rc == 0
        _check_final(counts, words, excl)


def test_stalled_tile_makes_successors_wait_then_finishes():
    counts = np.random.default_rng(9).integers(1, 50, size=(64, 4), dtype=np.uint32)
    rc, words, excl, stats = LB.random_interleaving(counts, window=4, in_flight=16, seed=11,
                                                    stalled_tile=10, stall_steps=20000)
    assert rc == 0
    assert stats[1] > 1000  # successors of the stalled tile read not-ready words
    assert stats[2] > 4     # some walk went past one window before it met G
    _check_final(counts, words, excl)


def test_spin_limit_reports_a_wait_that_would_not_end():
    counts = np.ones((50, 2), dtype=np.uint32)
    rc, _, _, stats = LB.random_interleaving(counts, window=4, in_flight=8, seed=2,
                                             stalled_tile=3, stall_steps=10 ** 9,
                                             spin_limit=1000)
    assert rc == 1


def test_values_up_to_the_30_bit_limit():
    """Inclusive prefixes reach 2^30 - 1, the largest value a word holds (Figure 6)."""
    top = (1 << 30) - 1
    counts = np.array([[top - 3000], [1000], [1000], [999], [1]], dtype=np.uint32)
    rc, words, excl, _ = LB.random_interleaving(counts, window=2, in_flight=5, seed=4)
    assert rc == 0
    _check_final(counts, words, excl)
    assert int(LB.unpack(words)[1][-1, 0]) == top


@pytest.mark.parametrize("window,first_g,n_threads", [(4, True, 16), (1, False, 8), (2, True, 32)])
def test_threads_with_delays_and_a_stalled_tile(window, first_g, n_threads):
    counts = np.random.default_rng(window).integers(0, 500, size=(400, 8), dtype=np.uint32)
    rc, words, excl, blocked = LB.threads(counts, n_threads=n_threads, window=window,
                                          first_publishes_g=first_g, seed=window, max_delay_us=30,
                                          stalled_tile=57, stall_us=20000)
    assert rc == 0
    assert blocked > 0
    _check_final(counts, words, excl)


def test_threads_spin_limit_stops_every_thread():
    counts = np.ones((200, 2), dtype=np.uint32)
    rc, _, _, _ = LB.threads(counts, n_threads=8, window=4, seed=3, max_delay_us=0,
                             stalled_tile=5, stall_us=300000, spin_limit=200)
    assert rc == 1


def test_threads_under_thread_sanitizer(tmp_path):
    exe = LB.build_tsan(str(tmp_path / "lookback_tsan"))
    for args in (["300", "16", "8", "4", "1", "7", "50", "37", "20000"],
                 ["200", "4", "16", "1", "0", "9", "20", "5", "30000"],
                 ["1000", "2", "32", "2", "1", "13", "0", "-1", "0"]):
        r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300,
                           env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
        assert r.returncode == 0, r.stderr[-3000:]
        assert "ThreadSanitizer" not in r.stderr, r.stderr[-3000:]
        assert r.stdout.startswith("ok:")


MUTANTS = {
    "not_ready_read_as_zero": ("            if (s == LB_N) break;\n", "\n"),
    "walk_goes_past_g": ("            found = s == LB_G;", "            found = 0;"),
    "own_count_left_out": ("lb_word(LB_G, (uint32_t)(w->sum + count))",
                           "lb_word(LB_G, (uint32_t)(w->sum))"),
    "window_skips_nearest": ("seen[i] = w->next - i >= 0 ? lb_load(m, w->next - i, d)",
                             "seen[i] = w->next - i - 1 >= 0 ? lb_load(m, w->next - i - 1, d)"),
    "status_below_bit_30": ("return (status << 30) | (value & LB_VALUE_MASK);",
                            "return (status << 29) | (value & LB_VALUE_MASK);"),
    "walk_skips_not_ready": ("            if (s == LB_N) break;", "            if (s == LB_N) continue;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_model_tests_catch_planted_mistake(name, tmp_path):
    if os.environ.get("ONESWEEP_LOOKBACK_LIB"):
        pytest.skip("already running against a mutant")
    old, new = MUTANTS[name]
    src = open(LB.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/present"
    mutant = tmp_path / "lookback_mutant.c"
    mutant.write_text(src.replace(old, new))
    so = tmp_path / "liblookback_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", str(mutant), "-o",
                           str(so), "-lpthread"])
    env = dict(os.environ, ONESWEEP_LOOKBACK_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-k", "not sanitizer and not planted",
                        os.path.join(ROOT, "tests", "test_lookback_model.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"model tests did not catch mutant {name}:\n{r.stdout[-2000:]}"
