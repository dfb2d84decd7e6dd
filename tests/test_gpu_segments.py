"""GPU parity of the batched segmented sort against the per-segment oracle.

Bit-exact: every segment of the output must equal the oracle's stable sort of
that segment. Segment lengths are chosen to hit every class boundary of the
LDS kernels (512, 2048, 8192 keys), the binning tile of the large segments,
empty and one-key segments, and the log-normal length mix of the batched
workload.
"""
import ctypes

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


# Lengths at and around every class limit and tile size, plus empty segments.
EDGE_LENGTHS = [0, 1, 2, 63, 64, 65, 0, 511, 512, 513, 1000, 2047, 2048, 2049, 0, 4096, 8191,
                8192, 8193, 8192 * 3 + 5, 16384, 1, 40000, 0]


def edge_offsets(reps: int = 1, seed: int = 0):
    lengths = list(EDGE_LENGTHS) * reps
    rng_words = W.words(seed, 77, len(lengths))
    order = np.argsort(rng_words, kind="stable")  # shuffle with the seeded generator
    lengths = np.array(lengths, dtype=np.int64)[order]
    return W.offsets_from_lengths(lengths)


def keys_for(kb, n, seed, dist="uniform"):
    return W.uniform(seed, n, kb) if dist == "uniform" else W.make_keys(dist, seed, n, kb)


def temp_error_flag(temp: torch.Tensor) -> int:
    return int(host(temp[:4]).view(np.uint32)[0])


def temp_wait_flag(temp: torch.Tensor) -> int:
    """Word 6 of the plan: bit 0 set by a binning tile that gave up waiting
    (for its predecessors' prefixes or for its segment's digit counts), bit 1
    by a tile whose destination run of a digit fell outside the keys (it then
    writes nothing)."""
    return int(host(temp[24:28]).view(np.uint32)[0])


def run(ow, keys, off, vals=None, begin=0, end=None, config=None, in_place=False, temp=None):
    """Sort on the GPU; returns (keys, vals, temp)."""
    kb = keys.dtype.itemsize * 8
    end = kb if end is None else end
    tk = dev(keys)
    tv = dev(vals) if vals is not None else None
    to = dev(off.astype(np.uint32))
    if temp is None:
        need = ow.sort_segments_temp_bytes(keys.size, off.size - 1, kb, vals is not None, begin,
                                           end, config)
        temp = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    kwargs = dict(begin_bit=begin, end_bit=end, temp=temp, config=config)
    if in_place:
        kwargs.update(keys_out=tk, values_out=tv)
    r = ow.sort_segments(tk, to, tv, **kwargs)
    torch.cuda.synchronize()
    if vals is None:
        return host(r), None, temp
    return host(r[0]), host(r[1]), temp


def check(ow, keys, off, vals=None, begin=0, end=None, config=None, in_place=False, what=""):
    kb = keys.dtype.itemsize * 8
    end = kb if end is None else end
    got_k, got_v, temp = run(ow, keys, off, vals, begin, end, config, in_place)
    want_k, want_v = oracle.sort_segments(keys, off, vals, begin, end, 8)
    if keys.size:  # the status word is not written for n == 0
        assert temp_error_flag(temp) == 0, what
        assert temp_wait_flag(temp) == 0, what
    bad = np.flatnonzero(got_k != want_k)
    assert bad.size == 0, (what, bad[:10], got_k[bad[:5]], want_k[bad[:5]])
    if vals is not None:
        assert np.array_equal(got_v, want_v), what


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("with_vals", [False, True])
def test_segments_every_class_boundary(ow, kb, with_vals):
    off = edge_offsets(reps=2, seed=kb + with_vals)
    n = int(off[-1])
    keys = keys_for(kb, n, 5)
    vals = np.arange(n, dtype=np.uint32) if with_vals else None
    check(ow, keys, off, vals, what=(kb, with_vals))


LIMITS = [(0, 0, 0), (-1, -1, -1), (-1, -1, 0), (100, 1000, 5000), (512, -1, 8192),
          (1, 2, 3)]


@pytest.mark.parametrize("kb", [32, 64])
def test_segments_one_stream_and_two_streams_agree(ow, kb):
    """The LDS classes on the second stream (default) and everything on the
    caller's stream give the same, oracle-exact result."""
    off = edge_offsets(reps=3, seed=kb)
    n = int(off[-1])
    keys = keys_for(kb, n, 12)
    vals = np.arange(n, dtype=np.uint32)
    check(ow, keys, off, vals, config=ow.make_config(segment_streams=1), what="one stream")
    check(ow, keys, off, vals, config=ow.make_config(segment_streams=0), what="two streams")
    # a non-default stream of the caller
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got_k, got_v, _ = run(ow, keys, off, vals)
    want_k, want_v = oracle.sort_segments(keys, off, vals)
    assert np.array_equal(got_k, want_k) and np.array_equal(got_v, want_v)


@pytest.mark.parametrize("limits", LIMITS)
@pytest.mark.parametrize("kb,shape", [(32, (256, 8)), (32, (256, 16)), (32, (512, 16)),
                                      (32, (1024, 8)), (32, (1024, 11)), (32, (1024, 16)),
                                      (32, (1024, 19)), (64, (256, 8)), (64, (512, 8)), (64, (256, 16)),
                                      (64, (1024, 9)), (64, (1024, 14))])
def test_segments_class_limits_and_tiles(ow, limits, kb, shape):
    cfg = ow.make_config(block_threads=shape[0], items_per_thread=shape[1],
                         segment_limits=limits)
    off = edge_offsets(reps=1, seed=sum(limits) & 0xFF)
    n = int(off[-1])
    keys = keys_for(kb, n, 6)
    vals = np.arange(n, dtype=np.uint32)
    check(ow, keys, off, vals, config=cfg, what=(limits, kb, shape))


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("dist", ["and4", "equal", "distinct16", "zipf", "presorted",
                                  "reverse"])
def test_segments_distributions(ow, kb, dist):
    off = edge_offsets(reps=1, seed=9)
    n = int(off[-1])
    keys = keys_for(kb, n, 7, dist)
    check(ow, keys, off, np.arange(n, dtype=np.uint32), what=dist)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("with_vals", [False, True])
def test_segments_one_digit_tiles(ow, kb, with_vals):
    """Large segments whose tiles share their high digits (runs of 4096 and
    8192 keys) take the short-circuit write; the last run has every high bit
    set, the digit of the padding lanes."""
    off = edge_offsets(reps=2, seed=21)
    n = int(off[-1])
    vals = np.arange(n, dtype=np.uint32) if with_vals else None
    for run_len in (4096, 8192):
        keys = W.runs(23, n, kb, run=run_len, low_bits=8, last_high_ones=True)
        for shape in ((256, 16), (1024, 8)):
            cfg = ow.make_config(block_threads=shape[0], items_per_thread=shape[1],
                                 segment_limits=(-1, -1, -1))
            check(ow, keys, off, vals, config=cfg, what=(run_len, shape))


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("in_place", [False, True])
def test_segments_partial_bit_ranges(ow, kb, in_place):
    off = edge_offsets(reps=1, seed=3)
    n = int(off[-1])
    keys = keys_for(kb, n, 8)
    vals = np.arange(n, dtype=np.uint32)
    # p = 3 (odd: the in-place path ends with a copy), 2, 1 and 0 places
    for begin, end in [(4, 28), (0, 12), (kb - 9, kb - 1), (8, 9), (5, 5)]:
        check(ow, keys, off, vals, begin, end, in_place=in_place, what=(begin, end, in_place))
        check(ow, keys, off, None, begin, end, in_place=in_place, what=(begin, end, in_place))


def test_segments_in_place_full_width(ow):
    for kb in (32, 64):
        off = edge_offsets(reps=1, seed=4)
        n = int(off[-1])
        keys = keys_for(kb, n, 9)
        check(ow, keys, off, np.arange(n, dtype=np.uint32), in_place=True, what=kb)
        check(ow, keys, off, None, in_place=True, what=kb)


def test_segments_degenerate(ow):
    # one segment covering everything equals the plain sort
    keys = W.uniform(10, 100003)
    off = np.array([0, keys.size], dtype=np.int64)
    got, _, _ = run(ow, keys, off)
    assert np.array_equal(got, oracle.sort(keys)[0])
    # only empty segments around a few keys; many one-key segments
    check(ow, W.uniform(11, 5), np.array([0, 0, 0, 2, 2, 5, 5], dtype=np.int64))
    check(ow, W.uniform(12, 3000), np.arange(3001, dtype=np.int64))
    # no keys at all
    check(ow, W.uniform(13, 0), np.zeros(4, dtype=np.int64))
    # segments made only of large ones
    check(ow, W.uniform(14, 3 * 8193), np.array([0, 8193, 2 * 8193, 3 * 8193], dtype=np.int64))


def test_segments_lognormal_mix(ow):
    lengths = W.lognormal_segment_lengths(num_segments=2000, total=1 << 22, seed=4)
    off = W.offsets_from_lengths(lengths)
    n = int(off[-1])
    keys = W.uniform(4, n)
    check(ow, keys, off, np.arange(n, dtype=np.uint32), what="lognormal")


def test_segments_bounded_waits(ow):
    """The first place's launch counts every place's digits and bins: its
    binning tiles wait until their segment's counts add up to its length.
    With the default limit no wait gives up and the sort matches the oracle;
    with a limit of one poll the tiles of a 2^22-key segment give up waiting
    (for counts or predecessors), record it in the plan, and still end."""
    off = np.array([0, 1 << 22, (1 << 22) + 3000], dtype=np.int64)
    n = int(off[-1])
    keys = W.uniform(91, n)
    check(ow, keys, off, what="default limit")
    _, _, temp = run(ow, keys, off, config=ow.make_config(lookback_spin_limit=1))
    assert temp_error_flag(temp) == 0
    assert temp_wait_flag(temp) & 1 == 1


def test_segments_invalid_offsets_write_nothing(ow):
    n = 20000
    keys = W.uniform(15, n)
    for off in (np.array([0, 5000, 4000, n]),          # decreasing
                np.array([0, 5000, n + 1]),             # beyond n
                np.array([1, 5000, n]),                 # does not start at 0
                np.array([0, 5000, n - 1])):            # does not end at n
        tk = dev(keys)
        out = torch.full_like(tk, 7)
        to = dev(off.astype(np.uint32))
        need = ow.sort_segments_temp_bytes(n, off.size - 1)
        temp = torch.empty(need, dtype=torch.uint8, device="cuda")
        ow.sort_segments(tk, to, keys_out=out, temp=temp)
        torch.cuda.synchronize()
        assert temp_error_flag(temp) == 1, off
        assert bool((out == 7).all()), off


def test_segments_trace_launch_sequence(ow):
    off = edge_offsets(reps=1, seed=1)
    n = int(off[-1])
    tk = dev(W.uniform(16, n))
    to = dev(off.astype(np.uint32))
    events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * 32)]
    for e in events:
        e.record()
    torch.cuda.synchronize()
    arr = (ctypes.c_void_p * len(events))(*[e.cuda_event for e in events])
    tr = ow.Trace()
    tr.events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    tr.capacity = 32
    ow.sort_segments(tk, to, config=ow.make_config(trace=tr))
    torch.cuda.synchronize()
    kinds = [tr.kinds[i] for i in range(tr.count)]
    # the first binning launch also counts every place's digits per segment:
    # no histogram or scan launch of its own
    assert kinds == [ow.KERNEL_CLASSIFY] + [ow.KERNEL_LDS_SORT] * 3 + \
        [ow.KERNEL_RESET] + [ow.KERNEL_BINNING] * 4


def test_segments_graph_capture_replays(ow):
    """One capture, replayed with new keys and new offsets (same n and
    segment count); eager sorts run between replays."""
    S = 300
    lengths = W.lognormal_segment_lengths(num_segments=S, total=1 << 20, seed=21)
    n = int(lengths.sum())
    static_k = torch.empty(n, dtype=torch.uint32, device="cuda")
    static_v = torch.empty(n, dtype=torch.uint32, device="cuda")
    static_off = torch.empty(S + 1, dtype=torch.uint32, device="cuda")
    out_k = torch.empty_like(static_k)
    out_v = torch.empty_like(static_v)
    temp = torch.empty(ow.sort_segments_temp_bytes(n, S, 32, True), dtype=torch.uint8,
                       device="cuda")
    off0 = W.offsets_from_lengths(lengths)
    static_k.copy_(dev(W.uniform(20, n)))
    static_v.copy_(dev(np.arange(n, dtype=np.uint32)))
    static_off.copy_(dev(off0.astype(np.uint32)))
    ow.sort_segments(static_k, static_off, static_v, keys_out=out_k, values_out=out_v, temp=temp)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ow.sort_segments(static_k, static_off, static_v, keys_out=out_k, values_out=out_v,
                             temp=temp, stream=s)
    torch.cuda.synchronize()
    for seed in (31, 32, 33, 34):
        keys = W.and_of_q(seed, 1 + seed % 3, n)
        # a different split of the same n into S segments
        lens = W.lognormal_segment_lengths(num_segments=S, total=n, seed=seed)
        off = W.offsets_from_lengths(lens)
        vals = np.arange(n, dtype=np.uint32)[::-1].copy()
        static_k.copy_(dev(keys))
        static_v.copy_(dev(vals))
        static_off.copy_(dev(off.astype(np.uint32)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        want_k, want_v = oracle.sort_segments(keys, off, vals)
        assert np.array_equal(host(out_k), want_k), seed
        assert np.array_equal(host(out_v), want_v), seed
        assert temp_error_flag(temp) == 0
        eager = ow.sort_segments(dev(keys), dev(off.astype(np.uint32)))
        torch.cuda.synchronize()
        assert np.array_equal(host(eager), want_k), seed


def test_segments_tuner_picks_a_built_config_and_sorts(ow):
    lengths = W.lognormal_segment_lengths(num_segments=1000, total=1 << 21, seed=22)
    off = W.offsets_from_lengths(lengths)
    n = int(off[-1])
    keys = W.uniform(22, n)
    vals = np.arange(n, dtype=np.uint32)
    tk, tv, to = dev(keys), dev(vals), dev(off.astype(np.uint32))
    ko, vo = torch.empty_like(tk), torch.empty_like(tv)
    cfg = ow.tune_segments(tk, to, tv, keys_out=ko, values_out=vo, repetitions=2)
    torch.cuda.synchronize()
    want_k, want_v = oracle.sort_segments(keys, off, vals)
    assert np.array_equal(host(ko), want_k)
    assert np.array_equal(host(vo), want_v)
    assert (cfg.block_threads, cfg.items_per_thread) in [(256, 8), (256, 16), (512, 16),
                                                         (1024, 8), (1024, 11), (1024, 16),
                                                         (1024, 19)]
    # the chosen config sorts the same data bit-exactly again
    k2, v2 = ow.sort_segments(tk, to, tv, config=cfg)
    torch.cuda.synchronize()
    assert np.array_equal(host(k2), want_k) and np.array_equal(host(v2), want_v)
