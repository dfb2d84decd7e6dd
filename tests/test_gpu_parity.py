"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle.

Integer work, so the bar is bit-exact everywhere. Inputs come from the seeded
generators in `workload`; expected values come only from `oracle`.
"""
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


def keys_of(dist, seed, n, kb):
    if dist == "uniform":
        return W.uniform(seed, n, kb)
    return W.make_keys(dist, seed, n, kb)


# ------------------------------------------------------------------ phase 1

@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("dist", ["uniform", "and4", "equal", "distinct16"])
@pytest.mark.parametrize("n", [1, 1000, 3 * 4096 + 5, (1 << 20) + 123])
def test_histogram_parity(ow, kb, dist, n):
    keys = keys_of(dist, 31, n, kb)
    for begin, end in [(0, kb), (3, kb - 5), (kb - 8, kb), (4, 9)]:
        got = host(ow.histogram(dev(keys), begin, end)).astype(np.uint64)
        want = oracle.histograms(keys, begin, end, 8)
        assert np.array_equal(got, want), (dist, n, begin, end)


@pytest.mark.parametrize("kb", [32, 64])
def test_histogram_of_constant_runs(ow, kb):
    """Runs of equal keys (of 64, 100 and 4096 keys, some aligned with
    waves, some not) mix waves whose keys are all equal with mixed waves."""
    n = 3 * 65536 + 77
    for run in (64, 100, 4096):
        keys = W.runs(37 + run, n, kb, run=run, low_bits=0)
        for begin, end in [(0, kb), (5, kb - 3)]:
            got = host(ow.histogram(dev(keys), begin, end)).astype(np.uint64)
            assert np.array_equal(got, oracle.histograms(keys, begin, end, 8)), (run, begin)
        check_sort(ow, keys, np.arange(n, dtype=np.uint32), 0, kb)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("dist", ["uniform", "and4"])
def test_histogram_several_trips_per_workgroup(ow, kb, dist):
    """A one-workgroup-per-CU grid over more keys than one sweep of it covers:
    each workgroup walks several whole tiles with the next tile's loads in
    flight, then the ragged tail; also the 16-byte-unaligned scalar path."""
    per_sweep = 256 * 1024 * 4 * 16 // (kb // 8)  # CUs x threads x 4 loads x 16 B / key bytes
    n = 2 * per_sweep + 3 * 4099
    keys = keys_of(dist, 43, n, kb)
    cfg = ow.make_config(hist_blocks_per_cu=1)
    t = dev(keys)
    for begin, end in [(0, kb), (6, kb - 2)]:
        got = host(ow.histogram(t, begin, end, config=cfg)).astype(np.uint64)
        assert np.array_equal(got, oracle.histograms(keys, begin, end, 8)), (begin, end)
    got = host(ow.histogram(t[1:], config=cfg)).astype(np.uint64)
    assert np.array_equal(got, oracle.histograms(keys[1:], 0, kb, 8))


def test_histogram_empty_and_unaligned(ow):
    h = ow.histogram(torch.empty(0, dtype=torch.uint32, device="cuda"))
    assert host(h).sum() == 0
    keys = W.uniform(3, 10001)
    t = dev(keys)
    sub = t[1:]  # 4-byte aligned but not 16-byte aligned: scalar load path
    assert np.array_equal(host(ow.histogram(sub)).astype(np.uint64),
                          oracle.histograms(keys[1:], 0, 32, 8))


# ------------------------------------------------------------------ phase 3 (one pass)

SHAPES = {
    (32, False): [(256, 8), (256, 16), (512, 16), (512, 12), (1024, 8), (1024, 10), (1024, 11),
                  (1024, 19)],
    (32, True): [(256, 8), (256, 16), (512, 16), (512, 12), (1024, 8), (1024, 10), (1024, 11),
                 (1024, 18)],
    (64, False): [(256, 8), (256, 16), (512, 8), (512, 12), (1024, 8), (1024, 9), (1024, 14)],
    (64, True): [(256, 8), (256, 16), (512, 8), (512, 12), (1024, 8), (1024, 9)],
}
RANKS = (1, 2, 3)  # one ballot per digit bit; LDS presence masks; ballots + LDS atomics


@pytest.mark.parametrize("kb,vals", [(32, False), (32, True), (64, False), (64, True)])
@pytest.mark.parametrize("rank", RANKS)
def test_binning_pass_parity_and_final_status(ow, kb, vals, rank):
    for block, ipt in SHAPES[(kb, vals)]:
        cfg = ow.make_config(block_threads=block, items_per_thread=ipt, rank_algorithm=rank)
        T = ow.tile_items(kb, vals, cfg)
        assert T == block * ipt
        for n in (1, T - 1, T, T + 1, 5 * T + 77):
            keys = W.uniform(100 + n % 97, n, kb)
            v = np.arange(n, dtype=np.uint32) if vals else None
            for shift, width in ((0, 8), (kb - 8, 8), (5, 3)):
                hist = oracle.histograms(keys, shift, shift + width, width)[0]
                off = oracle.exclusive_sums(hist[None, :])[0]
                off256 = np.zeros(256, dtype=np.uint32)
                off256[:off.size] = off
                off256[off.size:] = n
                dk, dv, temp = ow.binning_pass(dev(keys), dev(off256), shift, width,
                                               src_values=None if v is None else dev(v),
                                               config=cfg)
                wk, wv = oracle.binning_pass(keys, shift, width, off, v)
                assert np.array_equal(host(dk), wk), (block, ipt, n, shift, width)
                if vals:
                    assert np.array_equal(host(dv), wv), (block, ipt, n, shift, width)
                # The chained scan's final state (Figure 7f): every counter is G
                # and holds the inclusive prefix of its digit over tiles.
                g = -(-n // T)
                st = host(temp[256:256 + g * 256 * 4].view(torch.uint32)).reshape(g, 256)
                want = oracle.pass_status(keys, shift, width, T)
                assert np.array_equal(st[:, :1 << width], want)
                assert np.all(st[:, 1 << width:] == np.uint32(2 << 30))


def test_lookback_wait_is_bounded(ow):
    """The look-back wait is bounded: with a limit of one poll, a tile that does
    not meet an inclusive prefix in its first window of predecessors gives up
    and records the look-back error (word 1 of the binning pass's temporary
    storage) instead of waiting; the pass still ends and every store stays in
    bounds. With the default limit the same pass records no error and matches
    the oracle."""
    n = (1 << 24) + 4097
    keys = W.uniform(77, n)
    hist = oracle.histograms(keys, 0, 8, 8)[0]
    off = oracle.exclusive_sums(hist[None, :])[0].astype(np.uint32)
    want, _ = oracle.binning_pass(keys, 0, 8, off.astype(np.uint64))
    d_keys, d_off = dev(keys), dev(off)
    print("[lookback] default limit", flush=True)
    dk, _, temp = ow.binning_pass(d_keys, d_off, 0, 8)
    torch.cuda.synchronize()
    assert int(host(temp[4:8].view(torch.uint32))[0]) == 0
    assert np.array_equal(host(dk), want)
    print("[lookback] limit of one poll", flush=True)
    dk, _, temp = ow.binning_pass(d_keys, d_off, 0, 8,
                                  config=ow.make_config(lookback_spin_limit=1))
    torch.cuda.synchronize()
    assert int(host(temp[4:8].view(torch.uint32))[0]) & 1 == 1
    bad = ow.make_config(lookback_spin_limit=-1)
    with pytest.raises(ow.OnesweepError):
        ow.binning_pass(d_keys, d_off, 0, 8, config=bad)


def test_destination_runs_outside_the_output_write_nothing(ow):
    """Every tile checks once that the run of each of its digits lies inside
    the output. Bin starts moved 1000 places up (forced from the host) push
    the last runs of the top digit past the end: those tiles write nothing and
    set bit 1 of the error word; every other tile writes its keys (and values)
    1000 places above their places, and the first 1000 positions stay as
    they were."""
    n = (1 << 20) + 4097
    keys = W.uniform(78, n)
    vals = np.arange(n, dtype=np.uint32)
    hist = oracle.histograms(keys, 0, 8, 8)[0]
    off = oracle.exclusive_sums(hist[None, :])[0]
    want_k, want_v = oracle.binning_pass(keys, 0, 8, off.astype(np.uint64), vals)
    moved = dev((off + 1000).astype(np.uint32))
    d_keys, d_vals = dev(keys), dev(vals)
    for with_vals in (False, True):
        print(f"[outside] values={with_vals}", flush=True)
        dk = torch.full((n,), -1, dtype=torch.int32, device="cuda").view(torch.uint32)
        dv = torch.full((n,), -1, dtype=torch.int32, device="cuda").view(torch.uint32)
        _, _, temp = ow.binning_pass(d_keys, moved, 0, 8, dst=dk,
                                     src_values=d_vals if with_vals else None,
                                     dst_values=dv if with_vals else None)
        torch.cuda.synchronize()
        assert int(host(temp[4:8].view(torch.uint32))[0]) & 2 == 2
        got_k = host(dk)
        assert np.all(got_k[:1000] == np.uint32(0xFFFFFFFF))
        written = got_k[1000:] != np.uint32(0xFFFFFFFF)
        assert 0 < np.count_nonzero(~written) < n // 2
        assert np.array_equal(got_k[1000:][written], want_k[:n - 1000][written])
        if with_vals:
            got_v = host(dv)
            assert np.all(got_v[:1000] == np.uint32(0xFFFFFFFF))
            assert np.array_equal(got_v[1000:][written], want_v[:n - 1000][written])


# ------------------------------------------------------------------ whole sorts

def check_sort(ow, keys, vals, begin, end, cfg=None, inplace=False):
    kb = 32 if keys.dtype == np.uint32 else 64
    tk = dev(keys)
    if vals is None:
        out = tk if inplace else None
        res = ow.sort_keys(tk, begin, end, out=out, config=cfg)
        got_k, got_v = host(res), None
    else:
        tv = dev(vals)
        rk, rv = ow.sort_pairs(tk, tv, begin, end, keys_out=tk if inplace else None,
                               values_out=tv if inplace else None, config=cfg)
        got_k, got_v = host(rk), host(rv)
    wk, wv = oracle.sort(keys, vals, begin, end, 8)
    assert np.array_equal(got_k, wk)
    if vals is not None:
        assert np.array_equal(got_v, wv)


# Tile shapes built with ballot ranking only: large-input shapes of one
# value presence also built for the other (32-bit keys 1024 x 16 and
# 1024 x 18, 32-bit pairs 1024 x 16 and 1024 x 19, 64-bit keys 1024 x 12,
# 64-bit pairs 1024 x 12 and 1024 x 14), so that every learned-selector
# class serves keys and pairs.
BALLOT_ONLY_SHAPES = {(32, False): [(1024, 16), (1024, 18)], (32, True): [(1024, 16), (1024, 19)],
                      (64, False): [(1024, 12)], (64, True): [(1024, 12), (1024, 14)]}


@pytest.mark.parametrize("kb,vals", [(32, False), (32, True), (64, False), (64, True)])
def test_ballot_only_shapes(ow, kb, vals):
    for block, ipt in BALLOT_ONLY_SHAPES[(kb, vals)]:
        cfg = ow.make_config(block_threads=block, items_per_thread=ipt, rank_algorithm=1)
        T = ow.tile_items(kb, vals, cfg)
        assert T == block * ipt
        for n in (2, T - 1, T + 1, 7 * T + 333):
            keys = W.uniform(17 + n % 13, n, kb)
            v = np.arange(n, dtype=np.uint32) if vals else None
            check_sort(ow, keys, v, 0, kb, cfg)
        n = 5 * T + 77
        keys = W.uniform(23, n, kb)
        v = np.arange(n, dtype=np.uint32) if vals else None
        for shift, width in ((0, 8), (kb - 8, 8), (5, 3)):
            off = oracle.exclusive_sums(oracle.histograms(keys, shift, shift + width, width))[0]
            off256 = np.full(256, n, dtype=np.uint32)
            off256[:off.size] = off
            dk, dv, _ = ow.binning_pass(dev(keys), dev(off256), shift, width,
                                        src_values=None if v is None else dev(v), config=cfg)
            wk, wv = oracle.binning_pass(keys, shift, width, off, v)
            assert np.array_equal(host(dk), wk), (block, ipt, shift, width)
            if vals:
                assert np.array_equal(host(dv), wv), (block, ipt, shift, width)
        # the other ranking methods are not built for these shapes: refused
        for rank in (2, 3):
            bad = ow.make_config(block, ipt, rank_algorithm=rank)
            with pytest.raises(ow.OnesweepError):
                if vals:
                    ow.sort_pairs(dev(keys), dev(v), config=bad)
                else:
                    ow.sort_keys(dev(keys), config=bad)


@pytest.mark.parametrize("kb,vals", [(32, False), (32, True), (64, False), (64, True)])
@pytest.mark.parametrize("rank", RANKS)
def test_sort_every_shape_ragged_sizes(ow, kb, vals, rank):
    for block, ipt in SHAPES[(kb, vals)]:
        cfg = ow.make_config(block_threads=block, items_per_thread=ipt, rank_algorithm=rank)
        T = ow.tile_items(kb, vals, cfg)
        for n in (2, T - 1, T + 1, 7 * T + 333):
            keys = W.uniform(7 + n % 13, n, kb)
            v = np.arange(n, dtype=np.uint32) if vals else None
            check_sort(ow, keys, v, 0, kb, cfg)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("dist", ["and2", "and3", "and4", "equal", "zipf", "presorted",
                                  "reverse", "distinct16"])
def test_sort_distributions(ow, kb, dist):
    n = 300001
    keys = keys_of(dist, 17, n, kb)
    for rank in RANKS:
        cfg = ow.make_config(rank_algorithm=rank)
        check_sort(ow, keys, None, 0, kb, cfg)
        check_sort(ow, keys, np.arange(n, dtype=np.uint32), 0, kb, cfg)


@pytest.mark.parametrize("kb,vals", [(32, False), (32, True), (64, False), (64, True)])
@pytest.mark.parametrize("rank", RANKS)
def test_one_digit_tiles(ow, kb, vals, rank):
    """Tiles whose keys share the place's digit take the short-circuit write
    (Section 3, chained-scan digit-binning kernel): runs of a tile's length
    and of other lengths, so tiles are one-digit, mixed, or straddle two
    runs; the ragged last tile's real keys all carry the padding digit (it
    must not short-circuit)."""
    for block, ipt in SHAPES[(kb, vals)]:
        cfg = ow.make_config(block_threads=block, items_per_thread=ipt, rank_algorithm=rank)
        T = ow.tile_items(kb, vals, cfg)
        for run in (T, 3 * T // 2, 4096):
            n = 6 * T + 77
            keys = W.runs(11 + run % 7, n, kb, run=run, low_bits=8, last_high_ones=True)
            v = np.arange(n, dtype=np.uint32) if vals else None
            check_sort(ow, keys, v, 0, kb, cfg)
            # one pass at a high place: the final chained-scan state as well
            shift, width = kb - 8, 8
            hist = oracle.histograms(keys, shift, shift + width, width)[0]
            off = oracle.exclusive_sums(hist[None, :])[0].astype(np.uint32)
            dk, dv, temp = ow.binning_pass(dev(keys), dev(off), shift, width,
                                           src_values=None if v is None else dev(v), config=cfg)
            wk, wv = oracle.binning_pass(keys, shift, width, off, v)
            assert np.array_equal(host(dk), wk), (block, ipt, run)
            if vals:
                assert np.array_equal(host(dv), wv), (block, ipt, run)
            g = -(-n // T)
            st = host(temp[256:256 + g * 256 * 4].view(torch.uint32)).reshape(g, 256)
            assert np.array_equal(st, oracle.pass_status(keys, shift, width, T))


@pytest.mark.parametrize("kb", [32, 64])
def test_sort_partial_bit_ranges(ow, kb):
    n = 123457
    keys = W.uniform(5, n, kb)
    vals = np.arange(n, dtype=np.uint32)
    for begin, end in [(0, 1), (3, 11), (8, 16), (kb - 13, kb), (7, 7), (0, kb - 1), (1, kb)]:
        check_sort(ow, keys, None, begin, end)
        check_sort(ow, keys, vals, begin, end)


@pytest.mark.parametrize("kb", [32, 64])
def test_sort_in_place(ow, kb):
    n = 200003
    keys = W.and_of_q(9, 2, n, kb)
    check_sort(ow, keys, None, 0, kb, inplace=True)
    check_sort(ow, keys, np.arange(n, dtype=np.uint32), 0, kb, inplace=True)
    # skipped places change the parity of executed passes: 3 of 4 run here
    k2 = (keys & np.array(0x00FFFFFF if kb == 32 else 0x00FFFFFFFFFFFFFF, dtype=keys.dtype))
    check_sort(ow, k2, None, 0, kb, inplace=True)
    check_sort(ow, k2, np.arange(n, dtype=np.uint32), 0, kb, inplace=True)
    check_sort(ow, k2, None, 0, kb)


def test_small_and_degenerate_sizes(ow):
    for n in (0, 1, 2, 3, 63, 64, 65, 255, 256, 257, 4093):
        for kb in (32, 64):
            keys = W.uniform(n + 1, n, kb)
            check_sort(ow, keys, None, 0, kb)
            check_sort(ow, keys, np.arange(n, dtype=np.uint32), 0, kb)
    two = np.array([5, 3] * 5000, dtype=np.uint32)
    check_sort(ow, two, np.arange(two.size, dtype=np.uint32), 0, 32)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_one_million_uniform_u32_keys(ow, seed):
    """2^20 uniform uint32 keys, 8-bit digits, 4 passes, bit-exact."""
    keys = W.uniform(seed, 1 << 20)
    check_sort(ow, keys, None, 0, 32)


def test_trace_records_the_launch_sequence(ow):
    n = 1 << 16
    keys = dev(W.uniform(1, n))
    events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * 16)]
    for e in events:
        e.record()
    torch.cuda.synchronize()
    import ctypes
    arr = (ctypes.c_void_p * len(events))(*[e.cuda_event for e in events])
    tr = ow.Trace()
    tr.events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    tr.capacity = 16
    cfg = ow.make_config(trace=tr)
    ow.sort_keys(keys, config=cfg)
    torch.cuda.synchronize()
    kinds = [tr.kinds[i] for i in range(tr.count)]
    assert kinds == [ow.KERNEL_RESET, ow.KERNEL_HISTOGRAM, ow.KERNEL_SCAN] + \
        [ow.KERNEL_BINNING] * 4 + [ow.KERNEL_COPY]
    for i in range(tr.count):
        assert events[2 * i].elapsed_time(events[2 * i + 1]) >= 0.0


def test_graph_capture_replays(ow):
    """Capture one sort into a HIP graph; replay with fresh inputs, with eager
    work and synchronisation between replays; every replay must be exact."""
    n = (1 << 18) + 7
    static_in = torch.empty(n, dtype=torch.uint32, device="cuda")
    static_out = torch.empty_like(static_in)
    temp = torch.empty(ow.sort_temp_bytes(n), dtype=torch.uint8, device="cuda")
    static_in.copy_(dev(W.uniform(1, n)))
    ow.sort_keys(static_in, out=static_out, temp=temp)  # warm-up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ow.sort_keys(static_in, out=static_out, temp=temp, stream=s)
    torch.cuda.synchronize()
    for seed in (11, 12, 13, 14):
        keys = W.and_of_q(seed, 1 + seed % 3, n)
        static_in.copy_(dev(keys))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(static_out), oracle.sort(keys)[0]), seed
        # eager work between replays
        eager = ow.sort_keys(dev(keys[: n // 2]))
        torch.cuda.synchronize()
        assert np.array_equal(host(eager), oracle.sort(keys[: n // 2])[0])


# ------------------------------------------------------------------ reduce-then-scan baseline

RTS_SHAPES = {
    32: [(256, 8), (512, 16), (1024, 8), (1024, 11), (1024, 16), (1024, 18), (1024, 19)],
    64: [(256, 8), (512, 8), (1024, 8), (1024, 9), (1024, 12), (1024, 14)],
}


@pytest.mark.parametrize("kb,vals", [(32, False), (32, True), (64, False), (64, True)])
def test_reduce_then_scan_sorts(ow, kb, vals):
    """The Section 2 baseline gives the same unique stable result: every shape
    built for it, ragged sizes, skewed and one-digit-place inputs (skipped
    places, odd pass counts), partial bit ranges and in-place sorts."""
    for block, ipt in RTS_SHAPES[kb]:
        cfg = ow.make_config(block, ipt, algorithm=ow.ALGORITHM_REDUCE_THEN_SCAN)
        T = ow.tile_items(kb, vals, cfg)
        assert T == block * ipt
        for n in (1, T - 1, T + 1, 7 * T + 333):
            keys = W.uniform(41 + n % 11, n, kb)
            v = np.arange(n, dtype=np.uint32) if vals else None
            check_sort(ow, keys, v, 0, kb, cfg)
        n = 3 * T + 5
        v = np.arange(n, dtype=np.uint32) if vals else None
        for dist in ("and4", "equal", "distinct16", "presorted"):
            check_sort(ow, keys_of(dist, 43, n, kb), v, 0, kb, cfg)
        check_sort(ow, W.runs(44, n, kb, run=T), v, 0, kb, cfg)
        keys = W.uniform(45, n, kb)
        for begin, end in ((0, 1), (3, 11), (8, 16), (kb - 13, kb), (7, 7)):
            check_sort(ow, keys, v, begin, end, cfg)
        check_sort(ow, keys, v, 0, kb, cfg, inplace=True)


def test_reduce_then_scan_count_table(ow):
    """After the sort, the shared count table holds the last place's tile scan:
    row v, column t is the number of keys with digit v in tiles before t of
    that pass's input, i.e. the oracle's chained-scan inclusive prefix of tile
    t - 1 (Figure 4's prefix order within one digit)."""
    cfg = ow.make_config(1024, 8, algorithm=ow.ALGORITHM_REDUCE_THEN_SCAN)
    T = ow.tile_items(32, False, cfg)
    n = 5 * T + 77
    keys = W.uniform(47, n)
    temp = torch.empty(ow.sort_temp_bytes(n, config=cfg), dtype=torch.uint8, device="cuda")
    out = ow.sort_keys(dev(keys), temp=temp, config=cfg)
    assert np.array_equal(host(out), oracle.sort(keys)[0])
    pass_in = oracle.sort(keys, None, 0, 24, 8)[0]
    incl = (oracle.pass_status(pass_in, 24, 8, T) & np.uint32(0x3FFFFFFF)).astype(np.uint32)
    g = incl.shape[0]
    excl = np.vstack([np.zeros((1, 256), dtype=np.uint32), incl[:-1]])
    # temp layout: 8 x 256 histogram words, one 256-byte counter slot, then the table
    table = host(temp[8448:8448 + 256 * g * 4].view(torch.uint32)).reshape(256, g)
    assert np.array_equal(table, excl.T)


def test_reduce_then_scan_trace_and_graph_replay(ow):
    """Launch sequence per place: upsweep, tile scan, downsweep; a captured
    graph replays exactly with new keys."""
    import ctypes
    n = (1 << 18) + 7
    events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * 32)]
    for e in events:
        e.record()
    torch.cuda.synchronize()
    arr = (ctypes.c_void_p * len(events))(*[e.cuda_event for e in events])
    tr = ow.Trace()
    tr.events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    tr.capacity = 32
    cfg = ow.make_config(algorithm=ow.ALGORITHM_REDUCE_THEN_SCAN, trace=tr)
    keys = W.uniform(49, n)
    out = ow.sort_keys(dev(keys), config=cfg)
    torch.cuda.synchronize()
    assert np.array_equal(host(out), oracle.sort(keys)[0])
    kinds = [tr.kinds[i] for i in range(tr.count)]
    assert kinds == [ow.KERNEL_RESET, ow.KERNEL_HISTOGRAM, ow.KERNEL_SCAN] + \
        [ow.KERNEL_UPSWEEP, ow.KERNEL_TILE_SCAN, ow.KERNEL_DOWNSWEEP] * 4 + [ow.KERNEL_COPY]

    cfg = ow.make_config(algorithm=ow.ALGORITHM_REDUCE_THEN_SCAN)
    static_in = torch.empty(n, dtype=torch.uint32, device="cuda")
    static_vals = torch.empty(n, dtype=torch.uint32, device="cuda")
    static_out = torch.empty_like(static_in)
    static_vout = torch.empty_like(static_in)
    temp = torch.empty(ow.sort_temp_bytes(n, 32, True, config=cfg), dtype=torch.uint8,
                       device="cuda")
    static_in.copy_(dev(keys))
    static_vals.copy_(dev(np.arange(n, dtype=np.uint32)))
    ow.sort_pairs(static_in, static_vals, keys_out=static_out, values_out=static_vout, temp=temp,
                  config=cfg)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            ow.sort_pairs(static_in, static_vals, keys_out=static_out, values_out=static_vout,
                          temp=temp, config=cfg, stream=s)
    torch.cuda.synchronize()
    vals = np.arange(n, dtype=np.uint32)
    for seed in (51, 52, 53):
        k = W.and_of_q(seed, 1 + seed % 3, n)
        static_in.copy_(dev(k))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        wk, wv = oracle.sort(k, vals)
        assert np.array_equal(host(static_out), wk), seed
        assert np.array_equal(host(static_vout), wv), seed
        eager = ow.sort_keys(dev(k[: n // 3]), config=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(host(eager), oracle.sort(k[: n // 3])[0])


# ------------------------------------------------------------------ strips (large inputs)

@pytest.mark.parametrize("kb,vals", [(32, False), (32, True), (64, False), (64, True)])
def test_sorts_in_strips(ow, kb, vals):
    """Binning passes split into strips, each its own chained scan seeded by
    the previous strip's bin starts (Section 3, very large problems): forced
    here with small strips, including one-tile strips and a ragged last strip,
    every shape, typed and descending keys, and partial bit ranges."""
    for block, ipt in SHAPES[(kb, vals)]:
        T = block * ipt
        for strip_log2 in (11, 15):
            cfg = ow.make_config(block, ipt, strip_log2=strip_log2)
            n = 9 * T + 1234
            keys = W.uniform(61 + strip_log2, n, kb)
            v = np.arange(n, dtype=np.uint32) if vals else None
            check_sort(ow, keys, v, 0, kb, cfg)
    cfg = ow.make_config(strip_log2=14)
    n = 100003
    v = np.arange(n, dtype=np.uint32) if vals else None
    keys = W.and_of_q(63, 2, n, kb)
    check_sort(ow, keys, v, 3, kb - 2, cfg)
    check_sort(ow, keys, v, 0, kb, cfg, inplace=True)
    signed = W.signed_ints(64, n, kb)
    got = ow.sort_keys(dev(signed.view(np.int32 if kb == 32 else np.int64)), config=cfg,
                       descending=True)
    want = oracle.sort(signed, None, key_type=oracle.KEY_SIGNED, descending=True)[0]
    assert np.array_equal(host(got).view(signed.dtype), want)


def test_strip_trace_launch_sequence(ow):
    import ctypes
    n = 200001
    events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * 64)]
    for e in events:
        e.record()
    torch.cuda.synchronize()
    arr = (ctypes.c_void_p * len(events))(*[e.cuda_event for e in events])
    tr = ow.Trace()
    tr.events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    tr.capacity = 64
    cfg = ow.make_config(1024, 8, strip_log2=16, trace=tr)  # 8 tiles per strip, 4 strips
    keys = W.uniform(65, n)
    out = ow.sort_keys(dev(keys), config=cfg)
    torch.cuda.synchronize()
    assert np.array_equal(host(out), oracle.sort(keys)[0])
    kinds = [tr.kinds[i] for i in range(tr.count)]
    strips = -(-(-(-n // 8192)) // 8)
    assert strips == 4
    assert kinds == [ow.KERNEL_RESET, ow.KERNEL_HISTOGRAM, ow.KERNEL_SCAN] + \
        [ow.KERNEL_BINNING] * (4 * strips) + [ow.KERNEL_COPY]
