"""The allocation-free keys-only sort (onesweep_sort_keys_noalloc): its
output must equal onesweep_sort_keys' (and the oracle's) element by element,
on consecutive calls that share the library's scratch array, the second with
a smaller input; inputs beyond the array are rejected on the host."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workload as W


@pytest.fixture(scope="module")
def ow():
    import paper_2206_01784_amd as mod
    return mod


def _noalloc(ow, keys, out, begin_bit=0, end_bit=None, cfg=None):
    kb = 8 * keys.element_size()
    end_bit = kb if end_bit is None else end_bit
    rc = ow.library().onesweep_sort_keys_noalloc(
        ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(out.data_ptr()), keys.numel(), kb,
        begin_bit, end_bit, 1, None if cfg is None else ctypes.byref(cfg),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, ow.library().onesweep_last_error()
    return out


def _max_n(ow, key_bits):
    lo, hi = 1, 1 << 26
    while lo < hi:
        m = (lo + hi + 1) // 2
        if ow.sort_temp_bytes(m, key_bits) <= ow.NOALLOC_SCRATCH_BYTES:
            lo = m
        else:
            hi = m - 1
    return lo


def test_inputs_beyond_the_scratch_array_are_rejected(ow):
    """No GPU work: the size check precedes everything else."""
    lib = ow.library()
    for kb in (32, 64):
        m = _max_n(ow, kb)
        assert m > (7_500_000 if kb == 64 else 15_000_000)
        rc = lib.onesweep_sort_keys_noalloc(None, None, m + 1, kb, 0, kb, 1, None, None)
        assert rc == ow.ERROR_TOO_LARGE
        assert b"allocation-free" in lib.onesweep_last_error()
    assert lib.onesweep_sort_keys_noalloc(None, None, 100, 48, 0, 48, 1, None, None) == \
        ow.ERROR_INVALID_VALUE


@pytest.mark.gpu
@pytest.mark.parametrize("key_bits,n1,n2", [(32, 3_000_017, 100_003), (64, 1_500_001, 4_099)])
def test_noalloc_matches_the_allocating_sort_on_consecutive_calls(ow, key_bits, n1, n2):
    """Two calls in a row through the shared scratch array, the second
    smaller (its cleared state must not depend on the first call's)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    for seed, n in ((21, n1), (22, n2)):
        print(f"[noalloc] {key_bits}-bit keys, n={n}, seed={seed}", flush=True)
        keys = W.uniform(seed, n, key_bits)
        d = torch.from_numpy(keys).cuda()
        got = _noalloc(ow, d, torch.empty_like(d))
        ref = ow.sort_keys(d)
        torch.cuda.synchronize()
        got, ref = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(got, ref)
        assert np.array_equal(got, oracle.sort(keys)[0])


@pytest.mark.gpu
def test_noalloc_bit_range_and_largest_input(ow):
    """A partial bit range (odd pass count, stable by the field only) and the
    largest 32-bit input the array holds, each after a larger call."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    m = _max_n(ow, 32)
    print(f"[noalloc] largest 32-bit input n={m}", flush=True)
    keys = W.uniform(23, m)
    d = torch.from_numpy(keys).cuda()
    got = _noalloc(ow, d, torch.empty_like(d)).cpu().numpy()
    assert np.array_equal(got, ow.sort_keys(d).cpu().numpy())
    keys = W.uniform(24, 777_777)
    d = torch.from_numpy(keys).cuda()
    got = _noalloc(ow, d, torch.empty_like(d), begin_bit=5, end_bit=29).cpu().numpy()
    ref = ow.sort_keys(d, begin_bit=5, end_bit=29).cpu().numpy()
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.sort(keys, begin_bit=5, end_bit=29)[0])


@pytest.mark.gpu
def test_noalloc_graph_replays(ow):
    """Captured once (after an eager call on the device) and replayed with new
    keys and eager work between replays; every replay matches the eager sort."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    n = 250_001
    d = torch.from_numpy(W.uniform(25, n)).cuda()
    out = torch.empty_like(d)
    _noalloc(ow, d, out)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            rc = ow.library().onesweep_sort_keys_noalloc(
                ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(out.data_ptr()), n, 32, 0, 32, 1,
                None, ctypes.c_void_p(s.cuda_stream))
    assert rc == 0
    for seed in (26, 27, 28):
        keys = W.uniform(seed, n)
        d.copy_(torch.from_numpy(keys))
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = ow.sort_keys(d)  # eager work on the same device between replays
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy())
        assert np.array_equal(out.cpu().numpy(), np.sort(keys))
