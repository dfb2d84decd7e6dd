"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (default config): 2^28 uint32 keys (uniform, the entropy bands
AND-of-2/3/4/8/16, all equal), 2^27 uint64 keys, 2^28 uint32 pairs and 2^27
uint64-key pairs (values = original index), the batched segmented workload,
more than 2^30 keys and more than 2^31 keys (64-bit counts and positions).

Every element is compared, against the oracle run at full size, or, for the
permutation inputs beyond 2^31 keys, against their closed-form sorted order.
"""
import numpy as np
import pytest
import torch

import oracle
import workload as W

pytestmark = pytest.mark.gpu

N28 = 1 << 28


@pytest.fixture(scope="module")
def ow():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2206_01784_amd as mod
    return mod


def test_full_u32_keys_uniform(ow):
    keys = W.uniform(2, N28)
    t = torch.from_numpy(keys).cuda()
    out = ow.sort_keys(t)
    want, _ = oracle.sort(keys)
    assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("dist", ["and2", "and3", "and4", "and8", "and16", "equal"])
def test_full_u32_keys_entropy_bands(ow, dist):
    """2^28 keys of every entropy band of Section 4 (AND of q uniform words,
    Table 1) and the all-equal case, element by element against the oracle."""
    print(f"[full] 2^28 u32 keys, {dist}", flush=True)
    keys = W.make_keys(dist, 2, N28)
    out = ow.sort_keys(torch.from_numpy(keys).cuda())
    got = out.cpu().numpy()
    del out
    want, _ = oracle.sort(keys)
    assert np.array_equal(got, want)


def test_full_u64_keys_only(ow):
    """2^27 uniform uint64 keys, keys only (8 binning passes)."""
    n = 1 << 27
    keys = W.uniform(3, n, 64)
    out = ow.sort_keys(torch.from_numpy(keys).cuda())
    got = out.cpu().numpy()
    del out
    want, _ = oracle.sort(keys)
    assert np.array_equal(got, want)


def test_full_u32_pairs(ow):
    keys = W.uniform(3, N28)
    vals = np.arange(N28, dtype=np.uint32)
    ko, vo = ow.sort_pairs(torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda())
    wk, wv = oracle.sort(keys, vals)
    assert np.array_equal(ko.cpu().numpy(), wk)
    assert np.array_equal(vo.cpu().numpy(), wv)


def test_full_u64_pairs(ow):
    n = 1 << 27
    keys = W.uniform(3, n, 64)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = ow.sort_pairs(torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda())
    wk, wv = oracle.sort(keys, vals)
    assert np.array_equal(ko.cpu().numpy(), wk)
    assert np.array_equal(vo.cpu().numpy(), wv)


def test_full_segments_lognormal_20000(ow):
    """The batched workload at full size: 20,000 log-normal segments, 2^26
    uint32 pairs (values = index within the segment), default class limits
    and tiles, captured in a graph and replayed, checked against the
    per-segment oracle element by element."""
    lengths = W.lognormal_segment_lengths(num_segments=20000, total=1 << 26, seed=4)
    off = W.offsets_from_lengths(lengths)
    n = int(off[-1])
    keys = W.uniform(4, n)
    seg_of = np.repeat(np.arange(20000), lengths)
    vals = (np.arange(n, dtype=np.int64) - off[seg_of]).astype(np.uint32)
    tk, tv = torch.from_numpy(keys).cuda(), torch.from_numpy(vals).cuda()
    to = torch.from_numpy(off.astype(np.uint32)).cuda()
    ko, vo = torch.empty_like(tk), torch.empty_like(tv)
    temp = torch.empty(ow.sort_segments_temp_bytes(n, 20000, 32, True), dtype=torch.uint8,
                       device="cuda")
    ow.sort_segments(tk, to, tv, keys_out=ko, values_out=vo, temp=temp)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ow.sort_segments(tk, to, tv, keys_out=ko, values_out=vo, temp=temp, stream=s)
    ko.zero_()
    vo.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    wk, wv = oracle.sort_segments(keys, off, vals)
    assert np.array_equal(ko.cpu().numpy(), wk)
    assert np.array_equal(vo.cpu().numpy(), wv)


def test_full_keys_beyond_2p30(ow):
    """2^30 + 4097 uint32 keys: with the default 1024 x 19 tiles and strips of
    at most 2^29 keys, each binning pass runs three strips (27,594 + 27,594
    tiles and a last one-tile strip), each its own chained scan, the bin
    starts carried from strip to strip; more than 4 GiB of keys, so 64-bit
    counts and positions; bit-exact against the oracle."""
    n = (1 << 30) + 4097
    print(f"[full] 2^30 + 4097 u32 keys, n={n}", flush=True)
    keys = W.uniform(91, n)
    d = torch.from_numpy(keys).cuda()
    out = ow.sort_keys(d)
    del d
    got = out.cpu().numpy()
    del out
    torch.cuda.empty_cache()
    want = oracle.sort(keys)[0]
    assert np.array_equal(got, want)


N31 = (1 << 31) + 4097
# key_i = (A * i + B) mod n is a permutation of 0 .. n - 1 (A is prime and
# does not divide n), so the sorted keys are 0, 1, ..., n - 1 and the value
# (input index) at sorted position k is A^-1 (k - B) mod n.
PERM_A, PERM_B = 2654435761, 12345


def _perm_keys(n):
    import math
    assert math.gcd(PERM_A, n) == 1
    i = torch.arange(n, dtype=torch.int64, device="cuda")
    k = (i * (PERM_A % n) + PERM_B) % n
    del i
    return k.to(torch.int32).view(torch.uint32)


def _check_sorted_permutation(ko, vo, n, chunk=1 << 28):
    ainv = pow(PERM_A, -1, n)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        k = torch.arange(lo, hi, dtype=torch.int64, device="cuda")
        got = ko[lo:hi].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        assert torch.equal(got, k), f"keys differ in [{lo}, {hi})"
        if vo is not None:
            want = ((k - PERM_B) % n) * ainv % n
            gotv = vo[lo:hi].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
            assert torch.equal(gotv, want), f"values differ in [{lo}, {hi})"


def test_full_keys_beyond_2p31_permutation(ow):
    """2^31 + 4097 uint32 keys (a permutation of 0 .. n - 1): 64-bit
    histogram counts in portions of 2^30 keys, 64-bit bin starts carried
    across five strips per pass, 64-bit positions; the output must be
    0, 1, ..., n - 1."""
    n = N31
    print(f"[full] 2^31 + 4097 u32 keys (permutation), n={n}", flush=True)
    keys = _perm_keys(n)
    out = ow.sort_keys(keys)
    del keys
    torch.cuda.synchronize()
    _check_sorted_permutation(out, None, n)
    del out
    torch.cuda.empty_cache()


def test_full_pairs_beyond_2p31_permutation(ow):
    """2^31 + 4097 (uint32 key, uint32 value = input index) pairs, keys a
    permutation: every value must be the input index of the key at its
    position, A^-1 (k - B) mod n."""
    n = N31
    print(f"[full] 2^31 + 4097 u32 pairs (permutation), n={n}", flush=True)
    keys = _perm_keys(n)
    vals = torch.arange(n, dtype=torch.int64, device="cuda").to(torch.int32).view(torch.uint32)
    ko, vo = ow.sort_pairs(keys, vals)
    del keys, vals
    torch.cuda.synchronize()
    _check_sorted_permutation(ko, vo, n)
    del ko, vo
    torch.cuda.empty_cache()


def test_full_keys_beyond_2p31_uniform(ow):
    """2^31 + 4097 uniform uint32 keys against the oracle, element by
    element."""
    n = N31
    print(f"[full] 2^31 + 4097 u32 keys (uniform), n={n}", flush=True)
    keys = W.uniform(92, n)
    d = torch.from_numpy(keys).cuda()
    out = ow.sort_keys(d)
    del d
    got = out.cpu().numpy()
    del out
    torch.cuda.empty_cache()
    want = oracle.sort(keys)[0]
    del keys
    assert np.array_equal(got, want)
