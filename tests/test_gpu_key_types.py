"""GPU parity of signed, floating-point and descending sorts against the oracle.

Keys reach the library either as torch int32/int64/float32/float64 tensors
(the binding takes the key type from the dtype) or as raw uint bits with the
key type set in the config; expected values come only from the oracle's
typed sort of the raw bits. Bit-exact everywhere, NaN payloads included.
"""
import numpy as np
import pytest
import torch

import oracle
import workload as W

pytestmark = pytest.mark.gpu

KINDS = {"unsigned": oracle.KEY_UNSIGNED, "signed": oracle.KEY_SIGNED, "float": oracle.KEY_FLOAT}
DTYPES = {("unsigned", 32): np.uint32, ("unsigned", 64): np.uint64,
          ("signed", 32): np.int32, ("signed", 64): np.int64,
          ("float", 32): np.float32, ("float", 64): np.float64}
SHAPES = {
    (32, False): [(256, 8), (256, 16), (512, 16), (512, 12), (1024, 8), (1024, 10), (1024, 11),
                  (1024, 19)],
    (32, True): [(256, 8), (256, 16), (512, 16), (512, 12), (1024, 8), (1024, 10), (1024, 11),
                 (1024, 18)],
    (64, False): [(256, 8), (256, 16), (512, 8), (512, 12), (1024, 8), (1024, 9), (1024, 14)],
    (64, True): [(256, 8), (256, 16), (512, 8), (512, 12), (1024, 8), (1024, 9)],
}


@pytest.fixture(scope="module")
def ow():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2206_01784_amd as mod
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def bits_of(kind, seed, n, kb):
    if kind == "signed":
        return W.signed_ints(seed, n, kb)
    if kind == "float":
        return W.float_bits(seed, n, kb)
    return W.uniform(seed, n, kb)


def check(ow, bits, kind, vals=None, begin=0, end=None, descending=False, config=None,
          raw=False, inplace=False):
    """Sort on the GPU (typed tensor, or raw bits with key_type in the config)
    and compare bit for bit with the oracle."""
    kb = bits.dtype.itemsize * 8
    end = kb if end is None else end
    if raw:
        t = dev(bits)
        cfg = ow.make_config() if config is None else ow.Config.from_buffer_copy(config)
        cfg.key_type = KINDS[kind]
        cfg.descending = int(descending)
        desc_arg = False
    else:
        t = dev(bits.view(DTYPES[(kind, kb)]))
        cfg, desc_arg = config, descending
    if vals is None:
        out = ow.sort_keys(t, begin, end, out=t if inplace else None, config=cfg,
                           descending=desc_arg)
        got_v = None
    else:
        tv = dev(vals)
        out, ov = ow.sort_pairs(t, tv, begin, end, keys_out=t if inplace else None,
                                values_out=tv if inplace else None, config=cfg,
                                descending=desc_arg)
        got_v = ov.cpu().numpy()
    got_k = out.cpu().numpy().view(bits.dtype)
    wk, wv = oracle.sort(bits, vals, begin, end, 8, key_type=KINDS[kind], descending=descending)
    assert np.array_equal(got_k, wk), (kind, kb, begin, end, descending)
    if vals is not None:
        assert np.array_equal(got_v, wv), (kind, kb, begin, end, descending)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind", ["signed", "float", "unsigned"])
@pytest.mark.parametrize("descending", [False, True])
def test_typed_sorts_ragged_sizes(ow, kb, kind, descending):
    for vals in (False, True):
        T = ow.tile_items(kb, vals, None, 1 << 20)
        for n in (1, 2, 63, T - 1, T + 1, 5 * T + 77):
            bits = bits_of(kind, 3 + n % 17, n, kb)
            v = np.arange(n, dtype=np.uint32) if vals else None
            check(ow, bits, kind, v, descending=descending)


@pytest.mark.parametrize("kb,vals", [(32, False), (32, True), (64, False), (64, True)])
def test_typed_sorts_every_shape_and_ranking(ow, kb, vals):
    """Every compiled tile shape and ranking method with float and signed
    keys, both directions: the padding key of a ragged tile must carry the
    largest ordered digit in each case."""
    for block, ipt in SHAPES[(kb, vals)]:
        for rank in (1, 2, 3):
            cfg = ow.make_config(block, ipt, rank_algorithm=rank)
            T = ow.tile_items(kb, vals, cfg)
            n = 3 * T + 5
            v = np.arange(n, dtype=np.uint32) if vals else None
            for kind, descending in (("float", False), ("float", True), ("signed", True)):
                check(ow, bits_of(kind, 7 + rank, n, kb), kind, v, descending=descending,
                      config=cfg)


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("kind", ["signed", "float"])
def test_typed_partial_bit_ranges_raw_bits_and_in_place(ow, kb, kind):
    n = 70001
    bits = bits_of(kind, 11, n, kb)
    v = np.arange(n, dtype=np.uint32)
    for begin, end in ((0, 1), (3, 11), (kb - 13, kb), (kb - 1, kb), (7, 7), (0, kb - 1)):
        for descending in (False, True):
            check(ow, bits, kind, None, begin, end, descending)
            check(ow, bits, kind, v, begin, end, descending)
    for descending in (False, True):
        check(ow, bits, kind, v, descending=descending, raw=True)
        check(ow, bits, kind, None, descending=descending, inplace=True)
        check(ow, bits, kind, v, descending=descending, inplace=True)


@pytest.mark.parametrize("kb", [32, 64])
def test_typed_reduce_then_scan(ow, kb):
    cfg = ow.make_config(algorithm=ow.ALGORITHM_REDUCE_THEN_SCAN)
    n = 3 * ow.tile_items(kb, True, cfg, 1 << 20) + 9
    v = np.arange(n, dtype=np.uint32)
    for kind in ("signed", "float"):
        for descending in (False, True):
            check(ow, bits_of(kind, 13, n, kb), kind, v, descending=descending, config=cfg)


@pytest.mark.parametrize("kb", [32, 64])
def test_typed_histogram(ow, kb):
    n = 100003
    for kind in ("signed", "float"):
        bits = bits_of(kind, 17, n, kb)
        for descending in (False, True):
            for begin, end in ((0, kb), (5, kb - 3)):
                got = ow.histogram(dev(bits.view(DTYPES[(kind, kb)])), begin, end,
                                   descending=descending).cpu().numpy().astype(np.uint64)
                want = oracle.histograms(oracle.ordered_bits(bits, KINDS[kind], descending),
                                         begin, end, 8)
                assert np.array_equal(got, want), (kind, descending, begin, end)


EDGE_LENGTHS = [0, 1, 2, 63, 64, 65, 0, 511, 512, 513, 1000, 2047, 2048, 2049, 0, 4096, 8191,
                8192, 8193, 8192 * 3 + 5, 16384, 1, 40000, 0]


@pytest.mark.parametrize("kb", [32, 64])
@pytest.mark.parametrize("limits", [(0, 0, 0), (-1, -1, -1)])
def test_typed_segmented_sorts(ow, kb, limits):
    """Segments in every LDS class and the tiled path, both directions."""
    lengths = np.array(EDGE_LENGTHS * 2, dtype=np.int64)
    off = W.offsets_from_lengths(lengths)
    n = int(off[-1])
    v = np.arange(n, dtype=np.uint32)
    d_off = dev(off.astype(np.uint32))
    cfg = ow.make_config(segment_limits=limits)
    for kind in ("signed", "float", "unsigned"):
        bits = bits_of(kind, 19, n, kb)
        for descending in (False, True):
            if kind == "unsigned" and not descending:
                continue
            t = dev(bits.view(DTYPES[(kind, kb)]))
            ko, vo = ow.sort_segments(t, d_off, dev(v), config=cfg, descending=descending)
            wk, wv = oracle.sort_segments(bits, off, v, key_type=KINDS[kind],
                                          descending=descending)
            assert np.array_equal(ko.cpu().numpy().view(bits.dtype), wk), (kind, descending)
            assert np.array_equal(vo.cpu().numpy(), wv), (kind, descending)


def test_typed_large_float_pairs(ow):
    """2^22 float32 pairs descending: many tiles of every digit mix."""
    n = (1 << 22) + 3
    bits = W.float_bits(23, n, 32)
    check(ow, bits, "float", np.arange(n, dtype=np.uint32), descending=True)
    check(ow, bits, "float", None, descending=False)


def test_typed_segmented_tuner_keeps_the_key_order(ow):
    lengths = np.array(EDGE_LENGTHS, dtype=np.int64)
    off = W.offsets_from_lengths(lengths)
    n = int(off[-1])
    bits = bits_of("float", 29, n, 32)
    v = np.arange(n, dtype=np.uint32)
    t = dev(bits.view(np.float32))
    cfg = ow.tune_segments(t, dev(off.astype(np.uint32)), dev(v), keys_out=None,
                           repetitions=1, descending=True)
    assert cfg.key_type == ow.KEY_FLOAT and cfg.descending == 1
    ko, vo = ow.sort_segments(dev(bits), dev(off.astype(np.uint32)), dev(v), config=cfg)
    wk, wv = oracle.sort_segments(bits, off, v, key_type=oracle.KEY_FLOAT, descending=True)
    assert np.array_equal(ko.cpu().numpy(), wk) and np.array_equal(vo.cpu().numpy(), wv)


def test_learned_selection_keeps_the_key_type(ow):
    """The committed model's pick for float keys keeps the float order."""
    import os
    model = ow.Model(max_batch=1, path=os.path.join(os.path.dirname(ow.__file__),
                                                    "config_model.bin"))
    n = (1 << 20) + 17
    bits = bits_of("float", 31, n, 32)
    t = dev(bits.view(np.float32))
    cfg = ow.select_config(model, t)
    assert cfg.key_type == ow.KEY_FLOAT
    check(ow, bits, "float", None, config=cfg)
    check(ow, bits, "float", np.arange(n, dtype=np.uint32), descending=True, config=cfg)
