"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates arguments before touching any GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "onesweep.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(onesweep_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("onesweep_sort_keys", "onesweep_sort_pairs", "onesweep_histogram",
              "onesweep_binning_pass", "onesweep_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_2206_01784_amd as ow
    lib = ow.library()
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_library_is_built_for_gfx950_only():
    """The offload bundle ids in the library name gfx950 and no other target."""
    import paper_2206_01784_amd as ow
    blob = open(ow.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}, targets


def test_temp_size_query_needs_no_gpu():
    import paper_2206_01784_amd as ow
    t = ow.tile_items(32)
    n = 1 << 28
    need = ow.sort_temp_bytes(n, 32)
    # at least the ping-pong buffer plus p * tiles * 256 status words
    assert need >= 4 * n + 4 * (-(-n // t)) * 256 * 4
    assert ow.sort_temp_bytes(1 << 20, 64, True) >= (1 << 20) * 12
    assert ow.sort_temp_bytes(0, 32) > 0


@pytest.mark.parametrize("kwargs,code", [
    (dict(key_bits=48), 1),
    (dict(begin_bit=9, end_bit=8), 1),
    (dict(end_bit=33), 1),
    (dict(n=1 << 36), 2),
])
def test_invalid_arguments_are_rejected_on_the_host(kwargs, code):
    import paper_2206_01784_amd as ow
    lib = ow.library()
    args = dict(n=100, key_bits=32, begin_bit=0, end_bit=32)
    args.update(kwargs)
    size = ctypes.c_size_t(0)
    rc = lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, args["n"], args["key_bits"],
                                args["begin_bit"], args["end_bit"], 1, None, None)
    assert rc == code
    assert lib.onesweep_last_error()


def test_unsupported_config_is_rejected():
    import paper_2206_01784_amd as ow
    lib = ow.library()
    size = ctypes.c_size_t(0)
    cfg = ow.make_config(block_threads=384, items_per_thread=7)
    rc = lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, 100, 32, 0, 32, 1,
                                ctypes.byref(cfg), None)
    assert rc == ow.ERROR_UNSUPPORTED
    assert ow.tile_items(32, False, cfg) == 0
    # digit widths 4..8 are built; a sort covers at most 8 places
    for d, kb, end, code in ((3, 32, 32, ow.ERROR_UNSUPPORTED), (9, 32, 32, ow.ERROR_UNSUPPORTED),
                             (7, 64, 64, ow.ERROR_UNSUPPORTED), (7, 64, 56, 0),
                             (4, 32, 32, 0), (8, 64, 64, 0)):
        cfg = ow.make_config(digit_bits=d)
        rc = lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, 100, kb, 0, end, 1,
                                    ctypes.byref(cfg), None)
        assert rc == code, (d, kb, end)
    # narrower digits: more places, so more status words per sort
    n = 1 << 24
    assert ow.sort_temp_bytes(n, 32, config=ow.make_config(digit_bits=6)) > \
        ow.sort_temp_bytes(n, 32)


def test_reduce_then_scan_config_validation_needs_no_gpu():
    """The baseline algorithm: accepted by whole plain sorts for the shapes
    built for it; rejected elsewhere and for unknown values; its temporary
    storage holds one count table instead of one status table per place."""
    import paper_2206_01784_amd as ow
    lib = ow.library()
    rts = ow.make_config(algorithm=ow.ALGORITHM_REDUCE_THEN_SCAN)
    n = 1 << 28
    t = ow.tile_items(32, False, rts, n)
    assert t == ow.tile_items(32, False, None, n)
    tiles = -(-n // t)
    one = ow.sort_temp_bytes(n, 32, config=rts)
    assert one >= 4 * n + tiles * 256 * 4
    assert ow.sort_temp_bytes(n, 32) - one >= 3 * tiles * 256 * 4
    for kb in (32, 64):
        for vals in (False, True):
            for log2n in (12, 20, 28):
                assert ow.sort_temp_bytes(1 << log2n, kb, vals, config=rts) > 0
    size = ctypes.c_size_t(0)
    for alg in (-1, 2):
        cfg = ow.make_config(algorithm=alg)
        rc = lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, 100, 32, 0, 32, 1,
                                    ctypes.byref(cfg), None)
        assert rc == ow.ERROR_INVALID_VALUE, alg
    # shapes not built for the baseline
    for shape in ((512, 12), (256, 16)):
        cfg = ow.make_config(*shape, algorithm=1)
        rc = lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, 100, 32, 0, 32, 1,
                                    ctypes.byref(cfg), None)
        assert rc == ow.ERROR_UNSUPPORTED, shape
    cfg = ow.make_config(rank_algorithm=ow.RANK_PRESENCE, algorithm=1)
    rc = lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, 100, 32, 0, 32, 1,
                                ctypes.byref(cfg), None)
    assert rc == ow.ERROR_UNSUPPORTED
    # the segmented sort and the single-pass entry point take Onesweep only
    rc = lib.onesweep_sort_segments(None, ctypes.byref(size), None, None, None, None, 10, None, 1,
                                    32, 0, 32, 1, ctypes.byref(rts), None)
    assert rc == ow.ERROR_INVALID_VALUE
    rc = lib.onesweep_binning_pass(None, ctypes.byref(size), None, None, None, None, 10, 32, 0, 8,
                                   None, ctypes.byref(rts), None)
    assert rc == ow.ERROR_INVALID_VALUE


def test_key_type_and_direction_validation_needs_no_gpu():
    import paper_2206_01784_amd as ow
    lib = ow.library()
    size = ctypes.c_size_t(0)
    for kwargs in (dict(key_type=3), dict(key_type=-1), dict(descending=2)):
        cfg = ow.make_config(**kwargs)
        if "descending" in kwargs:
            cfg.descending = kwargs["descending"]
        rc = lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, 100, 32, 0, 32, 1,
                                    ctypes.byref(cfg), None)
        assert rc == ow.ERROR_INVALID_VALUE, kwargs
    for kt in (ow.KEY_UNSIGNED, ow.KEY_SIGNED, ow.KEY_FLOAT):
        for desc in (False, True):
            cfg = ow.make_config(key_type=kt, descending=desc)
            assert ow.sort_temp_bytes(1000, 64, True, config=cfg) == \
                ow.sort_temp_bytes(1000, 64, True)


def test_strip_configuration_and_size_limits_need_no_gpu():
    """Whole plain sorts accept n below 2^36 (strips of at most 2^29 keys per
    chained scan; from 2^31 keys, or more than 4 GiB of keys, on, 64-bit
    counts, bin starts and positions, built for the default large-input tile
    shapes only, and no reduce-then-scan); the single-pass, histogram and
    segmented entry points keep one chained scan and the 2^30 limit, and the
    single pass also at most 4 GiB of keys."""
    import paper_2206_01784_amd as ow
    lib = ow.library()
    size = ctypes.c_size_t(0)
    n = (1 << 31) - 1
    big = ow.sort_temp_bytes(n, 32)
    assert big >= 4 * n
    assert ow.sort_temp_bytes(n, 32, True) >= 8 * n
    # strip bin starts: one 256-word row per (place, strip) after the first
    one = ow.sort_temp_bytes(1 << 20, 32)
    strips = ow.sort_temp_bytes(1 << 20, 32, config=ow.make_config(strip_log2=14))
    assert strips - one >= (64 - 1) * 256 * 4
    for bad in (10, 30, -1):
        cfg = ow.make_config(strip_log2=bad)
        rc = lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, 100, 32, 0, 32, 1,
                                    ctypes.byref(cfg), None)
        assert rc == ow.ERROR_INVALID_VALUE, bad
    assert lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, 1 << 36, 32, 0, 32, 1,
                                  None, None) == ow.ERROR_TOO_LARGE
    # beyond 4 GiB of keys: 64-bit counts and bin offsets (8 bytes per entry)
    wide = ow.sort_temp_bytes((1 << 30) + 1, 32)
    narrow = ow.sort_temp_bytes(1 << 30, 32)
    assert wide - narrow >= 8 * 256 * 4
    assert ow.sort_temp_bytes(1 << 31, 64, True) >= 12 * (1 << 31)
    for kb, vals in ((32, False), (32, True), (64, False), (64, True)):
        assert ow.tile_items(kb, vals, None, 1 << 31) > 0
    for kb, last in ((32, 1 << 30), (64, 1 << 29)):
        for cfg in (ow.make_config(1024, 8),
                    ow.make_config(algorithm=ow.ALGORITHM_REDUCE_THEN_SCAN)):
            rc = lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, last + 1, kb, 0,
                                        kb, 1, ctypes.byref(cfg), None)
            assert rc == ow.ERROR_UNSUPPORTED, (kb, last)
            assert lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, last, kb, 0,
                                          kb, 1, ctypes.byref(cfg), None) == 0, (kb, last)
    assert lib.onesweep_binning_pass(None, ctypes.byref(size), None, None, None, None,
                                     (1 << 29) + 1, 64, 0, 8, None, None,
                                     None) == ow.ERROR_TOO_LARGE
    assert lib.onesweep_binning_pass(None, ctypes.byref(size), None, None, None, None, 1 << 29,
                                     64, 0, 8, None, None, None) == 0
    assert lib.onesweep_sort_segments(None, ctypes.byref(size), None, None, None, None, 1 << 30,
                                      None, 1, 32, 0, 32, 1, None,
                                      None) == ow.ERROR_TOO_LARGE
    assert lib.onesweep_binning_pass(None, ctypes.byref(size), None, None, None, None, 1 << 30,
                                     32, 0, 8, None, None, None) == ow.ERROR_TOO_LARGE


def test_insufficient_temp_and_null_pointers():
    import paper_2206_01784_amd as ow
    lib = ow.library()
    size = ctypes.c_size_t(10)
    rc = lib.onesweep_sort_keys(ctypes.c_void_p(256), ctypes.byref(size), ctypes.c_void_p(4096),
                                ctypes.c_void_p(8192), 100, 32, 0, 32, 1, None, None)
    assert rc == ow.ERROR_INSUFFICIENT_TEMP
    need = ow.sort_temp_bytes(100)
    size = ctypes.c_size_t(need)
    rc = lib.onesweep_sort_keys(ctypes.c_void_p(256), ctypes.byref(size), None,
                                ctypes.c_void_p(8192), 100, 32, 0, 32, 1, None, None)
    assert rc == ow.ERROR_INVALID_VALUE
    # partial overlap of input and output
    rc = lib.onesweep_sort_keys(ctypes.c_void_p(1 << 20), ctypes.byref(size),
                                ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 64), 100, 32, 0, 32,
                                1, None, None)
    assert rc == ow.ERROR_INVALID_VALUE
    # misaligned temp
    rc = lib.onesweep_sort_keys(ctypes.c_void_p((1 << 20) + 4), ctypes.byref(size),
                                ctypes.c_void_p(4096), ctypes.c_void_p(65536), 100, 32, 0, 32, 1,
                                None, None)
    assert rc == ow.ERROR_INVALID_VALUE


def test_empty_input_accepts_null_pointers():
    import paper_2206_01784_amd as ow
    lib = ow.library()
    size = ctypes.c_size_t(0)
    assert lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, 0, 32, 0, 32, 1, None,
                                  None) == 0
    assert lib.onesweep_sort_keys(ctypes.c_void_p(256), ctypes.byref(size), None, None, 0, 32, 0,
                                  32, 1, None, None) == 0


def test_segmented_temp_query_and_validation():
    import paper_2206_01784_amd as ow
    lib = ow.library()
    n, S = 1 << 26, 20000
    need = ow.sort_segments_temp_bytes(n, S, 32, True)
    assert need >= 8 * n  # ping-pong keys and values for the large segments
    # all segments fit in LDS: no temporary key buffer, no status rows
    small_only = ow.sort_segments_temp_bytes(8192, 4, 32, True)
    assert small_only < 8192
    # every segment routed to the tile path needs more than the default
    all_large = ow.make_config(segment_limits=(-1, -1, -1))
    assert ow.sort_segments_temp_bytes(n, S, 32, True, config=all_large) > need
    size = ctypes.c_size_t(0)
    # keys without a segment
    assert lib.onesweep_sort_segments(None, ctypes.byref(size), None, None, None, None, 10, None,
                                      0, 32, 0, 32, 1, None, None) == ow.ERROR_INVALID_VALUE
    # too many segments
    assert lib.onesweep_sort_segments(None, ctypes.byref(size), None, None, None, None, 10, None,
                                      1 << 30, 32, 0, 32, 1, None, None) == ow.ERROR_TOO_LARGE
    # class limits beyond a class's capacity, or below -1
    for limits in ((513, 0, 0), (0, 2049, 0), (0, 0, 8193), (-2, 0, 0)):
        cfg = ow.make_config(segment_limits=limits)
        assert lib.onesweep_sort_segments(None, ctypes.byref(size), None, None, None, None, 10,
                                          None, 1, 32, 0, 32, 1, ctypes.byref(cfg),
                                          None) == ow.ERROR_INVALID_VALUE, limits
    # a binning shape not built for the segmented path
    cfg = ow.make_config(block_threads=512, items_per_thread=12)
    assert lib.onesweep_sort_segments(None, ctypes.byref(size), None, None, None, None, 10, None,
                                      1, 32, 0, 32, 1, ctypes.byref(cfg),
                                      None) == ow.ERROR_UNSUPPORTED
    # NULL offsets with keys to sort
    need = ow.sort_segments_temp_bytes(100, 1)
    size = ctypes.c_size_t(need)
    assert lib.onesweep_sort_segments(ctypes.c_void_p(1 << 20), ctypes.byref(size),
                                      ctypes.c_void_p(4096), ctypes.c_void_p(8192), None, None,
                                      100, None, 1, 32, 0, 32, 1, None,
                                      None) == ow.ERROR_INVALID_VALUE


def test_learned_constants_match_the_oracle_and_need_no_gpu():
    import paper_2206_01784_amd as ow
    from oracle import mlp
    header = open(HEADER).read()
    for name, value in (("ONESWEEP_FEATURES", mlp.FEATURES),
                        ("ONESWEEP_MODEL_CLASSES", mlp.C),
                        ("ONESWEEP_MODEL_PARAMS", mlp.NUM_PARAMS)):
        assert re.search(rf"#define {name} {value}\b", header), name
    assert ow.library().onesweep_model_num_params() == mlp.NUM_PARAMS
    assert (ow.FEATURES, ow.MODEL_CLASSES, ow.MODEL_PARAMS) == \
        (mlp.FEATURES, mlp.C, mlp.NUM_PARAMS)
    # a missing or foreign model file is rejected before any GPU work
    h = ctypes.c_void_p()
    assert ow.library().onesweep_model_load(b"/nonexistent/model.bin", 4,
                                            ctypes.byref(h)) == ow.ERROR_INVALID_VALUE
    import tempfile
    with tempfile.NamedTemporaryFile(suffix=".bin") as f:
        f.write(b"NOTAMODEL" * 100)
        f.flush()
        assert ow.library().onesweep_model_load(f.name.encode(), 4,
                                                ctypes.byref(h)) == ow.ERROR_INVALID_VALUE
    # no model: the default configuration, no GPU touched
    cfg = ow.Config()
    assert ow.library().onesweep_select_config(None, None, 1000, 32, 0, 32, 0,
                                               ctypes.byref(cfg), None) == 0
    assert (cfg.block_threads, cfg.items_per_thread) == (0, 0)


def test_segmented_tuner_size_query_needs_no_gpu():
    import paper_2206_01784_amd as ow
    lib = ow.library()
    size = ctypes.c_size_t(0)
    dummy = ctypes.c_void_p(4)
    assert lib.onesweep_tune_segments(None, ctypes.byref(size), None, None, dummy, dummy,
                                      1 << 20, None, 100, 32, 0, 32, 3, None, None) == 0
    # the largest need over the candidates covers the default configuration
    assert size.value >= ow.sort_segments_temp_bytes(1 << 20, 100, 32, True)
    assert lib.onesweep_tune_segments(None, ctypes.byref(size), None, None, None, None,
                                      1 << 20, None, 100, 32, 0, 32, 0, None,
                                      None) == ow.ERROR_INVALID_VALUE
