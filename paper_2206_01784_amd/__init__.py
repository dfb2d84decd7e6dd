"""Python binding of the Onesweep HIP library for MI355X (gfx950).

Argument marshalling only: every step of the sort runs in the HIP kernels of
libonesweep.so, reached through its C ABI (include/onesweep.h). PyTorch
supplies device memory and the current stream. There is no CPU fallback: if
the library is not built, importing this package raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libonesweep.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python paper_2206_01784_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)

SUCCESS = 0
ERROR_INVALID_VALUE = 1
ERROR_TOO_LARGE = 2
ERROR_INSUFFICIENT_TEMP = 3
ERROR_HIP = 4
ERROR_UNSUPPORTED = 5

(KERNEL_RESET, KERNEL_HISTOGRAM, KERNEL_SCAN, KERNEL_BINNING, KERNEL_COPY, KERNEL_CLASSIFY,
 KERNEL_LDS_SORT, KERNEL_UPSWEEP, KERNEL_TILE_SCAN, KERNEL_DOWNSWEEP) = range(10)
KERNEL_NAMES = ("reset", "histogram", "scan", "binning", "copy", "classify", "lds_sort",
                "upsweep", "tile_scan", "downsweep")
SEGMENT_CLASS_CAPACITY = (512, 2048, 8192)
TRACE_MAX = 64
RADIX_BITS = 8
RADIX = 256


class Trace(ctypes.Structure):
    _fields_ = [("events", ctypes.POINTER(ctypes.c_void_p)), ("capacity", ctypes.c_int),
                ("count", ctypes.c_int), ("kinds", ctypes.c_int * TRACE_MAX)]


class Config(ctypes.Structure):
    _fields_ = [("digit_bits", ctypes.c_int), ("block_threads", ctypes.c_int),
                ("items_per_thread", ctypes.c_int), ("hist_blocks_per_cu", ctypes.c_int),
                ("rank_algorithm", ctypes.c_int), ("segment_limits", ctypes.c_int * 3),
                ("segment_streams", ctypes.c_int), ("algorithm", ctypes.c_int),
                ("key_type", ctypes.c_int), ("descending", ctypes.c_int),
                ("strip_log2", ctypes.c_int), ("lookback_spin_limit", ctypes.c_int),
                ("trace", ctypes.POINTER(Trace))]


_vp, _sz, _i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
_szp = ctypes.POINTER(ctypes.c_size_t)
_cfgp = ctypes.POINTER(Config)

_lib.onesweep_sort_keys.argtypes = [_vp, _szp, _vp, _vp, _sz, _i32, _i32, _i32, _i32, _cfgp, _vp]
_lib.onesweep_sort_keys_noalloc.argtypes = [_vp, _vp, _sz, _i32, _i32, _i32, _i32, _cfgp, _vp]
_lib.onesweep_sort_pairs.argtypes = [_vp, _szp, _vp, _vp, _vp, _vp, _sz, _i32, _i32, _i32, _i32,
                                     _cfgp, _vp]
_lib.onesweep_histogram.argtypes = [_vp, _sz, _i32, _i32, _i32, _vp, _cfgp, _vp]
_lib.onesweep_binning_pass.argtypes = [_vp, _szp, _vp, _vp, _vp, _vp, _sz, _i32, _i32, _i32, _vp,
                                       _cfgp, _vp]
_lib.onesweep_sort_segments.argtypes = [_vp, _szp, _vp, _vp, _vp, _vp, _sz, _vp, _sz, _i32, _i32,
                                        _i32, _i32, _cfgp, _vp]
_lib.onesweep_tune_segments.argtypes = [_vp, _szp, _vp, _vp, _vp, _vp, _sz, _vp, _sz, _i32, _i32,
                                        _i32, _i32, _cfgp, _vp]
_lib.onesweep_tune_segments.restype = _i32
_lib.onesweep_tile_items.argtypes = [_i32, _i32, _sz, _cfgp]
_lib.onesweep_tile_items.restype = _sz
_lib.onesweep_last_error.restype = ctypes.c_char_p
_lib.onesweep_version.restype = ctypes.c_char_p
NOALLOC_SCRATCH_BYTES = 64 << 20
for _f in ("onesweep_sort_keys", "onesweep_sort_keys_noalloc", "onesweep_sort_pairs", "onesweep_histogram",
           "onesweep_binning_pass", "onesweep_sort_segments"):
    getattr(_lib, _f).restype = _i32


class OnesweepError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"onesweep error {code}: {message}")
        self.code = code


def library():
    """The loaded ctypes handle of libonesweep.so."""
    return _lib


def version() -> str:
    return _lib.onesweep_version().decode()


def _check(code: int):
    if code != SUCCESS:
        raise OnesweepError(code, _lib.onesweep_last_error().decode())


RANK_DEFAULT, RANK_BALLOT, RANK_PRESENCE, RANK_ATOMIC = 0, 1, 2, 3
ALGORITHM_ONESWEEP, ALGORITHM_REDUCE_THEN_SCAN = 0, 1
KEY_UNSIGNED, KEY_SIGNED, KEY_FLOAT = 0, 1, 2


def make_config(block_threads: int = 0, items_per_thread: int = 0, hist_blocks_per_cu: int = 0,
                digit_bits: int = 0, rank_algorithm: int = 0, segment_limits=(0, 0, 0),
                segment_streams: int = 0, algorithm: int = 0, key_type: int = 0,
                descending: bool = False, strip_log2: int = 0, lookback_spin_limit: int = 0,
                trace: Trace | None = None) -> Config:
    c = Config(digit_bits, block_threads, items_per_thread, hist_blocks_per_cu, rank_algorithm,
               (ctypes.c_int * 3)(*segment_limits), segment_streams, algorithm, key_type,
               int(descending), strip_log2, lookback_spin_limit, None)
    if trace is not None:
        c.trace = ctypes.pointer(trace)
    return c


def _cfg_ptr(cfg):
    return None if cfg is None else ctypes.byref(cfg)


_KEY_DTYPES = {
    torch.uint32: (32, KEY_UNSIGNED), torch.uint64: (64, KEY_UNSIGNED),
    torch.int32: (32, KEY_SIGNED), torch.int64: (64, KEY_SIGNED),
    torch.float32: (32, KEY_FLOAT), torch.float64: (64, KEY_FLOAT),
}


def _key_bits(t: torch.Tensor) -> int:
    if t.dtype not in _KEY_DTYPES:
        raise TypeError(f"keys must be torch.uint32/uint64/int32/int64/float32/float64, "
                        f"got {t.dtype}")
    return _KEY_DTYPES[t.dtype][0]


def _ordered_config(config: Config | None, keys: torch.Tensor, descending: bool):
    """The config with the key type of a signed or floating-point dtype and
    the requested direction (a copy; the caller's config is left as it is).
    Unsigned tensors keep the config's key_type, so raw bits of signed or
    floating-point keys can be sorted through it."""
    key_type = _KEY_DTYPES[keys.dtype][1] if keys.dtype in _KEY_DTYPES else KEY_UNSIGNED
    if key_type == KEY_UNSIGNED and not descending:
        return config
    c = Config() if config is None else Config.from_buffer_copy(config)
    if key_type != KEY_UNSIGNED:
        c.key_type = key_type
    c.descending = int(bool(descending) or bool(c.descending))
    return c


def _dev_ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else None


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def tile_items(key_bits: int = 32, has_values: bool = False, config: Config | None = None,
               n: int = 1 << 28) -> int:
    """Binning tile size the config resolves to (the default depends on n)."""
    return int(_lib.onesweep_tile_items(key_bits, int(has_values), n, _cfg_ptr(config)))


def sort_temp_bytes(n: int, key_bits: int = 32, has_values: bool = False, begin_bit: int = 0,
                    end_bit: int | None = None, config: Config | None = None) -> int:
    """Temporary storage a sort of n keys needs (pure host computation)."""
    end_bit = key_bits if end_bit is None else end_bit
    size = ctypes.c_size_t(0)
    if has_values:
        _check(_lib.onesweep_sort_pairs(None, ctypes.byref(size), None, None, None, None, n,
                                        key_bits, begin_bit, end_bit, 1, _cfg_ptr(config), None))
    else:
        _check(_lib.onesweep_sort_keys(None, ctypes.byref(size), None, None, n, key_bits,
                                       begin_bit, end_bit, 1, _cfg_ptr(config), None))
    return int(size.value)


def _temp(temp, need, device):
    if temp is None:
        return torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    if temp.numel() < need:
        raise ValueError(f"temp holds {temp.numel()} bytes, needs {need}")
    return temp


def sort_keys(keys: torch.Tensor, begin_bit: int = 0, end_bit: int | None = None,
              out: torch.Tensor | None = None, temp: torch.Tensor | None = None,
              config: Config | None = None, stream=None, descending: bool = False) -> torch.Tensor:
    """Stable sort of keys by bits [begin_bit, end_bit) of their ordered bits.

    uint32/uint64 keys sort as unsigned integers, int32/int64 as signed,
    float32/float64 as IEEE 754 values (-NaN < -inf < -0 < +0 < +inf < +NaN).
    """
    kb = _key_bits(keys)
    config = _ordered_config(config, keys, descending)
    end_bit = kb if end_bit is None else end_bit
    n = keys.numel()
    if out is None:
        out = torch.empty_like(keys)
    need = sort_temp_bytes(n, kb, False, begin_bit, end_bit, config)
    temp = _temp(temp, need, keys.device)
    size = ctypes.c_size_t(temp.numel())
    _check(_lib.onesweep_sort_keys(_dev_ptr(temp), ctypes.byref(size), _dev_ptr(keys),
                                   _dev_ptr(out), n, kb, begin_bit, end_bit, 1,
                                   _cfg_ptr(config), _stream(stream)))
    return out


def sort_keys_noalloc(keys: torch.Tensor, begin_bit: int = 0, end_bit: int | None = None,
                      out: torch.Tensor | None = None, config: Config | None = None, stream=None,
                      descending: bool = False) -> torch.Tensor:
    """sort_keys through the allocation-free entry point: the library's own
    64 MiB device array per GPU serves as temporary storage, so the C call
    allocates nothing (pass `out` to avoid torch's allocation too). Calls
    that overlap on one GPU race."""
    kb = _key_bits(keys)
    config = _ordered_config(config, keys, descending)
    end_bit = kb if end_bit is None else end_bit
    if out is None:
        out = torch.empty_like(keys)
    _check(_lib.onesweep_sort_keys_noalloc(_dev_ptr(keys), _dev_ptr(out), keys.numel(), kb,
                                           begin_bit, end_bit, 1, _cfg_ptr(config),
                                           _stream(stream)))
    return out


def sort_pairs(keys: torch.Tensor, values: torch.Tensor, begin_bit: int = 0,
               end_bit: int | None = None, keys_out: torch.Tensor | None = None,
               values_out: torch.Tensor | None = None, temp: torch.Tensor | None = None,
               config: Config | None = None, stream=None, descending: bool = False):
    """Stable sort of (key, uint32 value) pairs (key types as in sort_keys);
    returns (keys_out, values_out)."""
    kb = _key_bits(keys)
    config = _ordered_config(config, keys, descending)
    if values.dtype != torch.uint32:
        raise TypeError("values must be torch.uint32")
    if values.numel() != keys.numel():
        raise ValueError("keys and values differ in length")
    end_bit = kb if end_bit is None else end_bit
    n = keys.numel()
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    values_out = torch.empty_like(values) if values_out is None else values_out
    need = sort_temp_bytes(n, kb, True, begin_bit, end_bit, config)
    temp = _temp(temp, need, keys.device)
    size = ctypes.c_size_t(temp.numel())
    _check(_lib.onesweep_sort_pairs(_dev_ptr(temp), ctypes.byref(size), _dev_ptr(keys),
                                    _dev_ptr(keys_out), _dev_ptr(values), _dev_ptr(values_out), n,
                                    kb, begin_bit, end_bit, 1, _cfg_ptr(config), _stream(stream)))
    return keys_out, values_out


def histogram(keys: torch.Tensor, begin_bit: int = 0, end_bit: int | None = None,
              out: torch.Tensor | None = None, config: Config | None = None,
              stream=None, descending: bool = False) -> torch.Tensor:
    """Phase 1 alone: uint32 digit counts of every place of the ordered key
    bits (config.digit_bits wide, 8 by default), shape (p, 256)."""
    kb = _key_bits(keys)
    config = _ordered_config(config, keys, descending)
    end_bit = kb if end_bit is None else end_bit
    d = config.digit_bits if config is not None and config.digit_bits else RADIX_BITS
    p = (end_bit - begin_bit + d - 1) // d
    if out is None:
        out = torch.empty((max(p, 0), RADIX), dtype=torch.uint32, device=keys.device)
    if p == 0:
        return out
    _check(_lib.onesweep_histogram(_dev_ptr(keys), keys.numel(), kb, begin_bit, end_bit,
                                   _dev_ptr(out), _cfg_ptr(config), _stream(stream)))
    return out


def binning_pass_temp_bytes(n: int, key_bits: int = 32, has_values: bool = False,
                            config: Config | None = None) -> int:
    size = ctypes.c_size_t(0)
    dummy = ctypes.c_void_p(1) if has_values else None
    _check(_lib.onesweep_binning_pass(None, ctypes.byref(size), None, None, dummy, dummy, n,
                                      key_bits, 0, RADIX_BITS, None, _cfg_ptr(config), None))
    return int(size.value)


def binning_pass(src: torch.Tensor, bin_offsets: torch.Tensor, shift: int, width: int = 8,
                 dst: torch.Tensor | None = None, src_values: torch.Tensor | None = None,
                 dst_values: torch.Tensor | None = None, temp: torch.Tensor | None = None,
                 config: Config | None = None, stream=None, descending: bool = False):
    """Phase 3, one iteration: stable scatter of src by digit
    (ordered bits >> shift) & (2^width - 1), key types as in sort_keys.

    Returns (dst, dst_values, temp); temp holds the tile counter and the
    chained-scan status words (see onesweep_binning_pass in include/onesweep.h).
    """
    kb = _key_bits(src)
    config = _ordered_config(config, src, descending)
    if bin_offsets.dtype != torch.uint32 or bin_offsets.numel() != RADIX:
        raise ValueError("bin_offsets must be 256 uint32")
    n = src.numel()
    has_values = src_values is not None
    dst = torch.empty_like(src) if dst is None else dst
    if has_values and dst_values is None:
        dst_values = torch.empty_like(src_values)
    need = binning_pass_temp_bytes(n, kb, has_values, config)
    temp = _temp(temp, need, src.device)
    size = ctypes.c_size_t(temp.numel())
    _check(_lib.onesweep_binning_pass(_dev_ptr(temp), ctypes.byref(size), _dev_ptr(src),
                                      _dev_ptr(dst), _dev_ptr(src_values), _dev_ptr(dst_values),
                                      n, kb, shift, width, _dev_ptr(bin_offsets),
                                      _cfg_ptr(config), _stream(stream)))
    return dst, dst_values, temp


def sort_segments_temp_bytes(n: int, num_segments: int, key_bits: int = 32,
                             has_values: bool = False, begin_bit: int = 0,
                             end_bit: int | None = None, config: Config | None = None) -> int:
    """Temporary storage of a segmented sort (pure host computation)."""
    end_bit = key_bits if end_bit is None else end_bit
    size = ctypes.c_size_t(0)
    dummy = ctypes.c_void_p(4) if has_values else None
    _check(_lib.onesweep_sort_segments(None, ctypes.byref(size), None, None, dummy, dummy, n, None,
                                       num_segments, key_bits, begin_bit, end_bit, 1,
                                       _cfg_ptr(config), None))
    return int(size.value)


def sort_segments(keys: torch.Tensor, offsets: torch.Tensor, values: torch.Tensor | None = None,
                  begin_bit: int = 0, end_bit: int | None = None,
                  keys_out: torch.Tensor | None = None, values_out: torch.Tensor | None = None,
                  temp: torch.Tensor | None = None, config: Config | None = None, stream=None,
                  descending: bool = False):
    """Stable sort of every segment [offsets[s], offsets[s+1]) on its own
    (key types as in sort_keys).

    offsets: uint32 device tensor of num_segments + 1 entries (0 first, n
    last, non-decreasing). Returns keys_out, or (keys_out, values_out) when
    values are given. After the work completes, temp[0:4] holds 1 if the
    device found the offsets invalid (then nothing was written), else 0.
    """
    kb = _key_bits(keys)
    config = _ordered_config(config, keys, descending)
    if offsets.dtype != torch.uint32:
        raise TypeError("offsets must be torch.uint32")
    if offsets.numel() < 1:
        raise ValueError("offsets needs num_segments + 1 >= 1 entries")
    end_bit = kb if end_bit is None else end_bit
    n = keys.numel()
    num_segments = offsets.numel() - 1
    has_values = values is not None
    if has_values:
        if values.dtype != torch.uint32:
            raise TypeError("values must be torch.uint32")
        if values.numel() != n:
            raise ValueError("keys and values differ in length")
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    if has_values and values_out is None:
        values_out = torch.empty_like(values)
    need = sort_segments_temp_bytes(n, num_segments, kb, has_values, begin_bit, end_bit, config)
    temp = _temp(temp, need, keys.device)
    size = ctypes.c_size_t(temp.numel())
    _check(_lib.onesweep_sort_segments(_dev_ptr(temp), ctypes.byref(size), _dev_ptr(keys),
                                       _dev_ptr(keys_out), _dev_ptr(values),
                                       _dev_ptr(values_out), n, _dev_ptr(offsets), num_segments,
                                       kb, begin_bit, end_bit, 1, _cfg_ptr(config),
                                       _stream(stream)))
    return (keys_out, values_out) if has_values else keys_out


def tune_segments(keys: torch.Tensor, offsets: torch.Tensor, values: torch.Tensor | None = None,
                  begin_bit: int = 0, end_bit: int | None = None,
                  keys_out: torch.Tensor | None = None, values_out: torch.Tensor | None = None,
                  repetitions: int = 3, stream=None, descending: bool = False) -> Config:
    """Time the segmented sort's candidate configurations on this data and
    return the fastest (the outputs hold the sorted segments afterwards).
    Key types as in sort_keys; the returned config keeps the key order."""
    kb = _key_bits(keys)
    end_bit = kb if end_bit is None else end_bit
    n = keys.numel()
    num_segments = offsets.numel() - 1
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    if values is not None and values_out is None:
        values_out = torch.empty_like(values)
    size = ctypes.c_size_t(0)
    dummy = ctypes.c_void_p(4) if values is not None else None
    _check(_lib.onesweep_tune_segments(None, ctypes.byref(size), None, None, dummy, dummy, n, None,
                                       num_segments, kb, begin_bit, end_bit, repetitions, None,
                                       None))
    cfg = _ordered_config(None, keys, descending) or Config()
    temp = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=keys.device)
    size = ctypes.c_size_t(temp.numel())
    _check(_lib.onesweep_tune_segments(_dev_ptr(temp), ctypes.byref(size), _dev_ptr(keys),
                                       _dev_ptr(keys_out), _dev_ptr(values), _dev_ptr(values_out),
                                       n, _dev_ptr(offsets), num_segments, kb, begin_bit, end_bit,
                                       repetitions, ctypes.byref(cfg), _stream(stream)))
    return cfg


# ------------------------------------------------------------------ learned configuration
FEATURES = 2051
MODEL_CLASSES = 12
MODEL_PARAMS = 17500
_fp = ctypes.POINTER(ctypes.c_float)
_lib.onesweep_model_create.argtypes = [_i32, ctypes.POINTER(_vp)]
_lib.onesweep_model_load.argtypes = [ctypes.c_char_p, _i32, ctypes.POINTER(_vp)]
_lib.onesweep_model_save.argtypes = [_vp, ctypes.c_char_p]
_lib.onesweep_model_free.argtypes = [_vp]
_lib.onesweep_model_free.restype = None
_lib.onesweep_model_num_params.restype = _sz
_lib.onesweep_model_set_params.argtypes = [_vp, _vp, _sz]
_lib.onesweep_model_get_params.argtypes = [_vp, _vp, _sz]
_lib.onesweep_model_class.argtypes = [_vp, _i32, _cfgp, ctypes.POINTER(_i32)]
_lib.onesweep_features.argtypes = [_vp, _sz, _i32, _i32, _i32, _i32, _vp, _vp]
_lib.onesweep_model_infer.argtypes = [_vp, _vp, ctypes.c_uint, _vp, _vp, _vp]
_lib.onesweep_model_forward.argtypes = [_vp, _vp, _vp, _i32, _vp, _vp]
_lib.onesweep_model_gradients.argtypes = [_vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp]
_lib.onesweep_model_train_step.argtypes = [_vp, _vp, _vp, _vp, _vp, _i32, ctypes.c_float, _vp,
                                           _vp]
_lib.onesweep_select_config.argtypes = [_vp, _vp, _sz, _i32, _i32, _i32, _i32, _cfgp, _vp]
_lib.onesweep_sort_learned.argtypes = [_vp, _vp, _szp, _vp, _vp, _vp, _vp, _sz, _i32, _i32, _i32,
                                       _cfgp, _cfgp, _vp]
for _f in ("onesweep_model_create", "onesweep_model_load", "onesweep_model_save",
           "onesweep_model_set_params", "onesweep_model_get_params", "onesweep_model_class",
           "onesweep_features", "onesweep_model_infer", "onesweep_model_forward",
           "onesweep_model_gradients", "onesweep_model_train_step", "onesweep_select_config",
           "onesweep_sort_learned"):
    getattr(_lib, _f).restype = _i32


def features(keys: torch.Tensor, begin_bit: int = 0, end_bit: int | None = None,
             has_values: bool = False, out: torch.Tensor | None = None, stream=None):
    """Sampled digit-histogram features of the keys (float32, FEATURES values)."""
    kb = _key_bits(keys)
    end_bit = kb if end_bit is None else end_bit
    if out is None:
        out = torch.empty(FEATURES, dtype=torch.float32, device=keys.device)
    _check(_lib.onesweep_features(_dev_ptr(keys), keys.numel(), kb, begin_bit, end_bit,
                                  int(has_values), _dev_ptr(out), _stream(stream)))
    return out


class Model:
    """A configuration-selection MLP on the current GPU (owns device memory)."""

    def __init__(self, max_batch: int = 1024, path: str | None = None):
        self._h = ctypes.c_void_p()
        if path is None:
            _check(_lib.onesweep_model_create(max_batch, ctypes.byref(self._h)))
        else:
            _check(_lib.onesweep_model_load(os.fsencode(path), max_batch, ctypes.byref(self._h)))
        self.max_batch = max_batch

    def __del__(self, _lib=_lib):  # the library bound here: module globals are gone at exit
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.onesweep_model_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def save(self, path: str):
        _check(_lib.onesweep_model_save(self._h, os.fsencode(path)))

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != MODEL_PARAMS:
            raise ValueError(f"expected {MODEL_PARAMS} parameters")
        _check(_lib.onesweep_model_set_params(self._h, a.ctypes.data, a.size))

    def get_params(self):
        import numpy as np
        a = np.empty(MODEL_PARAMS, dtype=np.float32)
        _check(_lib.onesweep_model_get_params(self._h, a.ctypes.data, a.size))
        return a

    def class_config(self, index: int):
        """(Config, key_bits_mask) of one class."""
        cfg = Config()
        mask = ctypes.c_int(0)
        _check(_lib.onesweep_model_class(self._h, index, ctypes.byref(cfg), ctypes.byref(mask)))
        return cfg, mask.value

    def infer(self, feats: torch.Tensor, class_mask: int = (1 << MODEL_CLASSES) - 1,
              stream=None):
        out = torch.empty(MODEL_CLASSES, dtype=torch.float32, device=feats.device)
        choice = torch.empty(1, dtype=torch.int32, device=feats.device)
        _check(_lib.onesweep_model_infer(self._h, _dev_ptr(feats), class_mask, _dev_ptr(out),
                                         _dev_ptr(choice), _stream(stream)))
        return out, choice

    @staticmethod
    def _split(x: torch.Tensor):
        if x.dim() != 2 or x.shape[1] != FEATURES or x.dtype != torch.float32:
            raise ValueError("x must be float32 of shape (batch, FEATURES)")
        return x[:, : FEATURES - 3].contiguous(), x[:, FEATURES - 3:].contiguous()

    def forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        hist, scal = self._split(x)
        out = torch.empty((x.shape[0], MODEL_CLASSES), dtype=torch.float32, device=x.device)
        _check(_lib.onesweep_model_forward(self._h, _dev_ptr(hist), _dev_ptr(scal), x.shape[0],
                                           _dev_ptr(out), _stream(stream)))
        return out

    def gradients(self, x: torch.Tensor, y: torch.Tensor, mask: torch.Tensor, stream=None):
        """(loss, flat gradient) of the masked squared error."""
        hist, scal = self._split(x)
        grad = torch.empty(MODEL_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(_lib.onesweep_model_gradients(self._h, _dev_ptr(hist), _dev_ptr(scal),
                                             _dev_ptr(y.contiguous()),
                                             _dev_ptr(mask.contiguous()), x.shape[0],
                                             _dev_ptr(grad), _dev_ptr(loss), _stream(stream)))
        return loss, grad

    def train_step(self, x: torch.Tensor, y: torch.Tensor, mask: torch.Tensor, lr: float = 1e-3,
                   stream=None, split=None):
        """One Adam step on a batch; returns the loss tensor (before the step)."""
        hist, scal = self._split(x) if split is None else split
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(_lib.onesweep_model_train_step(self._h, _dev_ptr(hist), _dev_ptr(scal),
                                              _dev_ptr(y), _dev_ptr(mask), x.shape[0], lr,
                                              _dev_ptr(loss), _stream(stream)))
        return loss

    def select_config(self, keys: torch.Tensor, begin_bit: int = 0, end_bit: int | None = None,
                      has_values: bool = False, stream=None) -> Config:
        return select_config(self, keys, begin_bit, end_bit, has_values, stream)


def sort_learned(model: Model | None, keys: torch.Tensor, values: torch.Tensor | None = None,
                 begin_bit: int = 0, end_bit: int | None = None, out: torch.Tensor | None = None,
                 values_out: torch.Tensor | None = None, temp: torch.Tensor | None = None,
                 config: Config | None = None, stream=None, descending: bool = False):
    """Sort keys (and values) with the tile configuration the model picks for
    them; the selection overlaps the sort's first phases (2^26..2^28 keys,
    else the default table). Returns (keys_out, values_out or None, the
    configuration the passes ran with)."""
    kb = _key_bits(keys)
    config = _ordered_config(config, keys, descending)
    end_bit = kb if end_bit is None else end_bit
    n = keys.numel()
    out = torch.empty_like(keys) if out is None else out
    if values is not None and values_out is None:
        values_out = torch.empty_like(values)
    h = None if model is None else model.handle
    size = ctypes.c_size_t(0)
    dummy = ctypes.c_void_p(4) if values is not None else None
    _check(_lib.onesweep_sort_learned(h, None, ctypes.byref(size), None, None, dummy, dummy, n,
                                      kb, begin_bit, end_bit, _cfg_ptr(config), None, None))
    temp = _temp(temp, int(size.value), keys.device)
    size = ctypes.c_size_t(temp.numel())
    used = Config()
    _check(_lib.onesweep_sort_learned(h, _dev_ptr(temp), ctypes.byref(size), _dev_ptr(keys),
                                      _dev_ptr(out), _dev_ptr(values), _dev_ptr(values_out), n,
                                      kb, begin_bit, end_bit, _cfg_ptr(config),
                                      ctypes.byref(used), _stream(stream)))
    return out, values_out, used


def select_config(model: Model | None, keys: torch.Tensor, begin_bit: int = 0,
                  end_bit: int | None = None, has_values: bool = False, stream=None) -> Config:
    """Configuration the model picks for these keys (synchronises the stream);
    it keeps the key type of the keys' dtype."""
    kb = _key_bits(keys)
    end_bit = kb if end_bit is None else end_bit
    cfg = _ordered_config(None, keys, False) or Config()
    _check(_lib.onesweep_select_config(None if model is None else model.handle, _dev_ptr(keys),
                                       keys.numel(), kb, begin_bit, end_bit, int(has_values),
                                       ctypes.byref(cfg), _stream(stream)))
    return cfg
