// C ABI of the Onesweep library: argument validation, temporary-storage
// layout, the launch sequence of the three phases (Section 3) and optional
// per-launch event tracing. No allocation, no synchronisation.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "internal.hpp"

namespace onesweep {

thread_local char g_error[512] = "";

onesweep_status_t fail(onesweep_status_t code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_error, sizeof(g_error), fmt, ap);
  va_end(ap);
  return code;
}

onesweep_status_t hip_fail(hipError_t e, const char *what) {
  return fail(ONESWEEP_ERROR_HIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_error[0] = '\0'; }

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMaxN = size_t(1) << 30;  // 30-bit status values, one chained scan
// Whole plain sorts run large inputs as strips of at most 2^29 keys per
// binning pass (each strip its own chained scan), so 30-bit status values
// never overflow. (2^29 rather than the paper's 2^28: tiles of 1024 x 11 keys
// do not divide 2^28, and a 2^28-key sort should stay one strip.) Below 2^31
// elements, counts, bin starts and element positions are 32-bit (a factor-2
// headroom in every 32-bit index computation); from 2^31 on they are 64-bit
// (Section 3, handling very large problems: 64-bit global histogram counts
// and carried bin starts), the upfront histogram runs over portions of at
// most 2^30 keys (32-bit counters in LDS) and adds into 64-bit global counts.
// 2^36 elements (256 GiB of 32-bit keys) is beyond one GPU's memory.
constexpr size_t kWideN = size_t(1) << 31;
constexpr size_t kMaxSortN = size_t(1) << 36;
// The 32-bit-position binning kernels store through buffer resources, whose
// offsets are 32-bit: a sort whose key output passes 4 GiB (32-bit keys from
// 2^30 + 1 on, 64-bit keys from 2^29 + 1) takes the 64-bit-position path too.
constexpr size_t kBufferBytes = size_t(1) << 32;
inline bool wide_positions(size_t n, int key_bits) {
  return n >= kWideN || n * static_cast<size_t>(key_bits / 8) > kBufferBytes;
}
constexpr size_t kHistPortion = size_t(1) << 30;
// A late tile choice (the learned selector) applies to at most 2^28 keys:
// then every tile of at most 65536 keys bins each place in one strip, so
// only the status region depends on the tile.
constexpr size_t kLateChoiceMaxN = size_t(1) << 28;
constexpr int kDefaultStripLog2 = 29;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int num_places(int begin_bit, int end_bit, int digit_bits) {
  return (end_bit - begin_bit + digit_bits - 1) / digit_bits;
}

// Smallest digit width built: narrower digits gain nothing on this GPU (a
// binning pass costs the same at every width from 5 to 8 bits) and only add
// passes.
constexpr int kMinDigitBits = 4;

// Compute units of the current device, cached per device id.
std::atomic<int> g_cus[64];

onesweep_status_t device_cus(int *cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev >= 0 && dev < 64) {
    int c = g_cus[dev].load(std::memory_order_relaxed);
    if (c > 0) {
      *cus = c;
      return ONESWEEP_SUCCESS;
    }
  }
  int c = 0;
  e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  if (c <= 0) c = 1;
  if (dev >= 0 && dev < 64) g_cus[dev].store(c, std::memory_order_relaxed);
  *cus = c;
  return ONESWEEP_SUCCESS;
}

// Resolved kernel configuration.
struct Resolved {
  BinningShape shape;
  int digit_bits;  // width of a digit place, 4..8 (places of a sort: at most 8)
  int hist_blocks_per_cu;
  int strip_log2;
  int algorithm;  // onesweep_algorithm_t
  KeyOrder order;
  uint32_t spin_limit;  // look-back polls without an inclusive prefix before giving up
  onesweep_trace_t *trace;
};

// Default bound of the look-back wait: 2^22 polls of a tile's window of
// predecessors, each a memory round trip of a microsecond or more, so
// seconds; a legitimate look-back takes a few polls.
constexpr uint32_t kDefaultSpinLimit = 1u << 22;

// Constants of the order transform for a key width, key type and direction;
// `pad` is the key whose transformed bits are all ones (the largest digit at
// every place), which fills the lanes past the end of a tile.
KeyOrder key_order(int key_bits, int key_type, bool descending) {
  const uint64_t all = key_bits == 64 ? ~uint64_t(0) : uint64_t(0xFFFFFFFFu);
  const uint64_t top = uint64_t(1) << (key_bits - 1);
  KeyOrder o{};
  o.sign = key_type != ONESWEEP_KEY_UNSIGNED ? top : 0u;
  o.negative = key_type == ONESWEEP_KEY_FLOAT ? all : 0u;
  o.invert = descending ? all : 0u;
  if (!descending)
    o.pad = key_type == ONESWEEP_KEY_UNSIGNED ? all : (all ^ top);
  else
    o.pad = key_type == ONESWEEP_KEY_UNSIGNED ? 0u : (key_type == ONESWEEP_KEY_SIGNED ? top : all);
  return o;
}

// Which entry point resolves: whole plain sorts offer both algorithms, the
// segmented sort has its own binning shapes, the rest take Onesweep's.
enum Caller { kCallSort, kCallSegments, kCallOther };

onesweep_status_t resolve(int key_bits, bool has_values, size_t n, const onesweep_config_t *cfg,
                          Resolved *r, Caller caller = kCallOther) {
  r->shape = caller == kCallSegments ? segment_default_shape(key_bits, has_values)
                                     : binning_default_shape(key_bits, has_values, n);
  // The histogram's 1024-thread workgroups use 64 KiB of LDS each, so two
  // fit a CU: a grid of two per CU is resident at once (at 2^28 u32 keys
  // 244 us against 250 us with four per CU, which runs in two rounds).
  r->hist_blocks_per_cu = 2;
  r->digit_bits = kRadixBits;
  r->algorithm = ONESWEEP_ALGORITHM_ONESWEEP;
  r->strip_log2 = kDefaultStripLog2;
  r->order = key_order(key_bits, ONESWEEP_KEY_UNSIGNED, false);
  r->spin_limit = kDefaultSpinLimit;
  r->trace = nullptr;
  if (cfg != nullptr) {
    if (cfg->digit_bits != 0 && (cfg->digit_bits < kMinDigitBits || cfg->digit_bits > kRadixBits))
      return fail(ONESWEEP_ERROR_UNSUPPORTED, "digit_bits %d not built (%d to %d)",
                  cfg->digit_bits, kMinDigitBits, kRadixBits);
    if (cfg->digit_bits != 0) r->digit_bits = cfg->digit_bits;
    if (cfg->block_threads != 0) r->shape.block = cfg->block_threads;
    if (cfg->items_per_thread != 0) r->shape.ipt = cfg->items_per_thread;
    if (cfg->hist_blocks_per_cu < 0 || cfg->hist_blocks_per_cu > 64)
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "hist_blocks_per_cu %d out of [0, 64]",
                  cfg->hist_blocks_per_cu);
    if (cfg->hist_blocks_per_cu != 0) r->hist_blocks_per_cu = cfg->hist_blocks_per_cu;
    if (cfg->rank_algorithm < 0 || cfg->rank_algorithm > 3)
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "rank_algorithm %d not in [0, 3]",
                  cfg->rank_algorithm);
    if (cfg->rank_algorithm != 0) r->shape.rank = cfg->rank_algorithm - 1;
    if (cfg->algorithm != ONESWEEP_ALGORITHM_ONESWEEP &&
        cfg->algorithm != ONESWEEP_ALGORITHM_REDUCE_THEN_SCAN)
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "algorithm %d not 0 or 1", cfg->algorithm);
    if (cfg->algorithm != ONESWEEP_ALGORITHM_ONESWEEP && caller != kCallSort)
      return fail(ONESWEEP_ERROR_INVALID_VALUE,
                  "algorithm %d: reduce-then-scan is offered by whole plain sorts only",
                  cfg->algorithm);
    r->algorithm = cfg->algorithm;
    if (cfg->strip_log2 != 0 && (cfg->strip_log2 < 11 || cfg->strip_log2 > kDefaultStripLog2))
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "strip_log2 %d not 0 or in [11, %d]",
                  cfg->strip_log2, kDefaultStripLog2);
    if (cfg->strip_log2 != 0) r->strip_log2 = cfg->strip_log2;
    if (cfg->key_type < ONESWEEP_KEY_UNSIGNED || cfg->key_type > ONESWEEP_KEY_FLOAT)
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "key_type %d not 0, 1 or 2", cfg->key_type);
    if (cfg->descending != 0 && cfg->descending != 1)
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "descending %d not 0 or 1", cfg->descending);
    if (key_bits == 32 || key_bits == 64)
      r->order = key_order(key_bits, cfg->key_type, cfg->descending != 0);
    if (cfg->lookback_spin_limit < 0)
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "lookback_spin_limit %d is negative",
                  cfg->lookback_spin_limit);
    if (cfg->lookback_spin_limit != 0) r->spin_limit = static_cast<uint32_t>(cfg->lookback_spin_limit);
    r->trace = cfg->trace;
    if (r->trace && (r->trace->capacity < 0 || r->trace->capacity > ONESWEEP_TRACE_MAX ||
                     (r->trace->capacity > 0 && r->trace->events == nullptr)))
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "trace capacity/events invalid");
  }
  const bool rts = r->algorithm == ONESWEEP_ALGORITHM_REDUCE_THEN_SCAN;
  const int mode = caller == kCallSegments ? kBinSegmented : (rts ? kBinDownsweep : kBinChained);
  const bool wide = caller == kCallSort && wide_positions(n, key_bits);
  if (wide && rts)
    return fail(ONESWEEP_ERROR_UNSUPPORTED,
                "reduce-then-scan is built for key outputs of at most 4 GiB (n = %zu)", n);
  if (!binning_shape_supported(r->shape, mode, wide) ||
      (rts && !upsweep_shape_supported(key_bits, r->shape.block, r->shape.ipt)))
    return fail(ONESWEEP_ERROR_UNSUPPORTED,
                "%sbinning shape (key_bits=%d, values=%d, block=%d, items=%d, rank=%d) not built",
                mode == kBinSegmented ? "segmented "
                                      : (rts ? "reduce-then-scan " : (wide ? "64-bit-position " : "")),
                key_bits, (int)has_values, r->shape.block, r->shape.ipt, r->shape.rank + 1);
  return ONESWEEP_SUCCESS;
}

// Temporary storage of a full sort. The cleared region (histograms, tile
// counters, status words) is contiguous so one kernel clears it.
struct SortLayout {
  size_t hist, counters, status, zero_end;
  size_t offsets, strip_offsets, plan, tmp_keys, tmp_vals, total;
  uint32_t tiles;
  uint32_t strip_tiles, strips;  // tiles per strip, strips per binning pass
  size_t status_words_per_place;
  size_t tiles_for_layout;       // the tile size the layout was computed for
};

// Reduce-then-scan keeps one count table of the same size as a place's
// status words, reused by every place and not cleared (the upsweep writes
// every entry); only the histograms and tile counters are cleared.
// Onesweep strips: `strip_log2` bounds a strip to 2^strip_log2 keys (whole
// tiles, at least one); strip k > 0 of place j reads its bin starts from
// strip_offsets[(j * strips + k) * 256], written by strip k - 1. Each
// (place, strip) has its own tile counter.
// With a late tile choice (`late_status`), the status rows go last, sized for
// `tile` (the smallest choice), and are not part of the first cleared
// region: they are cleared once the tile is chosen, as many as it needs.
SortLayout sort_layout(size_t n, int key_bits, bool has_values, int places, size_t tile,
                       bool rts = false, int strip_log2 = kDefaultStripLog2,
                       bool late_status = false) {
  SortLayout L{};
  L.tiles_for_layout = tile;
  const size_t cw = wide_positions(n, key_bits) ? 8 : 4;  // bytes of a count, offset or bin start
  L.tiles = static_cast<uint32_t>((n + tile - 1) / tile);
  L.status_words_per_place = static_cast<size_t>(L.tiles) * kRadix;
  L.strip_tiles = static_cast<uint32_t>(std::max<size_t>(1, (size_t(1) << strip_log2) / tile));
  L.strips = rts ? 1u : std::max<uint32_t>(1u, (L.tiles + L.strip_tiles - 1) / L.strip_tiles);
  if (rts) L.strip_tiles = std::max<uint32_t>(L.tiles, 1u);
  size_t off = 0;
  L.hist = off;
  off += align_up(cw * kMaxPlaces * kRadix);
  L.counters = off;
  off += align_up(sizeof(uint32_t) * static_cast<size_t>(std::max(places, 1)) * L.strips);
  L.status = off;
  if (rts || late_status) {
    L.zero_end = off;
    if (!late_status)
      off += align_up(sizeof(uint32_t) * L.status_words_per_place * (places > 0 ? 1 : 0));
  } else {
    off += align_up(sizeof(uint32_t) * L.status_words_per_place * places);
    L.zero_end = off;
  }
  L.offsets = off;
  off += align_up(cw * kMaxPlaces * kRadix);
  L.strip_offsets = off;
  if (L.strips > 1)
    off += align_up(cw * kRadix * static_cast<size_t>(places) * L.strips);
  L.plan = off;
  off += kAlign;
  L.tmp_keys = off;
  off += align_up(n * (key_bits / 8));
  L.tmp_vals = off;
  if (has_values) off += align_up(n * sizeof(uint32_t));
  if (late_status) {
    L.status = off;
    off += align_up(sizeof(uint32_t) * L.status_words_per_place * places);
  }
  L.total = off;
  return L;
}

bool ranges_overlap(const void *a, size_t abytes, const void *b, size_t bbytes) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

// Records events around launches when tracing is on.
struct Tracer {
  onesweep_trace_t *t;
  hipStream_t stream;
  int next = 0;
  Tracer(onesweep_trace_t *tr, hipStream_t s) : t(tr), stream(s) {
    if (t) t->count = 0;
  }
  hipError_t before(int kind) {
    if (!t || next >= t->capacity) return hipSuccess;
    t->kinds[next] = kind;
    return hipEventRecord(static_cast<hipEvent_t>(t->events[2 * next]), stream);
  }
  hipError_t after() {
    if (!t || next >= t->capacity) return hipSuccess;
    hipError_t e = hipEventRecord(static_cast<hipEvent_t>(t->events[2 * next + 1]), stream);
    ++next;
    t->count = next;
    return e;
  }
};

#define ONESWEEP_LAUNCH(tracer, kind, what, expr)          \
  do {                                                     \
    hipError_t e_ = (tracer).before(kind);                 \
    if (e_ == hipSuccess) e_ = (expr);                     \
    if (e_ == hipSuccess) e_ = (tracer).after();           \
    if (e_ != hipSuccess) return hip_fail(e_, what);       \
  } while (0)

onesweep_status_t check_common(size_t *temp_bytes, size_t n, int key_bits, int begin_bit,
                               int end_bit, size_t max_n = kMaxN) {
  if (temp_bytes == nullptr) return fail(ONESWEEP_ERROR_INVALID_VALUE, "temp_bytes is NULL");
  if (key_bits != 32 && key_bits != 64)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key_bits %d is not 32 or 64", key_bits);
  if (begin_bit < 0 || begin_bit > end_bit || end_bit > key_bits)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "bit range [%d, %d) invalid for %d-bit keys",
                begin_bit, end_bit, key_bits);
  if (n >= max_n)
    return fail(ONESWEEP_ERROR_TOO_LARGE, "n = %zu is not below 2^%d", n,
                max_n == kMaxSortN ? 36 : 30);
  return ONESWEEP_SUCCESS;
}

// Digit places of [begin_bit, end_bit) at the resolved digit width; a sort
// covers at most kMaxPlaces of them.
onesweep_status_t places_of(int begin_bit, int end_bit, const Resolved &rc, int *places) {
  *places = num_places(begin_bit, end_bit, rc.digit_bits);
  if (*places > kMaxPlaces)
    return fail(ONESWEEP_ERROR_UNSUPPORTED, "%d-bit digits make %d places of bits [%d, %d); at most %d",
                rc.digit_bits, *places, begin_bit, end_bit, kMaxPlaces);
  return ONESWEEP_SUCCESS;
}

onesweep_status_t sort_impl(void *d_temp, size_t *temp_bytes, const void *keys_in,
                            void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                            bool has_values, size_t n, int key_bits, int begin_bit, int end_bit,
                            const onesweep_config_t *cfg, hipStream_t stream,
                            const LateChoice *late = nullptr) {
  g_error[0] = '\0';
  onesweep_status_t st = check_common(temp_bytes, n, key_bits, begin_bit, end_bit, kMaxSortN);
  if (st) return st;
  Resolved rc;
  if ((st = resolve(key_bits, has_values, n, cfg, &rc, kCallSort))) return st;
  int places = 0;
  if ((st = places_of(begin_bit, end_bit, rc, &places))) return st;
  size_t tile = binning_tile_items(rc.shape);
  const bool rts = rc.algorithm == ONESWEEP_ALGORITHM_REDUCE_THEN_SCAN;
  if (late && (rts || n > kLateChoiceMaxN || late->layout_tile == 0))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "late tile choice needs Onesweep and n <= 2^28");
  // Temporary storage: laid out for the smallest tile a late choice can make
  // (most tiles, so the largest status region); at most 2^28 keys, one strip
  // whatever the tile.
  const SortLayout L = sort_layout(n, key_bits, has_values, places,
                                   late ? std::min(tile, late->layout_tile) : tile, rts,
                                   rc.strip_log2, late != nullptr);
  if (d_temp == nullptr) {
    *temp_bytes = L.total;
    return ONESWEEP_SUCCESS;
  }
  if (rc.trace) rc.trace->count = 0;
  if (n == 0) return ONESWEEP_SUCCESS;
  if (*temp_bytes < L.total)
    return fail(ONESWEEP_ERROR_INSUFFICIENT_TEMP, "temp storage %zu bytes, need %zu",
                *temp_bytes, L.total);
  const size_t kb = static_cast<size_t>(key_bits / 8);
  if (!keys_in || !keys_out) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL key pointer");
  if (has_values && (!vals_in || !vals_out))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL value pointer");
  if ((reinterpret_cast<uintptr_t>(d_temp) & (kAlign - 1)) != 0)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "d_temp is not 256-byte aligned");
  if ((reinterpret_cast<uintptr_t>(keys_in) | reinterpret_cast<uintptr_t>(keys_out)) & (kb - 1))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key pointers not %zu-byte aligned", kb);
  if (has_values &&
      ((reinterpret_cast<uintptr_t>(vals_in) | reinterpret_cast<uintptr_t>(vals_out)) & 3u))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "value pointers not 4-byte aligned");
  const bool keys_alias = keys_in == keys_out;
  if (!keys_alias && ranges_overlap(keys_in, n * kb, keys_out, n * kb))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key input and output partially overlap");
  bool vals_alias = false;
  if (has_values) {
    vals_alias = vals_in == vals_out;
    if (!vals_alias && ranges_overlap(vals_in, n * 4, vals_out, n * 4))
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "value input and output partially overlap");
    if (ranges_overlap(keys_in, n * kb, vals_out, n * 4) ||
        ranges_overlap(keys_out, n * kb, vals_in, n * 4) ||
        ranges_overlap(keys_out, n * kb, vals_out, n * 4))
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "key and value buffers overlap");
  }
  if (ranges_overlap(d_temp, L.total, keys_in, n * kb) ||
      ranges_overlap(d_temp, L.total, keys_out, n * kb) ||
      (has_values && (ranges_overlap(d_temp, L.total, vals_in, n * 4) ||
                      ranges_overlap(d_temp, L.total, vals_out, n * 4))))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "temp storage overlaps keys or values");
  const bool alias = keys_alias || vals_alias;

  int cus = 0;
  if ((st = device_cus(&cus))) return st;
  const uint32_t stream_grid = static_cast<uint32_t>(cus) * 4u;
  Tracer tr(rc.trace, stream);
  char *temp = static_cast<char *>(d_temp);

  CopyArgs ca{};
  ca.keys[kBufIn] = const_cast<void *>(keys_in);
  ca.keys[kBufOut] = keys_out;
  ca.keys[kBufTmp] = temp + L.tmp_keys;
  ca.vals[kBufIn] = const_cast<uint32_t *>(vals_in);
  ca.vals[kBufOut] = vals_out;
  ca.vals[kBufTmp] = has_values ? reinterpret_cast<uint32_t *>(temp + L.tmp_vals) : nullptr;
  ca.n = n;
  ca.key_bytes = static_cast<int>(kb);

  if (places == 0) {  // empty bit range: the sorted order is the input order
    ca.plan = nullptr;
    if (!alias || (has_values && keys_alias != vals_alias))
      ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_COPY, "copy", launch_copy(ca, stream_grid, stream));
    return ONESWEEP_SUCCESS;
  }

  // Sorts of 2^31 elements or more, or of more than 4 GiB of keys, keep
  // 64-bit counts, bin offsets and positions.
  const bool wide = wide_positions(n, key_bits);
  uint32_t *hist = wide ? nullptr : reinterpret_cast<uint32_t *>(temp + L.hist);
  unsigned long long *hist64 =
      wide ? reinterpret_cast<unsigned long long *>(temp + L.hist) : nullptr;
  uint32_t *counters = reinterpret_cast<uint32_t *>(temp + L.counters);
  uint32_t *status = reinterpret_cast<uint32_t *>(temp + L.status);
  uint32_t *offsets = wide ? nullptr : reinterpret_cast<uint32_t *>(temp + L.offsets);
  unsigned long long *offsets64 =
      wide ? reinterpret_cast<unsigned long long *>(temp + L.offsets) : nullptr;
  PassPlan *plan = reinterpret_cast<PassPlan *>(temp + L.plan);

  ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_RESET, "clear",
                  launch_fill_zero(temp + L.hist, L.zero_end - L.hist, stream_grid, stream));
  // Histogram portions of at most 2^30 keys (one launch below 2^30 keys);
  // one launch counts at most one place per key byte, so digits narrower
  // than 8 bits over more places take a launch per group of places. With a
  // late tile choice the selection kernel (one 1024-thread workgroup) runs
  // beside the histogram: one histogram workgroup fewer per XCD (workgroups
  // go to the eight XCDs in turn, and so may the selection's) leaves it room
  // on a CU from the start; else it waits for the histogram's workgroups to
  // finish, and the binning passes wait for it.
  constexpr uint32_t kXcds = 8;
  const int group = key_bits / 8;
  const uint32_t hist_grid =
      static_cast<uint32_t>(cus * rc.hist_blocks_per_cu) - (late != nullptr ? kXcds : 0u);
  for (size_t done = 0; done < n; done += kHistPortion) {
    const size_t part = std::min(kHistPortion, n - done);
    for (int g = 0; g < places; g += group) {
      const int lo = begin_bit + g * rc.digit_bits;
      const int hi = std::min(end_bit, lo + group * rc.digit_bits);
      const int gp = std::min(group, places - g);
      ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_HISTOGRAM, "histogram",
                      launch_histogram(key_bits, static_cast<const char *>(keys_in) + done * kb,
                                       hist ? hist + static_cast<size_t>(g) * kRadix : nullptr,
                                       hist64 ? hist64 + static_cast<size_t>(g) * kRadix : nullptr,
                                       static_cast<uint32_t>(part), lo, hi, gp, rc.digit_bits,
                                       rc.order, hist_grid, stream));
    }
  }
  ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_SCAN, "scan",
                  launch_scan(hist, hist64, offsets, offsets64, plan, places, n, alias, stream));
  if (late) {
    // The binning tile shape is decided now, while the kernels above run.
    onesweep_config_t c = cfg ? *cfg : onesweep_config_t{};
    if ((st = late->choose(late->ctx, &c))) return st;
    Resolved picked;
    if ((st = resolve(key_bits, has_values, n, &c, &picked, kCallSort))) return st;
    if (binning_tile_items(picked.shape) < L.tiles_for_layout)
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "chosen tile below the laid-out tile");
    rc.shape = picked.shape;
    tile = binning_tile_items(rc.shape);
  }
  // Launch geometry of the binning passes (the regions are L's).
  const SortLayout G = sort_layout(n, key_bits, has_values, places, tile, rts, rc.strip_log2);
  // With a late choice the status rows of every place are packed for the
  // chosen tile and cleared now, only as many as it needs.
  const size_t status_stride = late ? G.status_words_per_place : L.status_words_per_place;
  if (late)
    ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_RESET, "clear",
                    launch_fill_zero(status, sizeof(uint32_t) * status_stride * places,
                                     stream_grid, stream));
  // One place: the reduce-then-scan upsweep and tile scan when that algorithm
  // runs, then the binning (or downsweep) launches, one per strip. Idx is the
  // type of element positions, counts and bin offsets.
  auto bin_place = [&](auto key_tag, auto idx_tag, int j) -> onesweep_status_t {
    using K = decltype(key_tag);
    using Idx = decltype(idx_tag);
    Idx *strip_offsets = reinterpret_cast<Idx *>(temp + L.strip_offsets);
    const Idx *place_offsets = reinterpret_cast<const Idx *>(temp + L.offsets) + j * kRadix;
    const int lo = begin_bit + j * rc.digit_bits;
    const int width = (lo + rc.digit_bits <= end_bit) ? rc.digit_bits : end_bit - lo;
    // Onesweep: place j's own status words; reduce-then-scan: the shared
    // count table, filled by the upsweep and scanned before the downsweep.
    uint32_t *table = rts ? status : status + j * status_stride;
    if (rts) {
      UpsweepArgs<K> u{};
      for (int b = 0; b < 3; ++b) u.keys[b] = static_cast<K *>(ca.keys[b]);
      u.plan = plan;
      u.order = rc.order;
      u.counts = table;
      u.n = static_cast<uint32_t>(n);
      u.place = j;
      u.shift = lo;
      u.width = width;
      ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_UPSWEEP, "upsweep",
                      launch_upsweep(key_bits, rc.shape.block, rc.shape.ipt, &u, G.tiles,
                                     stream));
      ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_TILE_SCAN, "tile scan",
                      launch_tile_scan(table, G.tiles, plan, j, stream));
    }
    Idx *place_strips = strip_offsets + static_cast<size_t>(j) * G.strips * kRadix;
    for (uint32_t k = 0; k < G.strips; ++k) {
      BinningArgs<K, Idx> a{};
      for (int b = 0; b < 3; ++b) a.keys[b] = static_cast<K *>(ca.keys[b]);
      for (int b = 0; b < 3; ++b) a.vals[b] = ca.vals[b];
      a.bin_offsets = k == 0 ? place_offsets : place_strips + k * kRadix;
      a.next_bin_offsets = k + 1 < G.strips ? place_strips + (k + 1) * kRadix : nullptr;
      a.tile_first = k * G.strip_tiles;
      a.status = table;
      a.tile_counter = counters + static_cast<size_t>(j) * G.strips + k;
      a.plan = plan;
      a.order = rc.order;
      a.lookback_error = &plan->lookback_error;
      a.spin_limit = rc.spin_limit;
      a.n = static_cast<Idx>(n);
      a.place = j;
      a.shift = lo;
      a.width = width;
      const uint32_t grid = std::min(G.strip_tiles, G.tiles - a.tile_first);
      ONESWEEP_LAUNCH(tr, rts ? ONESWEEP_KERNEL_DOWNSWEEP : ONESWEEP_KERNEL_BINNING, "binning",
                      launch_binning(rc.shape, rts ? kBinDownsweep : kBinChained, &a, grid,
                                     stream, wide));
    }
    return ONESWEEP_SUCCESS;
  };
  for (int j = 0; j < places; ++j) {
    if (key_bits == 32)
      st = wide ? bin_place(uint32_t{}, uint64_t{}, j) : bin_place(uint32_t{}, uint32_t{}, j);
    else
      st = wide ? bin_place(uint64_t{}, uint64_t{}, j) : bin_place(uint64_t{}, uint32_t{}, j);
    if (st) return st;
  }
  ca.plan = plan;
  ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_COPY, "copy", launch_copy(ca, stream_grid, stream));
  return ONESWEEP_SUCCESS;
}

}  // namespace

onesweep_status_t sort_late_choice(void *d_temp, size_t *temp_bytes, const void *keys_in,
                                   void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                                   bool has_values, size_t n, int key_bits, int begin_bit,
                                   int end_bit, const onesweep_config_t *cfg, hipStream_t stream,
                                   const LateChoice &late) {
  return sort_impl(d_temp, temp_bytes, keys_in, keys_out, vals_in, vals_out, has_values, n,
                   key_bits, begin_bit, end_bit, cfg, stream, &late);
}

namespace {

// ------------------------------------------------------------ segmented sort

// Length limits of the LDS classes after applying the config: class c takes
// lengths in (limit[c - 1], limit[c]]; an unused class repeats the previous
// limit.
onesweep_status_t segment_limits(const onesweep_config_t *cfg, uint32_t limit[kSegClasses]) {
  if (cfg && (cfg->segment_streams < 0 || cfg->segment_streams > 1))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "segment_streams %d not 0 or 1",
                cfg->segment_streams);
  uint32_t prev = 0;
  for (int c = 0; c < kSegClasses; ++c) {
    const int cap = lds_class_capacity(c);
    const int v = cfg ? cfg->segment_limits[c] : 0;
    if (v < -1 || v > cap)
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "segment_limits[%d] = %d not in [-1, %d]", c, v,
                  cap);
    if (v != -1) prev = std::max(prev, static_cast<uint32_t>(v == 0 ? cap : v));
    limit[c] = prev;
  }
  return ONESWEEP_SUCCESS;
}

// Temporary storage of a segmented sort. Bounds hold for any valid offsets:
// a class whose lengths exceed L has at most n / (L + 1) segments, and the
// large segments have at most floor(n / T) + (number of large segments) tiles.
struct SegmentLayout {
  uint32_t capacity[kSegClasses];
  uint32_t max_large, max_tiles;
  size_t plan, counters, lists[kSegClasses], tile_info, large_len, hist, status, tmp_keys,
      tmp_vals, total;
  size_t status_words_per_place;
};

SegmentLayout segment_layout(size_t n, size_t num_segments, int key_bits, bool has_values,
                             int places, size_t tile, const uint32_t limit[kSegClasses]) {
  SegmentLayout L{};
  uint32_t prev = 0;
  for (int c = 0; c < kSegClasses; ++c) {
    L.capacity[c] = limit[c] > prev
                        ? static_cast<uint32_t>(std::min(num_segments, n / (size_t(prev) + 1)))
                        : 0u;
    prev = limit[c];
  }
  L.max_large = places > 0 ? static_cast<uint32_t>(std::min(num_segments, n / (size_t(prev) + 1)))
                           : 0u;
  L.max_tiles = L.max_large ? static_cast<uint32_t>(n / tile) + L.max_large : 0u;
  L.status_words_per_place = static_cast<size_t>(L.max_tiles) * kRadix;
  size_t off = 0;
  L.plan = off;
  off += kAlign;
  L.counters = off;
  off += kAlign;
  for (int c = 0; c < kSegClasses; ++c) {
    L.lists[c] = off;
    off += align_up(sizeof(uint32_t) * L.capacity[c]);
  }
  L.tile_info = off;
  off += align_up(sizeof(uint4) * L.max_tiles);
  L.large_len = off;
  off += align_up(sizeof(uint32_t) * L.max_large);
  L.hist = off;
  off += align_up(sizeof(uint32_t) * kRadix * places * static_cast<size_t>(L.max_large));
  L.status = off;
  off += align_up(sizeof(uint32_t) * L.status_words_per_place * places);
  L.tmp_keys = off;
  if (L.max_large) off += align_up(n * (key_bits / 8));
  L.tmp_vals = off;
  if (L.max_large && has_values) off += align_up(n * sizeof(uint32_t));
  L.total = off;
  return L;
}

// Resident workgroups per CU of each LDS class, cached per device.
std::atomic<int> g_lds_occupancy[64][2][2][kSegClasses];

onesweep_status_t lds_blocks_per_cu(int key_bits, bool has_values, int cls, int *blocks) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::atomic<int> *slot =
      (dev >= 0 && dev < 64) ? &g_lds_occupancy[dev][key_bits == 64][has_values][cls] : nullptr;
  if (slot && slot->load(std::memory_order_relaxed) > 0) {
    *blocks = slot->load(std::memory_order_relaxed);
    return ONESWEEP_SUCCESS;
  }
  int b = 0;
  e = lds_sort_blocks_per_cu(key_bits, has_values, cls, &b);
  if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  if (b <= 0) b = 1;
  if (slot) slot->store(b, std::memory_order_relaxed);
  *blocks = b;
  return ONESWEEP_SUCCESS;
}

// The segmented sort's second stream: after classify, the LDS-sort classes
// run on it while the large segments are binned on the caller's stream (the
// two touch disjoint key ranges), joined back through an event. One stream
// and two events per device, created on first use outside graph capture and
// kept for the life of the process; the lock serialises the enqueue of the
// fork/join pair across host threads.
struct SegmentStreams {
  std::mutex lock;
  bool ready = false;
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
SegmentStreams g_segment_streams[64];

onesweep_status_t segment_streams(hipStream_t stream, SegmentStreams **out,
                                  std::unique_lock<std::mutex> *hold) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return ONESWEEP_SUCCESS;
  SegmentStreams &r = g_segment_streams[dev];
  std::unique_lock<std::mutex> lk(r.lock);
  if (!r.ready) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      return ONESWEEP_SUCCESS;  // cannot create resources while capturing: one stream
    e = hipStreamCreateWithFlags(&r.aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r.join, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "segmented sort stream setup");
    r.ready = true;
  }
  *hold = std::move(lk);
  *out = &r;
  return ONESWEEP_SUCCESS;
}

onesweep_status_t segments_impl(void *d_temp, size_t *temp_bytes, const void *keys_in,
                                void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                                bool has_values, size_t n, const uint32_t *seg_offsets,
                                size_t num_segments, int key_bits, int begin_bit, int end_bit,
                                const onesweep_config_t *cfg, hipStream_t stream) {
  g_error[0] = '\0';
  onesweep_status_t st = check_common(temp_bytes, n, key_bits, begin_bit, end_bit);
  if (st) return st;
  if (num_segments >= kMaxN)
    return fail(ONESWEEP_ERROR_TOO_LARGE, "num_segments = %zu is not below 2^30", num_segments);
  if (num_segments == 0 && n != 0)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "%zu keys but no segment", n);
  Resolved rc;
  if ((st = resolve(key_bits, has_values, n, cfg, &rc, kCallSegments))) return st;
  uint32_t limit[kSegClasses];
  if ((st = segment_limits(cfg, limit))) return st;
  int places = 0;
  if ((st = places_of(begin_bit, end_bit, rc, &places))) return st;
  const size_t tile = binning_tile_items(rc.shape);
  const SegmentLayout L =
      segment_layout(n, num_segments, key_bits, has_values, places, tile, limit);
  if (d_temp == nullptr) {
    *temp_bytes = L.total;
    return ONESWEEP_SUCCESS;
  }
  if (rc.trace) rc.trace->count = 0;
  if (n == 0) return ONESWEEP_SUCCESS;
  if (*temp_bytes < L.total)
    return fail(ONESWEEP_ERROR_INSUFFICIENT_TEMP, "temp storage %zu bytes, need %zu",
                *temp_bytes, L.total);
  const size_t kb = static_cast<size_t>(key_bits / 8);
  if (!keys_in || !keys_out) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL key pointer");
  if (has_values && (!vals_in || !vals_out))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL value pointer");
  if (!seg_offsets) return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL segment offsets");
  if ((reinterpret_cast<uintptr_t>(d_temp) & (kAlign - 1)) != 0)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "d_temp is not 256-byte aligned");
  if ((reinterpret_cast<uintptr_t>(keys_in) | reinterpret_cast<uintptr_t>(keys_out)) & (kb - 1))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key pointers not %zu-byte aligned", kb);
  if ((has_values &&
       ((reinterpret_cast<uintptr_t>(vals_in) | reinterpret_cast<uintptr_t>(vals_out)) & 3u)) ||
      (reinterpret_cast<uintptr_t>(seg_offsets) & 3u))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "value or offset pointers not 4-byte aligned");
  const bool keys_alias = keys_in == keys_out;
  if (!keys_alias && ranges_overlap(keys_in, n * kb, keys_out, n * kb))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key input and output partially overlap");
  bool vals_alias = false;
  if (has_values) {
    vals_alias = vals_in == vals_out;
    if (!vals_alias && ranges_overlap(vals_in, n * 4, vals_out, n * 4))
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "value input and output partially overlap");
    if (ranges_overlap(keys_in, n * kb, vals_out, n * 4) ||
        ranges_overlap(keys_out, n * kb, vals_in, n * 4) ||
        ranges_overlap(keys_out, n * kb, vals_out, n * 4))
      return fail(ONESWEEP_ERROR_INVALID_VALUE, "key and value buffers overlap");
  }
  const size_t off_bytes = (num_segments + 1) * sizeof(uint32_t);
  if (ranges_overlap(seg_offsets, off_bytes, keys_out, n * kb) ||
      (has_values && ranges_overlap(seg_offsets, off_bytes, vals_out, n * 4)) ||
      ranges_overlap(seg_offsets, off_bytes, d_temp, L.total))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "segment offsets overlap an output or temp storage");
  if (ranges_overlap(d_temp, L.total, keys_in, n * kb) ||
      ranges_overlap(d_temp, L.total, keys_out, n * kb) ||
      (has_values && (ranges_overlap(d_temp, L.total, vals_in, n * 4) ||
                      ranges_overlap(d_temp, L.total, vals_out, n * 4))))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "temp storage overlaps keys or values");
  const bool alias = keys_alias || vals_alias;

  int cus = 0;
  if ((st = device_cus(&cus))) return st;
  const uint32_t stream_grid = static_cast<uint32_t>(cus) * 4u;
  Tracer tr(rc.trace, stream);
  char *temp = static_cast<char *>(d_temp);

  if (places == 0) {  // empty bit range: every segment is already in order
    // The offsets are not read; the status word reads 0.
    ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_RESET, "clear",
                    launch_fill_zero(temp + L.plan, kAlign, 1, stream));
    CopyArgs ca{};
    ca.keys[kBufIn] = const_cast<void *>(keys_in);
    ca.keys[kBufOut] = keys_out;
    ca.vals[kBufIn] = const_cast<uint32_t *>(vals_in);
    ca.vals[kBufOut] = vals_out;
    ca.n = static_cast<uint32_t>(n);
    ca.key_bytes = static_cast<int>(kb);
    if (!alias || (has_values && keys_alias != vals_alias))
      ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_COPY, "copy", launch_copy(ca, stream_grid, stream));
    return ONESWEEP_SUCCESS;
  }

  SegmentPlan *plan = reinterpret_cast<SegmentPlan *>(temp + L.plan);
  uint32_t *counters = reinterpret_cast<uint32_t *>(temp + L.counters);
  uint4 *tile_info = reinterpret_cast<uint4 *>(temp + L.tile_info);
  uint32_t *large_len = reinterpret_cast<uint32_t *>(temp + L.large_len);
  uint32_t *hist = reinterpret_cast<uint32_t *>(temp + L.hist);
  uint32_t *status = reinterpret_cast<uint32_t *>(temp + L.status);

  ClassifyArgs ca{};
  ca.offsets = seg_offsets;
  ca.num_segments = static_cast<uint32_t>(num_segments);
  ca.n = static_cast<uint32_t>(n);
  for (int c = 0; c < kSegClasses; ++c) {
    ca.limit[c] = limit[c];
    ca.capacity[c] = L.capacity[c];
    ca.lists[c] = reinterpret_cast<uint32_t *>(temp + L.lists[c]);
  }
  ca.max_large = L.max_large;
  ca.max_tiles = L.max_tiles;
  ca.tile_items = static_cast<uint32_t>(tile);
  ca.tile_info = tile_info;
  ca.large_len = large_len;
  ca.tile_counters = counters;
  ca.plan = plan;
  ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_CLASSIFY, "classify", launch_classify(ca, stream));

  // Both halves present and no per-launch tracing: fork the LDS classes
  // onto the second stream, at half their occupancy so that binning
  // workgroups share the CUs with them.
  bool any_lds = false;
  for (int c = 0; c < kSegClasses; ++c) any_lds = any_lds || L.capacity[c] > 0;
  SegmentStreams *ss = nullptr;
  std::unique_lock<std::mutex> hold;
  if (any_lds && L.max_large > 0 && !rc.trace && !(cfg && cfg->segment_streams == 1))
    if ((st = segment_streams(stream, &ss, &hold))) return st;
  hipStream_t lds_stream = stream;
  if (ss) {
    hipError_t e = hipEventRecord(ss->fork, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(ss->aux, ss->fork, 0);
    if (e != hipSuccess) return hip_fail(e, "segmented sort fork");
    lds_stream = ss->aux;
  }
  for (int c = 0; c < kSegClasses; ++c) {
    if (L.capacity[c] == 0) continue;
    int per_cu = 0;
    if ((st = lds_blocks_per_cu(key_bits, has_values, c, &per_cu))) return st;
    if (ss) per_cu = std::max(1, per_cu / 2);
    LdsSortArgs la{};
    la.keys_in = keys_in;
    la.keys_out = keys_out;
    la.vals_in = vals_in;
    la.vals_out = vals_out;
    la.offsets = seg_offsets;
    la.list = ca.lists[c];
    la.plan = plan;
    la.cls = c;
    la.begin_bit = begin_bit;
    la.end_bit = end_bit;
    la.places = places;
    la.digit_bits = rc.digit_bits;
    la.order = rc.order;
    const uint32_t grid =
        std::min<uint32_t>(L.capacity[c], static_cast<uint32_t>(cus) * static_cast<uint32_t>(per_cu));
    ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_LDS_SORT, "lds sort",
                    launch_lds_sort(key_bits, has_values, la, grid, lds_stream));
  }
  if (ss) {
    hipError_t e = hipEventRecord(ss->join, ss->aux);
    if (e != hipSuccess) return hip_fail(e, "segmented sort join");
  }
  if (L.max_large == 0) return ONESWEEP_SUCCESS;

  SegmentClearArgs za{};
  za.status = status;
  za.status_words_per_place = L.status_words_per_place;
  za.hist = hist;
  za.plan = plan;
  za.places = places;
  ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_RESET, "segment clear",
                  launch_segment_clear(za, stream_grid, stream));
  // Static routing of the large segments' passes: with the input aliasing
  // the output the first pass must not write the output, so the passes go
  // in -> tmp -> out -> tmp ... and an odd count ends with a copy; otherwise
  // the alternation is chosen so that the last pass writes the output.
  void *kbuf[3] = {const_cast<void *>(keys_in), keys_out, temp + L.tmp_keys};
  uint32_t *vbuf[3] = {const_cast<uint32_t *>(vals_in), vals_out,
                       has_values ? reinterpret_cast<uint32_t *>(temp + L.tmp_vals) : nullptr};
  auto buffer_after = [&](int passes_done) -> int {
    if (passes_done == 0) return kBufIn;
    if (alias) return (passes_done & 1) ? kBufTmp : kBufOut;
    return ((places - passes_done) & 1) ? kBufTmp : kBufOut;
  };
  // The first place's launch also counts the digits of every place per
  // segment (its first workgroups), so no separate histogram or scan launch
  // precedes it; each tile turns its segment's counts into bin starts.
  SegmentTiles seg{};
  seg.tile_info = tile_info;
  seg.counts = hist;
  seg.large_len = large_len;
  seg.plan = plan;
  seg.places = places;
  seg.begin_bit = begin_bit;
  seg.end_bit = end_bit;
  seg.digit_bits = rc.digit_bits;
  for (int j = 0; j < places; ++j) {
    const int mode = j == 0 ? kBinSegCounted : kBinSegmented;
    const uint32_t grid = (j == 0 ? 2u : 1u) * L.max_tiles;
    const int lo = begin_bit + j * rc.digit_bits;
    const int width = (lo + rc.digit_bits <= end_bit) ? rc.digit_bits : end_bit - lo;
    const int from = buffer_after(j), to = buffer_after(j + 1);
    if (key_bits == 32) {
      BinningArgs<uint32_t> a{};
      a.keys[kBufIn] = static_cast<uint32_t *>(kbuf[from]);
      a.keys[kBufOut] = static_cast<uint32_t *>(kbuf[to]);
      a.vals[kBufIn] = vbuf[from];
      a.vals[kBufOut] = vbuf[to];
      a.status = status + j * L.status_words_per_place;
      a.tile_counter = counters + j;
      a.seg = seg;
      a.order = rc.order;
      a.lookback_error = &plan->lookback_error;
      a.spin_limit = rc.spin_limit;
      a.n = static_cast<uint32_t>(n);
      a.place = j;
      a.shift = lo;
      a.width = width;
      ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_BINNING, "segment binning",
                      launch_binning(rc.shape, mode, &a, grid, stream));
    } else {
      BinningArgs<uint64_t> a{};
      a.keys[kBufIn] = static_cast<uint64_t *>(kbuf[from]);
      a.keys[kBufOut] = static_cast<uint64_t *>(kbuf[to]);
      a.vals[kBufIn] = vbuf[from];
      a.vals[kBufOut] = vbuf[to];
      a.status = status + j * L.status_words_per_place;
      a.tile_counter = counters + j;
      a.seg = seg;
      a.order = rc.order;
      a.lookback_error = &plan->lookback_error;
      a.spin_limit = rc.spin_limit;
      a.n = static_cast<uint32_t>(n);
      a.place = j;
      a.shift = lo;
      a.width = width;
      ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_BINNING, "segment binning",
                      launch_binning(rc.shape, mode, &a, grid, stream));
    }
  }
  if (buffer_after(places) != kBufOut) {
    SegmentCopyArgs pa{};
    pa.keys_src = kbuf[kBufTmp];
    pa.keys_dst = keys_out;
    pa.vals_src = vbuf[kBufTmp];
    pa.vals_dst = vals_out;
    pa.tile_info = tile_info;
    pa.plan = plan;
    pa.key_bytes = static_cast<int>(kb);
    ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_COPY, "segment copy",
                    launch_segment_copy(pa, std::min(L.max_tiles, stream_grid), stream));
  }
  if (ss) {
    hipError_t e = hipStreamWaitEvent(stream, ss->join, 0);
    if (e != hipSuccess) return hip_fail(e, "segmented sort join");
  }
  return ONESWEEP_SUCCESS;
}

// ------------------------------------------------ allocation-free keys sort

// Temporary storage of onesweep_sort_keys_noalloc: one array per GPU, loaded
// with the library's code object and kept until the process ends. Host code
// never uses the array's name as an address (in host code it is only a
// stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, resolved once per device.
constexpr size_t kNoAllocScratchBytes = size_t(ONESWEEP_NOALLOC_SCRATCH_BYTES);
static_assert(kNoAllocScratchBytes % kAlign == 0, "scratch is a whole number of 256-byte slots");

std::mutex g_scratch_mutex;
void *g_scratch_ptr[64];  // per device id, guarded by g_scratch_mutex

}  // namespace
}  // namespace onesweep

static __device__ __align__(256) unsigned char scratch[onesweep::kNoAllocScratchBytes];

namespace onesweep {
namespace {

// Device address of the current device's scratch array.
onesweep_status_t scratch_address(void **ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(ONESWEEP_ERROR_UNSUPPORTED, "device id %d not below 64", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (p == nullptr || (reinterpret_cast<uintptr_t>(p) & (kAlign - 1)) != 0)
      return fail(ONESWEEP_ERROR_HIP, "scratch array address %p is not 256-byte aligned", p);
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return ONESWEEP_SUCCESS;
}

}  // namespace
}  // namespace onesweep

using namespace onesweep;

extern "C" {

onesweep_status_t onesweep_sort_keys_noalloc(const void *d_keys_in, void *d_keys_out, size_t n,
                                             int key_bits, int begin_bit, int end_bit,
                                             int stable, const onesweep_config_t *cfg,
                                             onesweep_stream_t stream) {
  (void)stable;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  size_t need = 0;
  onesweep_status_t st = sort_impl(nullptr, &need, d_keys_in, d_keys_out, nullptr, nullptr, false,
                                   n, key_bits, begin_bit, end_bit, cfg, s);
  if (st) return st;
  if (need > kNoAllocScratchBytes)
    return fail(ONESWEEP_ERROR_TOO_LARGE,
                "n = %zu %d-bit keys need %zu bytes of temporary storage; the allocation-free "
                "sort has %zu (use onesweep_sort_keys)",
                n, key_bits, need, kNoAllocScratchBytes);
  if (n == 0) return ONESWEEP_SUCCESS;
  void *temp = nullptr;
  if ((st = scratch_address(&temp))) return st;
  size_t have = kNoAllocScratchBytes;
  return sort_impl(temp, &have, d_keys_in, d_keys_out, nullptr, nullptr, false, n, key_bits,
                   begin_bit, end_bit, cfg, s);
}

onesweep_status_t onesweep_sort_keys(void *d_temp, size_t *temp_bytes, const void *d_keys_in,
                                     void *d_keys_out, size_t n, int key_bits, int begin_bit,
                                     int end_bit, int stable, const onesweep_config_t *cfg,
                                     onesweep_stream_t stream) {
  (void)stable;
  return sort_impl(d_temp, temp_bytes, d_keys_in, d_keys_out, nullptr, nullptr, false, n,
                   key_bits, begin_bit, end_bit, cfg, reinterpret_cast<hipStream_t>(stream));
}

onesweep_status_t onesweep_sort_pairs(void *d_temp, size_t *temp_bytes, const void *d_keys_in,
                                      void *d_keys_out, const uint32_t *d_vals_in,
                                      uint32_t *d_vals_out, size_t n, int key_bits,
                                      int begin_bit, int end_bit, int stable,
                                      const onesweep_config_t *cfg, onesweep_stream_t stream) {
  (void)stable;
  return sort_impl(d_temp, temp_bytes, d_keys_in, d_keys_out, d_vals_in, d_vals_out, true, n,
                   key_bits, begin_bit, end_bit, cfg, reinterpret_cast<hipStream_t>(stream));
}

onesweep_status_t onesweep_histogram(const void *d_keys, size_t n, int key_bits, int begin_bit,
                                     int end_bit, uint32_t *d_hist,
                                     const onesweep_config_t *cfg, onesweep_stream_t stream) {
  g_error[0] = '\0';
  size_t dummy = 0;
  onesweep_status_t st = check_common(&dummy, n, key_bits, begin_bit, end_bit);
  if (st) return st;
  Resolved rc;
  if ((st = resolve(key_bits, false, n, cfg, &rc))) return st;
  int places = 0;
  if ((st = places_of(begin_bit, end_bit, rc, &places))) return st;
  if (places == 0) return ONESWEEP_SUCCESS;
  if (!d_hist) return fail(ONESWEEP_ERROR_INVALID_VALUE, "d_hist is NULL");
  if (n > 0 && !d_keys) return fail(ONESWEEP_ERROR_INVALID_VALUE, "d_keys is NULL");
  if (reinterpret_cast<uintptr_t>(d_keys) & (key_bits / 8 - 1))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "d_keys not aligned to the key size");
  if (reinterpret_cast<uintptr_t>(d_hist) & 3u)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "d_hist not 4-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int cus = 0;
  if ((st = device_cus(&cus))) return st;
  Tracer tr(rc.trace, s);
  ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_RESET, "clear",
                  launch_fill_zero(d_hist, sizeof(uint32_t) * places * kRadix, 1, s));
  if (n == 0) return ONESWEEP_SUCCESS;
  const int group = key_bits / 8;  // places one histogram launch counts
  for (int g = 0; g < places; g += group) {
    const int lo = begin_bit + g * rc.digit_bits;
    const int hi = std::min(end_bit, lo + group * rc.digit_bits);
    ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_HISTOGRAM, "histogram",
                    launch_histogram(key_bits, d_keys, d_hist + static_cast<size_t>(g) * kRadix,
                                     nullptr, static_cast<uint32_t>(n), lo, hi,
                                     std::min(group, places - g), rc.digit_bits, rc.order,
                                     static_cast<uint32_t>(cus * rc.hist_blocks_per_cu), s));
  }
  return ONESWEEP_SUCCESS;
}

onesweep_status_t onesweep_binning_pass(void *d_temp, size_t *temp_bytes,
                                        const void *d_src_keys, void *d_dst_keys,
                                        const uint32_t *d_src_vals, uint32_t *d_dst_vals,
                                        size_t n, int key_bits, int shift, int width,
                                        const uint32_t *d_bin_offsets,
                                        const onesweep_config_t *cfg,
                                        onesweep_stream_t stream) {
  g_error[0] = '\0';
  if (temp_bytes == nullptr) return fail(ONESWEEP_ERROR_INVALID_VALUE, "temp_bytes is NULL");
  if (key_bits != 32 && key_bits != 64)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key_bits %d is not 32 or 64", key_bits);
  if (width < 1 || width > kRadixBits || shift < 0 || shift + width > key_bits)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "digit bits [%d, %d) invalid", shift,
                shift + width);
  if (n >= kMaxN) return fail(ONESWEEP_ERROR_TOO_LARGE, "n = %zu is not below 2^30", n);
  if (n * static_cast<size_t>(key_bits / 8) > kBufferBytes)
    return fail(ONESWEEP_ERROR_TOO_LARGE, "n = %zu %d-bit keys pass 4 GiB", n, key_bits);
  const bool has_values = d_src_vals != nullptr || d_dst_vals != nullptr;
  Resolved rc;
  onesweep_status_t st;
  if ((st = resolve(key_bits, has_values, n, cfg, &rc))) return st;
  const size_t tile = binning_tile_items(rc.shape);
  const uint32_t tiles = static_cast<uint32_t>((n + tile - 1) / tile);
  const size_t need = kAlign + align_up(sizeof(uint32_t) * kRadix * static_cast<size_t>(tiles));
  if (d_temp == nullptr) {
    *temp_bytes = need;
    return ONESWEEP_SUCCESS;
  }
  if (rc.trace) rc.trace->count = 0;
  if (n == 0) return ONESWEEP_SUCCESS;
  if (*temp_bytes < need)
    return fail(ONESWEEP_ERROR_INSUFFICIENT_TEMP, "temp storage %zu bytes, need %zu",
                *temp_bytes, need);
  const size_t kb = static_cast<size_t>(key_bits / 8);
  if (!d_src_keys || !d_dst_keys || !d_bin_offsets)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "NULL pointer");
  if (has_values && (!d_src_vals || !d_dst_vals))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "only one value pointer given");
  if ((reinterpret_cast<uintptr_t>(d_temp) & (kAlign - 1)) != 0)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "d_temp is not 256-byte aligned");
  if ((reinterpret_cast<uintptr_t>(d_src_keys) | reinterpret_cast<uintptr_t>(d_dst_keys)) &
      (kb - 1))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "key pointers not aligned");
  if (ranges_overlap(d_src_keys, n * kb, d_dst_keys, n * kb) ||
      (has_values && ranges_overlap(d_src_vals, n * 4, d_dst_vals, n * 4)))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "source and destination overlap");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int cus = 0;
  if ((st = device_cus(&cus))) return st;
  Tracer tr(rc.trace, s);
  char *temp = static_cast<char *>(d_temp);
  ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_RESET, "clear",
                  launch_fill_zero(temp, need, static_cast<uint32_t>(cus) * 4u, s));
  uint32_t *counter = reinterpret_cast<uint32_t *>(temp);
  uint32_t *status = reinterpret_cast<uint32_t *>(temp + kAlign);
  if (key_bits == 32) {
    BinningArgs<uint32_t> a{};
    a.keys[kBufIn] = static_cast<uint32_t *>(const_cast<void *>(d_src_keys));
    a.keys[kBufOut] = static_cast<uint32_t *>(d_dst_keys);
    a.vals[kBufIn] = const_cast<uint32_t *>(d_src_vals);
    a.vals[kBufOut] = d_dst_vals;
    a.bin_offsets = d_bin_offsets;
    a.status = status;
    a.tile_counter = counter;
    a.plan = nullptr;
    a.order = rc.order;
    a.lookback_error = counter + 1;
    a.spin_limit = rc.spin_limit;
    a.n = static_cast<uint32_t>(n);
    a.place = 0;
    a.shift = shift;
    a.width = width;
    ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_BINNING, "binning",
                    launch_binning(rc.shape, kBinChained, &a, tiles, s));
  } else {
    BinningArgs<uint64_t> a{};
    a.keys[kBufIn] = static_cast<uint64_t *>(const_cast<void *>(d_src_keys));
    a.keys[kBufOut] = static_cast<uint64_t *>(d_dst_keys);
    a.vals[kBufIn] = const_cast<uint32_t *>(d_src_vals);
    a.vals[kBufOut] = d_dst_vals;
    a.bin_offsets = d_bin_offsets;
    a.status = status;
    a.tile_counter = counter;
    a.plan = nullptr;
    a.order = rc.order;
    a.lookback_error = counter + 1;
    a.spin_limit = rc.spin_limit;
    a.n = static_cast<uint32_t>(n);
    a.place = 0;
    a.shift = shift;
    a.width = width;
    ONESWEEP_LAUNCH(tr, ONESWEEP_KERNEL_BINNING, "binning",
                    launch_binning(rc.shape, kBinChained, &a, tiles, s));
  }
  return ONESWEEP_SUCCESS;
}

onesweep_status_t onesweep_sort_segments(void *d_temp, size_t *temp_bytes,
                                         const void *d_keys_in, void *d_keys_out,
                                         const uint32_t *d_vals_in, uint32_t *d_vals_out,
                                         size_t n, const uint32_t *d_seg_offsets,
                                         size_t num_segments, int key_bits, int begin_bit,
                                         int end_bit, int stable, const onesweep_config_t *cfg,
                                         onesweep_stream_t stream) {
  (void)stable;
  const bool has_values = d_vals_in != nullptr || d_vals_out != nullptr;
  return segments_impl(d_temp, temp_bytes, d_keys_in, d_keys_out, d_vals_in, d_vals_out,
                       has_values, n, d_seg_offsets, num_segments, key_bits, begin_bit, end_bit,
                       cfg, reinterpret_cast<hipStream_t>(stream));
}

onesweep_status_t onesweep_tune_segments(void *d_temp, size_t *temp_bytes,
                                         const void *d_keys_in, void *d_keys_out,
                                         const uint32_t *d_vals_in, uint32_t *d_vals_out,
                                         size_t n, const uint32_t *d_seg_offsets,
                                         size_t num_segments, int key_bits, int begin_bit,
                                         int end_bit, int repetitions,
                                         onesweep_config_t *cfg_out, onesweep_stream_t stream) {
  // Candidates: every tile shape built for the segmented path, crossed with
  // class limits that move segments between the LDS classes and the tile
  // path.
  static const int kShapes32[][2] = {{256, 8},  {256, 16},  {512, 16}, {1024, 8},
                                     {1024, 11}, {1024, 16}, {1024, 19}};
  static const int kShapes64[][2] = {{256, 8},  {256, 16}, {512, 8},
                                     {1024, 8}, {1024, 9}, {1024, 14}};
  static const int kLimits[][3] = {{0, 0, 0},   {0, 0, 4096},  {0, 0, 2048}, {0, 0, -1},
                                   {0, -1, 0},  {-1, 0, 0},    {256, 1024, 4096}};
  // Digit widths: 8 bits, and 7 (one more place for 32-bit keys, fewer
  // buckets per pass); wider places than 8 bits are not built.
  static const int kDigits[] = {8, 7};
  constexpr int kNumLimits = sizeof(kLimits) / sizeof(kLimits[0]);
  constexpr int kNumDigits = sizeof(kDigits) / sizeof(kDigits[0]);
  const int num_shapes = key_bits == 64 ? static_cast<int>(sizeof(kShapes64) / sizeof(kShapes64[0]))
                                        : static_cast<int>(sizeof(kShapes32) / sizeof(kShapes32[0]));
  // The key order comes in through *cfg_out and is kept by every candidate.
  const int key_type = cfg_out ? cfg_out->key_type : ONESWEEP_KEY_UNSIGNED;
  const int descending = cfg_out ? cfg_out->descending : 0;
  auto candidate = [&](int i) {
    onesweep_config_t c{};
    c.key_type = key_type;
    c.descending = descending;
    const int(*shapes)[2] = key_bits == 64 ? kShapes64 : kShapes32;
    const int shape = i / (kNumLimits * kNumDigits);
    c.block_threads = shapes[shape][0];
    c.items_per_thread = shapes[shape][1];
    for (int k = 0; k < 3; ++k) c.segment_limits[k] = kLimits[(i / kNumDigits) % kNumLimits][k];
    c.digit_bits = kDigits[i % kNumDigits];
    return c;
  };
  // a digit width whose places would exceed a sort's is not a candidate
  auto applies = [&](int i) {
    return num_places(begin_bit, end_bit, kDigits[i % kNumDigits]) <= kMaxPlaces;
  };
  const int count = num_shapes * kNumLimits * kNumDigits;
  g_error[0] = '\0';
  if (temp_bytes == nullptr) return fail(ONESWEEP_ERROR_INVALID_VALUE, "temp_bytes is NULL");
  if (d_temp != nullptr && cfg_out == nullptr)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "cfg_out is NULL");
  if (d_temp != nullptr && ((d_keys_in != nullptr && d_keys_in == d_keys_out) ||
                            (d_vals_in != nullptr && d_vals_in == d_vals_out)))
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "the tuner needs separate input and output");
  if (repetitions < 1 || repetitions > 100)
    return fail(ONESWEEP_ERROR_INVALID_VALUE, "repetitions %d not in [1, 100]", repetitions);
  size_t need = 0;
  for (int i = 0; i < count; ++i) {
    if (!applies(i)) continue;
    onesweep_config_t c = candidate(i);
    size_t sz = 0;
    onesweep_status_t st = onesweep_sort_segments(nullptr, &sz, d_keys_in, d_keys_out, d_vals_in,
                                                  d_vals_out, n, d_seg_offsets, num_segments,
                                                  key_bits, begin_bit, end_bit, 1, &c, stream);
    if (st) return st;
    need = std::max(need, sz);
  }
  if (d_temp == nullptr) {
    *temp_bytes = need;
    return ONESWEEP_SUCCESS;
  }
  if (*temp_bytes < need)
    return fail(ONESWEEP_ERROR_INSUFFICIENT_TEMP, "temp storage %zu bytes, need %zu",
                *temp_bytes, need);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    return hip_fail(e, "hipEventCreate");
  }
  onesweep_status_t st = ONESWEEP_SUCCESS;
  float best_ms = 0.0f;
  int best = -1;
  for (int i = 0; i < count && st == ONESWEEP_SUCCESS; ++i) {
    if (!applies(i)) continue;
    onesweep_config_t c = candidate(i);
    size_t sz = *temp_bytes;
    auto run = [&]() {
      return onesweep_sort_segments(d_temp, &sz, d_keys_in, d_keys_out, d_vals_in, d_vals_out, n,
                                    d_seg_offsets, num_segments, key_bits, begin_bit, end_bit, 1,
                                    &c, stream);
    };
    if ((st = run())) break;  // warm-up
    if ((e = hipEventRecord(ev[0], s)) != hipSuccess) { st = hip_fail(e, "hipEventRecord"); break; }
    for (int r = 0; r < repetitions && st == ONESWEEP_SUCCESS; ++r) st = run();
    if (st) break;
    if ((e = hipEventRecord(ev[1], s)) != hipSuccess ||
        (e = hipEventSynchronize(ev[1])) != hipSuccess) {
      st = hip_fail(e, "timing event");
      break;
    }
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) {
      st = hip_fail(e, "hipEventElapsedTime");
      break;
    }
    if (best < 0 || ms < best_ms) {
      best = i;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (st) return st;
  *cfg_out = candidate(best);
  // Leave the output sorted by the chosen configuration.
  size_t sz = *temp_bytes;
  return onesweep_sort_segments(d_temp, &sz, d_keys_in, d_keys_out, d_vals_in, d_vals_out, n,
                                d_seg_offsets, num_segments, key_bits, begin_bit, end_bit, 1,
                                cfg_out, stream);
}

size_t onesweep_tile_items(int key_bits, int has_values, size_t n, const onesweep_config_t *cfg) {
  if (key_bits != 32 && key_bits != 64) return 0;
  Resolved rc;
  if (resolve(key_bits, has_values != 0, n, cfg, &rc, kCallSort) != ONESWEEP_SUCCESS) return 0;
  return binning_tile_items(rc.shape);
}

const char *onesweep_last_error(void) { return g_error; }

const char *onesweep_version(void) { return "onesweep-gfx950 0.1"; }

}  // extern "C"
