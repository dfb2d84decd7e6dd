// Shared device-side definitions of the Onesweep kernels for gfx950 (CDNA4,
// wave64). Included by every kernel translation unit; host-only code uses
// internal.hpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace onesweep {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;  // r = 256 bins per digit place
constexpr int kMaxPlaces = 8;            // digit places of one sort (64-bit keys, 8-bit digits)
constexpr int kWave = 64;

// Chained-scan status word (Section 3, Figure 6): 2-bit status above a
// 30-bit value. N = not ready, L = tile-local count, G = inclusive prefix.
constexpr uint32_t kValueMask = (1u << 30) - 1u;
constexpr uint32_t kFlagMask = 3u << 30;
constexpr uint32_t kFlagL = 1u << 30;
constexpr uint32_t kFlagG = 2u << 30;

// Buffer ids used by the pass plan.
enum : uint32_t { kBufIn = 0, kBufOut = 1, kBufTmp = 2, kNoBuffer = 3 };

// Order of the key bits. Signed and floating-point keys are ranked through a
// magnitude-preserving transform onto unsigned order (Section 3, binning
// kernel): the sign bit flips, and negative floating-point keys flip every
// bit; descending order complements the result. The transform only decides
// digits: keys are read and written unchanged. 32-bit keys use the low halves
// of the fields.
struct KeyOrder {
  uint64_t sign;      // the top key bit for signed and floating-point keys, else 0
  uint64_t negative;  // all ones for floating-point keys, else 0
  uint64_t invert;    // all ones for descending order, else 0
  uint64_t pad;       // the key whose transformed bits are all ones (padding lanes)
};

// The pass plan is computed on the device by the scan kernel from the exact
// histograms, so the host never synchronises to learn which passes run:
// a place whose histogram puts all n keys in one bin is an identity
// permutation and is skipped; executed passes alternate buffers so that the
// last one lands in the output.
struct PassPlan {
  uint32_t run[kMaxPlaces];
  uint32_t src[kMaxPlaces];
  uint32_t dst[kMaxPlaces];
  uint32_t copy_src;  // buffer copied into the output at the end, or kNoBuffer
  uint32_t executed;
  uint32_t lookback_error;  // bit 0: a look-back gave up; bit 1: a run fell outside
  uint32_t pad[13];
};
static_assert(sizeof(PassPlan) <= 256, "plan fits one 256-byte slot");

// Segmented sort (independent stable sorts of the ranges
// [offsets[s], offsets[s + 1])). The classify kernel sorts the segments into
// classes by length: three classes sorted whole inside one workgroup's LDS
// and a "large" class whose segments are cut into binning tiles. Each large
// segment is an Onesweep sort of its own, with its own histograms, bin offsets
// and chained scan; the tiles of all large segments are enumerated together so
// one binning launch per digit place covers them all.
constexpr int kSegClasses = 3;  // LDS-sorted classes; class kSegClasses is "large"

struct SegmentPlan {
  uint32_t error;                      // 1: offsets invalid, nothing is sorted
  uint32_t count[kSegClasses + 1];     // segments per class (last: large)
  uint32_t large_tiles;                // binning tiles of all large segments
  uint32_t lookback_error;             // bit 0: a wait gave up; bit 1: a run fell outside
  uint32_t pad[57];
};
static_assert(sizeof(SegmentPlan) == 256, "one 256-byte slot");

// One binning tile of a large segment: x = first key, y = keys in the tile,
// z = first key of the segment, w = index of the segment among large ones.
// A tile with x == z starts its segment's chained scan.
struct SegmentTiles {
  const uint4 *tile_info;       // [tiles]
  uint32_t *counts;             // [large][places][256] digit counts within the segment
  const uint32_t *large_len;    // [large] keys per large segment
  const SegmentPlan *plan;
  int places;
  int begin_bit, end_bit;       // bit range of all places (the counting workgroups)
  int digit_bits;               // width of a digit place (4..8)
};

// Idx is the type of element positions: uint32_t below 2^31 elements,
// uint64_t for larger sorts (Section 3, handling very large problems: 64-bit
// global counts and carried bin starts; status words stay 30-bit because each
// strip is its own chained scan of fewer than 2^30 keys).
template <typename K, typename Idx = uint32_t>
struct BinningArgs {
  K *keys[3];                  // in, out, tmp (in is only read)
  uint32_t *vals[3];           // same ids; unused for keys-only
  const Idx *bin_offsets;      // 256 global bin offsets of this place
  uint32_t *status;            // [tiles][256] status words of this place
  uint32_t *tile_counter;      // dynamic tile ids of this place
  const PassPlan *plan;        // NULL: run unconditionally in -> out
  SegmentTiles seg;            // segmented sort only
  KeyOrder order;
  // Strips of a large sort (Section 3, handling very large problems): this
  // launch bins the tiles [tile_first, tile_first + grid) as one chained
  // scan, and its last tile writes bin_offsets + the strip's digit counts to
  // next_bin_offsets, the bin starts of the next strip (NULL: last strip).
  uint32_t tile_first;
  Idx *next_bin_offsets;
  // Bounded look-back wait: a tile that has polled its window of
  // predecessors spin_limit times without reaching an inclusive prefix gives
  // up, sets bit 0 of *lookback_error and carries on with what it has summed (its
  // output is then wrong, but every workgroup exits). Legitimate look-backs
  // take a few polls; the default limit is seconds of waiting.
  uint32_t *lookback_error;
  uint32_t spin_limit;
  Idx n;
  int place;
  int shift;
  int width;
};

template <typename K>
struct HistogramArgs {
  const K *keys;
  uint32_t *hist;              // [places][256], cleared before launch
  unsigned long long *hist64;  // if not NULL: 64-bit counts, added here instead
  uint32_t n;
  int begin_bit;
  int end_bit;
  int places;      // at most one per byte of the key in one launch
  int digit_bits;  // width of a digit place (4..8)
  KeyOrder order;
};

// Agent-scope atomics: successive tiles usually run on different XCDs, whose
// L2 caches are not coherent with each other, so status words and tile
// counters go through device-coherent accesses. A status word carries its own
// value, so relaxed ordering is enough for the look-back protocol.
__device__ __forceinline__ void store_status(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_status(const uint32_t *p) {
  return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t count_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Unsigned ascending order: the transform is the identity, and kernels are
// instantiated without it (kOrdered = false) so that default sorts pay
// nothing for it.
__host__ __device__ inline bool key_order_is_plain(const KeyOrder &o) {
  return (o.sign | o.negative | o.invert) == 0u;
}

template <typename K>
__device__ __forceinline__ K ordered_bits(K key, const KeyOrder &o) {
  using S = typename std::make_signed<K>::type;
  const K neg = static_cast<K>(static_cast<S>(key) >> (8 * sizeof(K) - 1));
  return key ^ ((neg & static_cast<K>(o.negative)) | static_cast<K>(o.sign)) ^
         static_cast<K>(o.invert);
}

// Inverse of ordered_bits: u is the transformed key with the direction
// undone; a floating-point key was negative exactly when u's top bit is 0.
template <typename K>
__device__ __forceinline__ K original_bits(K t, const KeyOrder &o) {
  using S = typename std::make_signed<K>::type;
  const K u = t ^ static_cast<K>(o.invert);
  const K was_negative = ~static_cast<K>(static_cast<S>(u) >> (8 * sizeof(K) - 1));
  return u ^ ((was_negative & static_cast<K>(o.negative)) | static_cast<K>(o.sign));
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask) {
  return static_cast<uint32_t>(key >> shift) & mask;
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask, const KeyOrder &o) {
  return digit_of(ordered_bits(key, o), shift, mask);
}

// Inclusive sum over the lanes of a wavefront.
#ifndef ONESWEEP_DPP_SCAN
#define ONESWEEP_DPP_SCAN 1
#endif
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
#if ONESWEEP_DPP_SCAN
  // Data-parallel primitives: within each row of 16 lanes add the values
  // 1, 2, 4 and 8 lanes back (lanes whose source lies outside the row add
  // 0), then broadcast the last lane of rows 0 and 2 into rows 1 and 3 and
  // the last lane of row 1 into rows 2 and 3. No LDS traffic.
  constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
  v += __builtin_amdgcn_update_dpp(0u, v, kRowShr | 1, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0u, v, kRowShr | 2, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0u, v, kRowShr | 4, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0u, v, kRowShr | 8, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0u, v, kRowBcast15, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0u, v, kRowBcast31, 0xc, 0xf, false);
  return v;
#else
  const int lane = static_cast<int>(threadIdx.x) & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t t = __shfl_up(v, off, kWave);
    if (lane >= off) v += t;
  }
  return v;
#endif
}

// In-place exclusive scan of a table of per-wave digit counts,
// table[w * 256 + d], taken in digit-major order: afterwards entry (w, d)
// holds the number of keys with a smaller digit plus the keys of digit d in
// waves before w, i.e. the position in the workgroup's digit-sorted order of
// wave w's first key with digit d. Every thread of the workgroup owns four
// consecutive entries of that order, so the scan costs one LDS read and one
// write per entry and a workgroup-wide sum of per-thread totals. The caller
// synchronises before (table complete) and after (table rewritten);
// s_wave_sum holds kBlock / 64 words.
template <int kBlock>
__device__ __forceinline__ void digit_major_exclusive_scan(uint32_t *table,
                                                           uint32_t *s_wave_sum) {
  constexpr int kWaves = kBlock / kWave;
  static_assert(kWaves * kRadix == 4 * kBlock, "four entries per thread");
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  uint32_t c[4], ex[4], sum = 0u;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int f = 4 * tid + k;
    c[k] = table[(f % kWaves) * kRadix + f / kWaves];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ex[k] = sum;
    sum += c[k];
  }
  const uint32_t incl = wave_inclusive_sum(sum);
  uint32_t base = incl - sum;
  if constexpr (kWaves > 1) {
    if (lane == kWave - 1) s_wave_sum[wave] = incl;
    __syncthreads();
    for (int w = 0; w < wave; ++w) base += s_wave_sum[w];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int f = 4 * tid + k;
    table[(f % kWaves) * kRadix + f / kWaves] = base + ex[k];
  }
}

}  // namespace onesweep
