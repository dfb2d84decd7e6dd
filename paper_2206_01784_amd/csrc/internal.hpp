// Host-side interface between the C ABI (api.hip) and the kernel translation
// units. Each launcher enqueues exactly one kernel on `stream` and returns the
// launch status; none of them allocates or synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/onesweep.h"
#include "device_common.hpp"

namespace onesweep {

// Thread-local error message of the C ABI (api.hip).
onesweep_status_t fail(onesweep_status_t code, const char *fmt, ...);
onesweep_status_t hip_fail(hipError_t e, const char *what);
void clear_error();

// One binning-kernel instantiation: key width, values or not, workgroup size,
// items per thread (tile = block * ipt keys) and the wave-level match used
// for ranking (0: one ballot per digit bit, 1: LDS presence masks).
struct BinningShape {
  int key_bits;
  bool has_values;
  int block;
  int ipt;
  int rank;
};

// A binning configuration chosen on the host after the clear, histogram and
// exclusive-sum kernels of a whole sort are enqueued (the learned selector
// decides while they run): `choose` fills the tile fields (block_threads,
// items_per_thread, rank_algorithm) of *cfg, which holds the caller's
// configuration on entry; `layout_tile` is the smallest tile any choice can
// make, which sizes the temporary storage. Onesweep only, n <= 2^28.
struct LateChoice {
  size_t layout_tile;
  onesweep_status_t (*choose)(void *ctx, onesweep_config_t *cfg);
  void *ctx;
};
onesweep_status_t sort_late_choice(void *d_temp, size_t *temp_bytes, const void *keys_in,
                                   void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                                   bool has_values, size_t n, int key_bits, int begin_bit,
                                   int end_bit, const onesweep_config_t *cfg, hipStream_t stream,
                                   const LateChoice &late);

// Binning kernel modes: Onesweep's chained scan over the tiles of one
// sequence; the same per large segment of a segmented sort
// (BinningArgs::seg); or the scatter (downsweep) step of the reduce-then-scan
// baseline. Fewer shapes are built for the last two.
enum BinningMode : int { kBinChained = 0, kBinSegmented = 1, kBinDownsweep = 2, kBinSegCounted = 3 };

// `wide`: 64-bit element positions (sorts of 2^31 elements or more), built
// for the default large-input shapes of the chained mode only.
bool binning_shape_supported(const BinningShape &s, int mode, bool wide = false);
BinningShape binning_default_shape(int key_bits, bool has_values, size_t n);
BinningShape segment_default_shape(int key_bits, bool has_values);
// Keys per binning tile of a shape.
size_t binning_tile_items(const BinningShape &s);

// `args` points to BinningArgs<K, Idx> with K the key type of the shape and
// Idx uint64_t when `wide`, else uint32_t.
hipError_t launch_binning(const BinningShape &s, int mode, const void *args,
                          uint32_t grid, hipStream_t stream, bool wide = false);

// Reduce-then-scan baseline, per place: the upsweep counts every tile's
// digits into a digit-major table [256][tiles]; the tile scan turns each
// digit's row into exclusive prefixes over tiles in place. Both follow the
// pass plan (a skipped place does nothing). The tile shape is the
// downsweep's.
template <typename K>
struct UpsweepArgs {
  K *keys[3];
  const PassPlan *plan;
  uint32_t *counts;  // [256][tiles]
  uint32_t n;
  int place;
  int shift;
  int width;
  KeyOrder order;
};
bool upsweep_shape_supported(int key_bits, int block, int ipt);
hipError_t launch_upsweep(int key_bits, int block, int ipt, const void *args, uint32_t tiles,
                          hipStream_t stream);
hipError_t launch_tile_scan(uint32_t *counts, uint32_t tiles, const PassPlan *plan, int place,
                            hipStream_t stream);

// Histogram of the places of [begin_bit, end_bit) (phase 1), digit_bits
// wide, at most key_bits / 8 places per launch, persistent tile-cyclic grid,
// over n < 2^31 keys; the counts are added to hist, or to the 64-bit hist64
// when it is not NULL (larger sorts histogram portions of the keys into it).
hipError_t launch_histogram(int key_bits, const void *keys, uint32_t *hist,
                            unsigned long long *hist64, uint32_t n, int begin_bit, int end_bit,
                            int places, int digit_bits, const KeyOrder &order, uint32_t grid,
                            hipStream_t stream);

// Exclusive sums of every place's histogram and the pass plan (phase 2):
// 32-bit counts and offsets (hist, offsets), or 64-bit ones (hist64,
// offsets64) when those are not NULL.
hipError_t launch_scan(const uint32_t *hist, const unsigned long long *hist64, uint32_t *offsets,
                       unsigned long long *offsets64, PassPlan *plan, int places, uint64_t n,
                       bool alias, hipStream_t stream);

// Copy of keys (and values) into the output. With a plan, the source buffer
// is the plan's copy_src and nothing is copied when it is kNoBuffer; without
// a plan the source is buffer kBufIn.
struct CopyArgs {
  void *keys[3];
  uint32_t *vals[3];
  const PassPlan *plan;
  uint64_t n;
  int key_bytes;
};
hipError_t launch_copy(const CopyArgs &a, uint32_t grid, hipStream_t stream);

// Zero `bytes` (a multiple of 4) bytes at `p` with a kernel, so that the
// enqueued sequence stays free of memset nodes.
hipError_t launch_fill_zero(void *p, size_t bytes, uint32_t grid, hipStream_t stream);

// ---------------------------------------------------------------- segmented sort
// Class c (< kSegClasses) takes the non-empty segments with
// limit[c - 1] < length <= limit[c] (limit[-1] = 0); longer ones are large.
struct ClassifyArgs {
  const uint32_t *offsets;
  uint32_t num_segments;
  uint32_t n;
  uint32_t limit[kSegClasses];
  uint32_t capacity[kSegClasses];  // entries of lists[c]
  uint32_t *lists[kSegClasses];    // segment ids per LDS class
  uint32_t max_large;
  uint32_t max_tiles;
  uint32_t tile_items;             // binning tile of the large segments
  uint4 *tile_info;                // [max_tiles]
  uint32_t *large_len;             // [max_large] keys per large segment
  uint32_t *tile_counters;         // kMaxPlaces words, cleared
  SegmentPlan *plan;
};
hipError_t launch_classify(const ClassifyArgs &a, hipStream_t stream);

struct SegmentClearArgs {
  uint32_t *status;
  size_t status_words_per_place;
  uint32_t *hist;
  const SegmentPlan *plan;
  int places;
};
hipError_t launch_segment_clear(const SegmentClearArgs &a, uint32_t grid, hipStream_t stream);

struct SegmentCopyArgs {
  const void *keys_src;
  void *keys_dst;
  const uint32_t *vals_src;
  uint32_t *vals_dst;
  const uint4 *tile_info;
  const SegmentPlan *plan;
  int key_bytes;
};
hipError_t launch_segment_copy(const SegmentCopyArgs &a, uint32_t grid, hipStream_t stream);

struct LdsSortArgs {
  const void *keys_in;
  void *keys_out;
  const uint32_t *vals_in;
  uint32_t *vals_out;
  const uint32_t *offsets;
  const uint32_t *list;  // segment ids of this class
  const SegmentPlan *plan;
  int cls;
  int begin_bit;
  int end_bit;
  int places;
  int digit_bits;
  KeyOrder order;
};
int lds_class_capacity(int cls);
int lds_class_block(int key_bits, bool has_values, int cls);
hipError_t lds_sort_blocks_per_cu(int key_bits, bool has_values, int cls, int *blocks);
hipError_t launch_lds_sort(int key_bits, bool has_values, const LdsSortArgs &a, uint32_t grid,
                           hipStream_t stream);

// ---------------------------------------------------------------- learned configuration
constexpr int kMlpPlaces = 8, kMlpEnc = 16, kMlpScalars = 3, kMlpH1 = 64, kMlpH2 = 64;
constexpr int kMlpClasses = 12;
constexpr int kMlpU = kMlpPlaces * kMlpEnc + kMlpScalars;           // 131
constexpr int kMlpFeatures = kMlpPlaces * kRadix + kMlpScalars;     // 2051
constexpr uint32_t kMlpSamples = 4096;
constexpr int kOffWe = 0;
constexpr int kOffBe = kOffWe + kRadix * kMlpEnc;
constexpr int kOffW1 = kOffBe + kMlpEnc;
constexpr int kOffB1 = kOffW1 + kMlpU * kMlpH1;
constexpr int kOffW2 = kOffB1 + kMlpH1;
constexpr int kOffB2 = kOffW2 + kMlpH1 * kMlpH2;
constexpr int kOffW3 = kOffB2 + kMlpH2;
constexpr int kOffB3 = kOffW3 + kMlpH2 * kMlpClasses;
constexpr int kMlpParams = kOffB3 + kMlpClasses;                    // 17500

struct FeatureArgs {
  const void *keys;
  uint64_t n;
  int begin_bit;
  int end_bit;
  int places;
  int has_values;
  float *out;  // kMlpFeatures
};
hipError_t launch_features(int key_bits, const FeatureArgs &a, hipStream_t stream);

struct InferArgs {
  const float *params;
  const float *x;        // kMlpFeatures
  uint32_t class_mask;   // classes that may be chosen
  float *out;            // kMlpClasses
  int *choice;
};
hipError_t launch_infer(const InferArgs &a, hipStream_t stream);

struct SelectArgs {
  const float *params;
  const void *keys;
  uint64_t n;
  int begin_bit;
  int end_bit;
  int places;
  int has_values;
  uint32_t class_mask;
  // The autotuned default's class (-1: none applies): it stays the choice
  // unless another class is predicted faster by more than `margin` (in the
  // predictions' log-time units).
  int default_class;
  float margin;
  float *out;         // kMlpClasses
  int *choice;        // device
  int *host_choice;   // mapped pinned host memory, may be NULL
};
hipError_t launch_select(int key_bits, const SelectArgs &a, hipStream_t stream);

struct GemmArgs {
  const float *A;
  const float *B;
  float *C;
  const float *bias;  // may be NULL
  const float *mask;  // may be NULL: zero C where mask <= 0 (same layout as C)
  int M, N, K;
  long a_rs, a_cs, b_rs, b_cs, c_rs;
  int relu;
};
hipError_t launch_gemm(const GemmArgs &g, hipStream_t stream);
hipError_t launch_colsum(const float *dz, int rows, int cols, int rs, float *db,
                         hipStream_t stream);
hipError_t launch_assemble(const float *enc, const float *scalars, float *u, int batch,
                           hipStream_t stream);
hipError_t launch_split(const float *d_u, const float *enc, float *d_enc, int batch,
                        hipStream_t stream);
hipError_t launch_loss(const float *out, const float *y, const float *mask, int count,
                       float *d_out, float *loss, hipStream_t stream);

struct AdamArgs {
  float *theta, *m, *v;
  const float *grad;
  int count;
  float lr, beta1, beta2, eps, c1, c2;
};
hipError_t launch_adam(const AdamArgs &a, hipStream_t stream);

}  // namespace onesweep
