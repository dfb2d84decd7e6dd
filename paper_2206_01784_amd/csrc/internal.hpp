// Host-side interface between the C ABI (api.hip) and the kernel translation
// units. Each launcher enqueues exactly one kernel on `stream` and returns the
// launch status; none of them allocates or synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_common.hpp"

namespace onesweep {

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

bool binning_shape_supported(const BinningShape &s);
BinningShape binning_default_shape(int key_bits, bool has_values);

// `args` points to BinningArgs<uint32_t> or BinningArgs<uint64_t>.
hipError_t launch_binning(const BinningShape &s, const void *args, uint32_t grid,
                          hipStream_t stream);

// Histogram of all places (phase 1), persistent tile-cyclic grid.
constexpr int kHistBlock = 256;
hipError_t launch_histogram(int key_bits, const void *keys, uint32_t *hist, uint32_t n,
                            int begin_bit, int end_bit, int places, uint32_t grid,
                            hipStream_t stream);

// Exclusive sums of every place's histogram and the pass plan (phase 2).
hipError_t launch_scan(const uint32_t *hist, uint32_t *offsets, PassPlan *plan, int places,
                       uint32_t n, bool alias, hipStream_t stream);

// Copy of keys (and values) into the output. With a plan, the source buffer
// is the plan's copy_src and nothing is copied when it is kNoBuffer; without
// a plan the source is buffer kBufIn.
struct CopyArgs {
  void *keys[3];
  uint32_t *vals[3];
  const PassPlan *plan;
  uint32_t n;
  int key_bytes;
};
hipError_t launch_copy(const CopyArgs &a, uint32_t grid, hipStream_t stream);

// Zero `bytes` (a multiple of 4) bytes at `p` with a kernel, so that the
// enqueued sequence stays free of memset nodes.
hipError_t launch_fill_zero(void *p, size_t bytes, uint32_t grid, hipStream_t stream);

}  // namespace onesweep
