// Reduce-then-scan radix sorting, the prior scheme that Onesweep improves on
// (Section 2, reduce-then-scan digit binning; Figures 1, 3 and 4): every
// digit place takes three steps,
//   1. upsweep: each tile counts its keys' digits (reads n keys);
//   2. tile scan: per digit, an exclusive scan of the counts over tiles;
//   3. downsweep: each tile re-reads its keys, ranks them and scatters them
//      to bin offset + its exclusive prefix (reads n keys, writes n keys).
// That is 3n key movements per place against Onesweep's 2n (plus one upfront
// read of n shared by all places). The downsweep is the binning kernel in
// its kBinDownsweep mode, so both schemes rank and scatter with the same
// code and differ only in how a tile learns its prefix. The global bin
// offsets and the pass plan (exact skip of one-digit places, buffer routing)
// come from the same upfront histogram as Onesweep's. Figure 4's one prefix
// sum over the digit-major concatenation of tile counts equals that bin
// offset plus the digit's own prefix over tiles, so the scan runs as 256
// independent rows.
#include "device_common.hpp"
#include "internal.hpp"

namespace onesweep {

// One workgroup per tile (the downsweep's tile shape and order): LDS
// counters, one LDS atomic per key, then each digit's total is written to row
// `digit` of the digit-major count table. kCopies interleaved copies of each
// counter (copy = lane % kCopies, copy index fastest) keep lanes that share a
// digit on different banks, bounding same-address serialisation of skewed
// inputs to 64 / kCopies-way within one atomic instruction.
template <typename K, int kBlock, int kIpt, bool kOrdered>
__global__ void __launch_bounds__(kBlock) upsweep_kernel(UpsweepArgs<K> a) {
  constexpr int kCopies = 8;
  constexpr int kTile = kBlock * kIpt;
  constexpr int kWaveItems = kWave * kIpt;
  __shared__ uint32_t s_count[kRadix * kCopies];
  if (a.plan->run[a.place] == 0u) return;  // skipped place: no table is read
  const K *__restrict__ src = a.keys[a.plan->src[a.place]];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  for (int i = tid; i < kRadix * kCopies; i += kBlock) s_count[i] = 0u;
  __syncthreads();

  const uint32_t tile = blockIdx.x;
  const uint32_t tiles = gridDim.x;
  const uint32_t n = a.n;
  const uint32_t base = tile * static_cast<uint32_t>(kTile);
  const uint32_t count = min(n - base, static_cast<uint32_t>(kTile));
  const uint32_t wb = base + static_cast<uint32_t>(wave * kWaveItems + lane);
  const int shift = a.shift;
  const uint32_t mask = (1u << a.width) - 1u;
  uint32_t *mine = s_count + (lane & (kCopies - 1));
  auto digit = [&](K k) -> uint32_t {
    if constexpr (kOrdered) return digit_of(k, shift, mask, a.order);
    else return digit_of(k, shift, mask);
  };
  K key[kIpt];
  if (count == static_cast<uint32_t>(kTile)) {
#pragma unroll
    for (int i = 0; i < kIpt; ++i) key[i] = src[wb + i * kWave];
#pragma unroll
    for (int i = 0; i < kIpt; ++i)
      __hip_atomic_fetch_add(&mine[digit(key[i]) * kCopies], 1u,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  } else {
    const uint32_t end = base + count;
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      const uint32_t idx = wb + i * kWave;
      if (idx < end)
        __hip_atomic_fetch_add(&mine[digit(src[idx]) * kCopies], 1u,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  __syncthreads();
  if (tid < kRadix) {
    uint32_t total = 0u;
#pragma unroll
    for (int c = 0; c < kCopies; ++c) total += s_count[tid * kCopies + c];
    a.counts[static_cast<size_t>(tid) * tiles + tile] = total;
  }
}

// One 1024-thread workgroup per digit row: chunks of 8 consecutive counts per
// thread, a workgroup exclusive scan of the per-thread sums, and a carry from
// chunk to chunk. The row is rewritten in place with exclusive prefixes.
constexpr int kTileScanBlock = 1024;
constexpr int kTileScanItems = 8;

__global__ void __launch_bounds__(kTileScanBlock)
    tile_scan_kernel(uint32_t *counts, uint32_t tiles, const PassPlan *plan, int place) {
  constexpr int kWaves = kTileScanBlock / kWave;
  constexpr uint32_t kChunk = kTileScanBlock * kTileScanItems;
  __shared__ uint32_t s_wave_sum[kWaves];
  if (plan->run[place] == 0u) return;
  uint32_t *row = counts + static_cast<size_t>(blockIdx.x) * tiles;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  uint32_t carry = 0u;
  for (uint32_t base = 0; base < tiles; base += kChunk) {
    const uint32_t i0 = base + static_cast<uint32_t>(tid) * kTileScanItems;
    uint32_t v[kTileScanItems];
    uint32_t sum = 0u;
#pragma unroll
    for (int j = 0; j < kTileScanItems; ++j) {
      v[j] = i0 + j < tiles ? row[i0 + j] : 0u;
      sum += v[j];
    }
    const uint32_t incl = wave_inclusive_sum(sum);
    if (lane == kWave - 1) s_wave_sum[wave] = incl;
    __syncthreads();
    uint32_t before = 0u, total = 0u;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t t = s_wave_sum[w];
      before += w < wave ? t : 0u;
      total += t;
    }
    uint32_t run = carry + before + incl - sum;
#pragma unroll
    for (int j = 0; j < kTileScanItems; ++j) {
      if (i0 + j < tiles) row[i0 + j] = run;
      run += v[j];
    }
    carry += total;
    __syncthreads();  // s_wave_sum is rewritten by the next chunk
  }
}

#define ONESWEEP_UPSWEEP_SHAPES(X) \
  X(uint32_t, 256, 8)              \
  X(uint32_t, 512, 16)             \
  X(uint32_t, 1024, 8)             \
  X(uint32_t, 1024, 11)            \
  X(uint32_t, 1024, 16)            \
  X(uint32_t, 1024, 18)            \
  X(uint32_t, 1024, 19)            \
  X(uint64_t, 1024, 9)             \
  X(uint64_t, 1024, 12)            \
  X(uint64_t, 1024, 14)            \
  X(uint64_t, 256, 8)              \
  X(uint64_t, 512, 8)              \
  X(uint64_t, 1024, 8)

bool upsweep_shape_supported(int key_bits, int block, int ipt) {
#define ONESWEEP_MATCH(K, B, I) \
  if (key_bits == 8 * (int)sizeof(K) && block == B && ipt == I) return true;
  ONESWEEP_UPSWEEP_SHAPES(ONESWEEP_MATCH)
#undef ONESWEEP_MATCH
  return false;
}

hipError_t launch_upsweep(int key_bits, int block, int ipt, const void *args, uint32_t tiles,
                          hipStream_t stream) {
#define ONESWEEP_LAUNCH(K, B, I)                                                             \
  if (key_bits == 8 * (int)sizeof(K) && block == B && ipt == I) {                            \
    const UpsweepArgs<K> &a = *static_cast<const UpsweepArgs<K> *>(args);                    \
    if (key_order_is_plain(a.order))                                                         \
      hipLaunchKernelGGL((upsweep_kernel<K, B, I, false>), dim3(tiles), dim3(B), 0, stream, a); \
    else                                                                                     \
      hipLaunchKernelGGL((upsweep_kernel<K, B, I, true>), dim3(tiles), dim3(B), 0, stream, a);  \
    return hipGetLastError();                                                                \
  }
  ONESWEEP_UPSWEEP_SHAPES(ONESWEEP_LAUNCH)
#undef ONESWEEP_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_tile_scan(uint32_t *counts, uint32_t tiles, const PassPlan *plan, int place,
                            hipStream_t stream) {
  hipLaunchKernelGGL(tile_scan_kernel, dim3(kRadix), dim3(kTileScanBlock), 0, stream, counts,
                     tiles, plan, place);
  return hipGetLastError();
}

}  // namespace onesweep
