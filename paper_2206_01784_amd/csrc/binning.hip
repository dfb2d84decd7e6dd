// Chained-scan digit-binning kernel: one Onesweep iteration over one digit
// place (Section 3, "Chained scan digit-binning kernel", Figures 7 and 8).
//
// One workgroup per tile of kBlock * kIpt keys, tiles handed out in order by
// an atomic counter so that a tile only ever waits on tiles that are already
// being processed. Per tile:
//   1. coalesced load; wave w owns a contiguous slice of the tile and its
//      batch i is 64 consecutive keys, so (wave, batch, lane) order equals
//      input order and ranks are stable;
//   2. wave64 multi-split ranking: 8 ballots give every lane the mask of
//      lanes holding its digit; the lowest such lane bumps the wave's LDS
//      counter for that digit and each lane's rank is the counter's previous
//      value plus the peers below it (the warp-level multi-split of
//      Ashkiani et al. that the paper uses, on 64-lane wavefronts);
//   3. per-digit exclusive sum over waves and over digits gives the tile's
//      digit counts and every key's position in the tile's local sort;
//   4. thread v publishes the tile's count of digit v, looks back over the
//      status words of earlier tiles until it meets an inclusive prefix, and
//      publishes its own inclusive prefix (decoupled look-back, r = 256
//      concurrent chained scans);
//   5. keys are regrouped by digit in LDS and written out as runs at
//      global bin offset + bin-relative tile offset + position in the run;
//      values follow with the same destinations.
#include "device_common.hpp"
#include "internal.hpp"

namespace onesweep {

template <typename K, bool kVals, int kBlock, int kIpt>
__global__ void __launch_bounds__(kBlock) binning_kernel(BinningArgs<K> a) {
  constexpr int kWaves = kBlock / kWave;
  constexpr int kTile = kBlock * kIpt;
  constexpr int kWaveItems = kWave * kIpt;
  static_assert(kBlock >= kRadix, "one thread per digit takes part in the look-back");
  static_assert(kBlock % kWave == 0, "whole wavefronts");

  uint32_t src_id = kBufIn, dst_id = kBufOut;
  if (a.plan != nullptr) {
    if (a.plan->run[a.place] == 0u) return;  // identity permutation: pass skipped
    src_id = a.plan->src[a.place];
    dst_id = a.plan->dst[a.place];
  }
  const K *__restrict__ src = a.keys[src_id];
  K *__restrict__ dst = a.keys[dst_id];

  constexpr size_t kKeyBytes = sizeof(K) * kTile;
  constexpr size_t kCountBytes = sizeof(uint32_t) * kWaves * kRadix;
  constexpr size_t kStageBytes = kKeyBytes > kCountBytes ? kKeyBytes : kCountBytes;
  // One LDS region serves first as the per-wave digit counters, then as the
  // tile regrouped by digit (keys, then values).
  __shared__ __attribute__((aligned(16))) unsigned char s_stage[kStageBytes];
  __shared__ uint32_t s_gbase[kRadix];
  __shared__ uint32_t s_wave_sum[kRadix / kWave];
  __shared__ uint32_t s_tile;

  uint32_t(*counts)[kRadix] = reinterpret_cast<uint32_t(*)[kRadix]>(s_stage);
  K *s_keys = reinterpret_cast<K *>(s_stage);
  uint32_t *s_vals = reinterpret_cast<uint32_t *>(s_stage);

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int shift = a.shift;
  const uint32_t mask = (1u << a.width) - 1u;
  const uint32_t n = a.n;

  for (int i = tid; i < kWaves * kRadix; i += kBlock) (&counts[0][0])[i] = 0u;
  if (tid == 0) s_tile = atomicAdd(a.tile_counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint32_t tile_base = tile * static_cast<uint32_t>(kTile);
  const uint32_t tile_count = min(n - tile_base, static_cast<uint32_t>(kTile));
  const bool full = tile_count == static_cast<uint32_t>(kTile);

  // 1. Load. Lanes past the end get an all-ones key: its digit is the
  // largest one the place can hold and it ranks after every real key, so the
  // padding occupies the last tile positions and is never written out.
  K key[kIpt];
  const uint32_t wave_base = tile_base + wave * kWaveItems + lane;
  if (full) {
#pragma unroll
    for (int i = 0; i < kIpt; ++i) key[i] = src[wave_base + i * kWave];
  } else {
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      const uint32_t idx = wave_base + i * kWave;
      key[i] = idx < n ? src[idx] : static_cast<K>(~static_cast<K>(0));
    }
  }

  // 2. Wave64 multi-split ranking.
  uint32_t pos[kIpt];
#pragma unroll
  for (int i = 0; i < kIpt; ++i) {
    const uint32_t d = digit_of(key[i], shift, mask);
    uint64_t peers = ~0ull;
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const uint32_t bit = (d >> b) & 1u;
      const uint64_t vote = __ballot(bit);
      const uint64_t mine = bit ? ~0ull : 0ull;
      peers &= ~(vote ^ mine);
    }
    const uint32_t below = count_below(peers);
    const uint32_t prior = counts[wave][d];
    pos[i] = prior + below;
    if (below == 0u) counts[wave][d] = prior + static_cast<uint32_t>(__popcll(peers));
  }
  __syncthreads();

  // 3. Per-digit sums: over waves (each wave's start inside its digit run)
  // and over digits (the run's start inside the tile).
  uint32_t total = 0u, local_start = 0u, published = 0u;
  if (tid < kRadix) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = counts[w][tid];
      counts[w][tid] = total;
      total += c;
    }
    published = total;
    if (!full && static_cast<uint32_t>(tid) == mask) published -= kTile - tile_count;
    // 4a. Publish this tile's count (tile 0's count is already its prefix).
    store_status(&a.status[static_cast<size_t>(tile) * kRadix + tid],
                 (tile == 0u ? kFlagG : kFlagL) | published);
    uint32_t incl = total;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += t;
    }
    if (lane == kWave - 1) s_wave_sum[wave] = incl;
    local_start = incl - total;
  }
  __syncthreads();
  if (tid < kRadix) {
    for (int w = 0; w < wave; ++w) local_start += s_wave_sum[w];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) counts[w][tid] += local_start;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kIpt; ++i) pos[i] += counts[wave][digit_of(key[i], shift, mask)];
  __syncthreads();  // the counters are dead; the region now holds the tile

  // 5a. Regroup the keys by digit in LDS.
#pragma unroll
  for (int i = 0; i < kIpt; ++i) s_keys[pos[i]] = key[i];

  uint32_t val[kVals ? kIpt : 1];
  if constexpr (kVals) {
    const uint32_t *__restrict__ vsrc = a.vals[src_id];
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      const uint32_t idx = wave_base + i * kWave;
      val[i] = (full || idx < n) ? vsrc[idx] : 0u;
    }
  }

  // 4b. Decoupled look-back: thread v sums the counts of earlier tiles for
  // digit v, walking backwards until it meets an inclusive prefix.
  if (tid < kRadix) {
    const uint32_t bin_start = a.bin_offsets[tid];
    uint32_t exclusive = 0u;
    if (tile != 0u) {
      uint32_t pred = tile - 1u;
      while (true) {
        const uint32_t s = load_status(&a.status[static_cast<size_t>(pred) * kRadix + tid]);
        const uint32_t flag = s & kFlagMask;
        if (flag == 0u) {
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        exclusive += s & kValueMask;
        if (flag == kFlagG) break;
        --pred;
      }
      store_status(&a.status[static_cast<size_t>(tile) * kRadix + tid],
                   kFlagG | (exclusive + published));
    }
    // Global position of the key at tile position q with digit v is
    // s_gbase[v] + q (unsigned wrap-around cancels in the sum).
    s_gbase[tid] = bin_start + exclusive - local_start;
  }
  __syncthreads();

  // 5b. Write runs of keys to their bins.
  uint32_t dst_idx[kVals ? kIpt : 1];
#pragma unroll
  for (int i = 0; i < kIpt; ++i) {
    const uint32_t q = i * kBlock + tid;
    if (full || q < tile_count) {
      const K k = s_keys[q];
      const uint32_t g = s_gbase[digit_of(k, shift, mask)] + q;
      if (g < n) dst[g] = k;  // always true when the counts are consistent
      if constexpr (kVals) dst_idx[i] = g;
    }
  }

  // 5c. Values follow their keys through the same LDS positions.
  if constexpr (kVals) {
    uint32_t *__restrict__ vdst = a.vals[dst_id];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kIpt; ++i) s_vals[pos[i]] = val[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      const uint32_t q = i * kBlock + tid;
      if ((full || q < tile_count) && dst_idx[i] < n) vdst[dst_idx[i]] = s_vals[q];
    }
  }
}

// Instantiated shapes: (key type, values, workgroup size, items per thread).
#define ONESWEEP_BINNING_SHAPES(X) \
  X(uint32_t, false, 256, 16)      \
  X(uint32_t, false, 512, 16)      \
  X(uint32_t, false, 512, 12)      \
  X(uint32_t, false, 256, 24)      \
  X(uint32_t, false, 1024, 8)      \
  X(uint32_t, true, 256, 16)       \
  X(uint32_t, true, 512, 16)       \
  X(uint32_t, true, 512, 12)       \
  X(uint32_t, true, 256, 24)       \
  X(uint64_t, false, 256, 16)      \
  X(uint64_t, false, 512, 8)       \
  X(uint64_t, false, 512, 12)      \
  X(uint64_t, true, 256, 16)       \
  X(uint64_t, true, 512, 8)        \
  X(uint64_t, true, 512, 12)

bool binning_shape_supported(const BinningShape &s) {
#define ONESWEEP_MATCH(K, V, B, I) \
  if (s.key_bits == 8 * (int)sizeof(K) && s.has_values == V && s.block == B && s.ipt == I) return true;
  ONESWEEP_BINNING_SHAPES(ONESWEEP_MATCH)
#undef ONESWEEP_MATCH
  return false;
}

BinningShape binning_default_shape(int key_bits, bool has_values) {
  if (key_bits == 64) return BinningShape{64, has_values, 512, 8};
  return BinningShape{32, has_values, 512, 16};
}

hipError_t launch_binning(const BinningShape &s, const void *args, uint32_t grid,
                          hipStream_t stream) {
#define ONESWEEP_LAUNCH(K, V, B, I)                                                          \
  if (s.key_bits == 8 * (int)sizeof(K) && s.has_values == V && s.block == B && s.ipt == I) { \
    hipLaunchKernelGGL((binning_kernel<K, V, B, I>), dim3(grid), dim3(B), 0, stream,          \
                       *static_cast<const BinningArgs<K> *>(args));                          \
    return hipGetLastError();                                                                \
  }
  ONESWEEP_BINNING_SHAPES(ONESWEEP_LAUNCH)
#undef ONESWEEP_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace onesweep
