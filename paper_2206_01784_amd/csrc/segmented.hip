// Segmented sort: many independent stable sorts, one per range
// [offsets[s], offsets[s + 1]), enqueued as a fixed sequence of kernels (so the
// whole batch can be captured in one HIP graph) and driven by device-side
// offsets, so the host never learns the segment lengths.
//
//  - classify: one thread per segment validates its offsets and assigns the
//    segment to a class by length: three classes small enough to be sorted
//    inside one workgroup's LDS (up to 512, 2048 and 8192 keys) and a
//    "large" class. Each large segment is cut into binning tiles whose
//    descriptors are consecutive.
//  - LDS sort: one workgroup per segment loads it once, runs the LSD passes
//    over 8-bit digits in LDS with the same wave64 multi-split ranking as the
//    binning kernel, and writes it once.
//  - large segments: an Onesweep sort per segment (Section 3), one binning
//    launch per place over the tiles of all large segments, each segment its
//    own chained scan. The first place's launch also counts the digits of
//    every place per segment: its first workgroups count, the later ones bin
//    (kBinSegCounted in the binning kernel); every binning tile turns its
//    segment's counts of the place into bin starts itself.
#include "device_common.hpp"
#include "internal.hpp"

namespace onesweep {

// ---------------------------------------------------------------- classify
constexpr int kClassifyBlock = 1024;

// Clears the plan (counts, error word) and the binning tile counters; the
// classify workgroups then accumulate into the plan with atomics.
__global__ void __launch_bounds__(64) segment_init_kernel(SegmentPlan *plan,
                                                          uint32_t *tile_counters) {
  const int tid = threadIdx.x;
  if (tid < kMaxPlaces) tile_counters[tid] = 0u;
  reinterpret_cast<uint32_t *>(plan)[tid] = 0u;
}

// One thread per segment. A workgroup counts its segments per class and its
// large segments' tiles, reserves that many list entries and tiles with one
// atomic per class, and writes the entries (list order across workgroups
// is arbitrary; every segment is sorted on its own, so order does not
// matter, and each large segment's tiles stay consecutive).
__global__ void __launch_bounds__(kClassifyBlock) classify_kernel(ClassifyArgs a) {
  constexpr int kWaves = kClassifyBlock / kWave;
  constexpr int kQ = kSegClasses + 2;  // per-class counts, then tiles
  __shared__ uint32_t s_wave[kWaves][kQ];
  __shared__ uint32_t s_base[kQ];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const uint32_t T = a.tile_items;
  const uint32_t s = blockIdx.x * kClassifyBlock + tid;
  bool bad = false;
  uint32_t cls = kQ, tiles = 0u, lo = 0u, len = 0u;
  if (s < a.num_segments) {
    lo = a.offsets[s];
    const uint32_t hi = a.offsets[s + 1];
    if (hi < lo || hi > a.n) {
      bad = true;
    } else {
      len = hi - lo;
      if (len > 0u) {
        cls = kSegClasses;
        for (int c = kSegClasses - 1; c >= 0; --c)
          if (len <= a.limit[c]) cls = c;
        if (cls == kSegClasses) tiles = (len + T - 1u) / T;
      }
    }
  }
  if (s == 0 && (a.offsets[0] != 0u || a.offsets[a.num_segments] != a.n)) bad = true;
  uint32_t rank = 0u;
#pragma unroll
  for (int c = 0; c <= kSegClasses; ++c) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(cls == static_cast<uint32_t>(c));
    if (cls == static_cast<uint32_t>(c)) rank = count_below(m);
    if (lane == 0) s_wave[wave][c] = static_cast<uint32_t>(__popcll(m));
  }
  uint32_t incl = tiles;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) s_wave[wave][kQ - 1] = incl;
  const int any_bad = __syncthreads_or(bad);
  if (tid < kQ) {
    uint32_t total = 0u;
    for (int w = 0; w < kWaves; ++w) total += s_wave[w][tid];
    uint32_t *counter = tid < kQ - 1 ? &a.plan->count[tid] : &a.plan->large_tiles;
    s_base[tid] = total ? atomicAdd(counter, total) : 0u;
  }
  if (tid == 0 && any_bad) atomicOr(&a.plan->error, 1u);
  __syncthreads();
  uint32_t pre[kQ];
#pragma unroll
  for (int c = 0; c < kQ; ++c) {
    uint32_t before = 0u;
    for (int w = 0; w < wave; ++w) before += s_wave[w][c];
    pre[c] = s_base[c] + before;
  }
  if (cls < static_cast<uint32_t>(kSegClasses)) {
    const uint32_t idx = pre[cls] + rank;
    if (idx < a.capacity[cls]) a.lists[cls][idx] = s;
    else atomicOr(&a.plan->error, 1u);  // only reachable with invalid offsets
  } else if (cls == static_cast<uint32_t>(kSegClasses)) {
    const uint32_t li = pre[kSegClasses] + rank;
    const uint32_t first = pre[kQ - 1] + incl - tiles;
    if (li >= a.max_large || first + tiles > a.max_tiles) {
      atomicOr(&a.plan->error, 1u);  // only reachable with invalid offsets
    } else {
      a.large_len[li] = len;
      for (uint32_t k = 0; k < tiles; ++k)
        a.tile_info[first + k] = make_uint4(lo + k * T, min(T, len - k * T), lo, li);
    }
  }
}

hipError_t launch_classify(const ClassifyArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(segment_init_kernel, dim3(1), dim3(64), 0, stream, a.plan, a.tile_counters);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.num_segments == 0) return e;
  const uint32_t grid = (a.num_segments + kClassifyBlock - 1) / kClassifyBlock;
  hipLaunchKernelGGL(classify_kernel, dim3(grid), dim3(kClassifyBlock), 0, stream, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- clear
// Clears the status rows of the tiles that exist and the histograms of the
// large segments that exist, sized from the plan on the device.
__global__ void __launch_bounds__(256) segment_clear_kernel(SegmentClearArgs a) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  const size_t first = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
  if (a.plan->error) return;
  const size_t status_vecs = static_cast<size_t>(a.plan->large_tiles) * (kRadix / 4);
  for (int j = 0; j < a.places; ++j) {
    uint4 *row = reinterpret_cast<uint4 *>(a.status + j * a.status_words_per_place);
    for (size_t i = first; i < status_vecs; i += stride) row[i] = zero;
  }
  const size_t hist_vecs =
      static_cast<size_t>(a.plan->count[kSegClasses]) * a.places * (kRadix / 4);
  uint4 *hist = reinterpret_cast<uint4 *>(a.hist);
  for (size_t i = first; i < hist_vecs; i += stride) hist[i] = zero;
}

hipError_t launch_segment_clear(const SegmentClearArgs &a, uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(segment_clear_kernel, dim3(grid), dim3(256), 0, stream, a);
  return hipGetLastError();
}

// Copy of the large segments' keys (and values) from the temporary buffer to
// the output, for an odd number of passes with the input aliasing the output.
__global__ void __launch_bounds__(256) segment_copy_kernel(SegmentCopyArgs a) {
  const uint32_t tiles = a.plan->error ? 0u : a.plan->large_tiles;
  for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const uint4 info = a.tile_info[t];
    if (a.key_bytes == 4) {
      const uint32_t *s = static_cast<const uint32_t *>(a.keys_src);
      uint32_t *d = static_cast<uint32_t *>(a.keys_dst);
      for (uint32_t i = threadIdx.x; i < info.y; i += 256) d[info.x + i] = s[info.x + i];
    } else {
      const uint64_t *s = static_cast<const uint64_t *>(a.keys_src);
      uint64_t *d = static_cast<uint64_t *>(a.keys_dst);
      for (uint32_t i = threadIdx.x; i < info.y; i += 256) d[info.x + i] = s[info.x + i];
    }
    if (a.vals_src != nullptr && a.vals_dst != nullptr && a.vals_src != a.vals_dst)
      for (uint32_t i = threadIdx.x; i < info.y; i += 256)
        a.vals_dst[info.x + i] = a.vals_src[info.x + i];
  }
}

hipError_t launch_segment_copy(const SegmentCopyArgs &a, uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(segment_copy_kernel, dim3(grid), dim3(256), 0, stream, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- LDS sort
// One workgroup sorts one segment of at most kBlock * kIpt keys at a time
// (workgroups take the class's segments cyclically). The key at slot
// q = wave * 64 * kIpt + 64 * i + lane sits in register i of that lane, so
// (wave, i, lane) order is slot order and the multi-split ranks are stable.
// Per digit place: rank every key among the earlier keys with its digit,
// turn the per-wave digit counts into positions, scatter the keys to their
// positions in LDS and read them back in slot order. Batches of 64 slots
// that start past the segment's end take no part; the last partial batch is
// padded with all-ones keys, which rank after every real key and so stay in
// the slots past the end. Keys are held as their ordered bits (signed,
// floating-point and descending orders) from load to store.
// The 1024-thread class (32-bit keys only) is held to 64 registers so two
// workgroups fit a CU.
template <typename K, int kBlock>
constexpr int lds_sort_waves_per_eu() {
  return kBlock >= 1024 && sizeof(K) == 4 ? 8 : 4;
}

// Wave-level digit match of the LDS sort: one ballot per digit bit (the
// default: with the three-input OR-of-XOR per ballot half, 20000 log-normal
// segments of 2^26 32-bit keys sort in 0.75 ms against 0.79 with masks;
// pairs and 64-bit keys are even), or 64-bit presence masks in LDS (an
// atomic OR per lane and one read per batch). The masks overlay the tile
// buffer, which is idle while keys are ranked.
#ifndef ONESWEEP_LDS_PRESENCE
#define ONESWEEP_LDS_PRESENCE 0
#endif
constexpr bool kLdsPresence = ONESWEEP_LDS_PRESENCE != 0;

template <typename K, bool kVals, int kBlock, int kIpt, bool kOrdered>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(lds_sort_waves_per_eu<K, kBlock>())))
    lds_sort_kernel(LdsSortArgs a) {
  constexpr int kWaves = kBlock / kWave;
  constexpr int kTile = kBlock * kIpt;
  constexpr int kWaveItems = kWave * kIpt;
  constexpr size_t kDataBytes = kTile * (sizeof(K) > 4 ? sizeof(K) : 4);
  __shared__ __attribute__((aligned(16))) unsigned char s_data[kDataBytes];
  __shared__ uint32_t s_cnt[kWaves * kRadix];
  __shared__ uint32_t s_wave_sum[kWaves];
  K *s_keys = reinterpret_cast<K *>(s_data);
  uint32_t *s_vals = reinterpret_cast<uint32_t *>(s_data);
  uint64_t *s_mask = reinterpret_cast<uint64_t *>(s_data);  // [wave][digit] while ranking
  static_assert(!kLdsPresence || kDataBytes >= sizeof(uint64_t) * kWaves * kRadix,
                "presence masks fit the tile buffer");
  auto clear_masks = [&]() {
    if constexpr (kLdsPresence) {
      uint4 *z = reinterpret_cast<uint4 *>(s_data);
      for (int x = threadIdx.x; x < kWaves * kRadix / 2; x += kBlock)
        z[x] = make_uint4(0u, 0u, 0u, 0u);
    }
  };

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const K *__restrict__ kin = static_cast<const K *>(a.keys_in);
  K *__restrict__ kout = static_cast<K *>(a.keys_out);
  const uint32_t count = a.plan->error ? 0u : a.plan->count[a.cls];
  const uint32_t *list = a.list;
  const uint32_t wave_first = static_cast<uint32_t>(wave) * kWaveItems;

  for (int x = tid; x < kWaves * kRadix; x += kBlock) s_cnt[x] = 0u;
  clear_masks();
  __syncthreads();

  for (uint32_t e = blockIdx.x; e < count; e += gridDim.x) {
    const uint32_t s = list[e];
    const uint32_t lo = a.offsets[s];
    const uint32_t len = a.offsets[s + 1] - lo;
    K key[kIpt];
    uint32_t val[kVals ? kIpt : 1];
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      const uint32_t q = wave_first + i * kWave + lane;
      // keys are held as their ordered bits from load to store
      key[i] = q >= len ? static_cast<K>(~static_cast<K>(0))
                        : (kOrdered ? ordered_bits(kin[lo + q], a.order) : kin[lo + q]);
      if constexpr (kVals) val[i] = q < len ? a.vals_in[lo + q] : 0u;
    }
    for (int j = 0; j < a.places; ++j) {
      const int shift = a.begin_bit + j * a.digit_bits;
      const int width = min(a.digit_bits, a.end_bit - shift);
      const uint32_t mask = (1u << width) - 1u;
      uint32_t pos[kIpt];
#pragma unroll
      for (int i = 0; i < kIpt; ++i) {
        pos[i] = 0u;
        if (wave_first + i * kWave < len) {
          const uint32_t d = digit_of(key[i], shift, mask);
          uint32_t peers_lo = ~0u, peers_hi = ~0u;
          uint64_t *m = &s_mask[wave * kRadix + d];
          if constexpr (kLdsPresence) {
            __hip_atomic_fetch_or(m, 1ull << lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __builtin_amdgcn_wave_barrier();
            const uint64_t peers = *m;
            peers_lo = static_cast<uint32_t>(peers);
            peers_hi = static_cast<uint32_t>(peers >> 32);
          } else {
            // lanes holding another digit: per bit, the vote XOR this lane's
            // bit, ORed in (one three-input operation per 32-lane half)
            uint32_t mis_lo = 0u, mis_hi = 0u;
#pragma unroll
            for (int b = 0; b < kRadixBits; ++b) {
              uint32_t own = static_cast<uint32_t>(__builtin_amdgcn_sbfe(static_cast<int>(d), b, 1));
              asm volatile("" : "+v"(own));  // vote on the extracted bit: one compare
              const uint64_t vote = __builtin_amdgcn_ballot_w64(own != 0u);
              mis_lo = __builtin_amdgcn_bitop3_b32(mis_lo, static_cast<uint32_t>(vote), own, 0xF6);
              mis_hi = __builtin_amdgcn_bitop3_b32(mis_hi, static_cast<uint32_t>(vote >> 32), own, 0xF6);
            }
            peers_lo = ~mis_lo;
            peers_hi = ~mis_hi;
          }
          uint32_t &c = s_cnt[wave * kRadix + d];
          const uint32_t prior = c;
          pos[i] = prior + __builtin_amdgcn_mbcnt_hi(peers_hi,
                                                     __builtin_amdgcn_mbcnt_lo(peers_lo, 0u));
          c = prior + static_cast<uint32_t>(__popc(peers_lo) + __popc(peers_hi));
          // every lane of the group writes the same values
          if constexpr (kLdsPresence) *m = 0ull;
          __builtin_amdgcn_wave_barrier();
        }
      }
      __syncthreads();
      // Digit starts: exclusive scan of the counts in (digit, wave) order.
      digit_major_exclusive_scan<kBlock>(s_cnt, s_wave_sum);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kIpt; ++i)
        if (wave_first + i * kWave < len) {
          pos[i] += s_cnt[wave * kRadix + digit_of(key[i], shift, mask)];
          s_keys[pos[i]] = key[i];
        }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kIpt; ++i)
        if (wave_first + i * kWave < len) key[i] = s_keys[wave_first + i * kWave + lane];
      if constexpr (kVals) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kIpt; ++i)
          if (wave_first + i * kWave < len) s_vals[pos[i]] = val[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kIpt; ++i)
          if (wave_first + i * kWave < len) val[i] = s_vals[wave_first + i * kWave + lane];
      }
      // The counters were last read before the scatter's barrier; the masks
      // overlay the tile buffer, so they are cleared once every thread has
      // read its keys (and values) back.
      if constexpr (kLdsPresence) __syncthreads();
      for (int x = tid; x < kWaves * kRadix; x += kBlock) s_cnt[x] = 0u;
      clear_masks();
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      const uint32_t q = wave_first + i * kWave + lane;
      if (q < len) {
        kout[lo + q] = kOrdered ? original_bits(key[i], a.order) : key[i];
        if constexpr (kVals) a.vals_out[lo + q] = val[i];
      }
    }
  }
}

// Classes of 512, 2048 and 8192 keys: 64 and 256 threads with 8 keys each;
// the largest class with 1024 threads x 8 keys for 32-bit keys only and
// 512 threads x 16 keys otherwise. Measured on 20000 log-normal segments of
// 2^26 keys in all (ms per sort, 1024 x 8 against 512 x 16 in that class):
// 32-bit keys 0.73 / 0.75, 32-bit pairs 1.01 / 0.99, 64-bit keys 2.19 / 1.87,
// 64-bit pairs 3.02 / 2.54 (64-bit 1024-thread workgroups fit one per CU).
constexpr int kLdsCapacity[kSegClasses] = {512, 2048, 8192};

int lds_class_capacity(int cls) { return kLdsCapacity[cls]; }

int lds_class_block(int key_bits, bool has_values, int cls) {
  if (cls == 0) return 64;
  if (cls == 1) return 256;
  return key_bits == 32 && !has_values ? 1024 : 512;
}

namespace {
template <typename K, bool V, int B>
const void *lds_kernel_ptr(bool ordered) {
  constexpr int I = B <= 256 ? 8 : 8192 / B;  // keys per thread
  return ordered ? reinterpret_cast<const void *>(&lds_sort_kernel<K, V, B, I, true>)
                 : reinterpret_cast<const void *>(&lds_sort_kernel<K, V, B, I, false>);
}

const void *lds_kernel(int key_bits, bool has_values, int cls, bool ordered) {
  switch (cls) {
    case 0:
      if (key_bits == 32)
        return has_values ? lds_kernel_ptr<uint32_t, true, 64>(ordered)
                          : lds_kernel_ptr<uint32_t, false, 64>(ordered);
      return has_values ? lds_kernel_ptr<uint64_t, true, 64>(ordered)
                        : lds_kernel_ptr<uint64_t, false, 64>(ordered);
    case 1:
      if (key_bits == 32)
        return has_values ? lds_kernel_ptr<uint32_t, true, 256>(ordered)
                          : lds_kernel_ptr<uint32_t, false, 256>(ordered);
      return has_values ? lds_kernel_ptr<uint64_t, true, 256>(ordered)
                        : lds_kernel_ptr<uint64_t, false, 256>(ordered);
    default:
      if (key_bits == 32)
        return has_values ? lds_kernel_ptr<uint32_t, true, 512>(ordered)
                          : lds_kernel_ptr<uint32_t, false, 1024>(ordered);
      return has_values ? lds_kernel_ptr<uint64_t, true, 512>(ordered)
                        : lds_kernel_ptr<uint64_t, false, 512>(ordered);
  }
}
}  // namespace

hipError_t lds_sort_blocks_per_cu(int key_bits, bool has_values, int cls, int *blocks) {
  // the ordered variants differ only at load and store
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks, lds_kernel(key_bits, has_values, cls, false),
      lds_class_block(key_bits, has_values, cls), 0);
}

hipError_t launch_lds_sort(int key_bits, bool has_values, const LdsSortArgs &a, uint32_t grid,
                           hipStream_t stream) {
  const void *k = lds_kernel(key_bits, has_values, a.cls, !key_order_is_plain(a.order));
  LdsSortArgs copy = a;
  void *params[] = {&copy};
  return hipLaunchKernel(k, dim3(grid), dim3(lds_class_block(key_bits, has_values, a.cls)),
                         params, 0, stream);
}

}  // namespace onesweep
