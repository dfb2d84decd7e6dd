// Phases 1 and 2 of Onesweep (Section 3, "Upfront histogram kernel" and
// "Exclusive sum kernel", Figure 5), plus the small support kernels (clear,
// copy) that keep the launch sequence free of memset/memcpy nodes.
#include "device_common.hpp"
#include "internal.hpp"

namespace onesweep {

// ---------------------------------------------------------------- histogram
//
// A persistent grid (a fixed number of workgroups per CU) walks the keys in
// tile-cyclic order. Every workgroup counts into private LDS histograms with
// LDS atomics and, once its tiles are consumed, adds them to the global
// histograms with global atomics. Counts depend only on the multiset of keys,
// so one read of the keys yields the histograms of every digit place.
//
// kCopies interleaved copies of each counter (copy = lane % kCopies, copy
// index fastest) keep lanes that share a digit on different LDS banks, which
// bounds the serialisation of skewed inputs (all-equal keys) to
// 64 / kCopies-way.
template <typename K, int kBlock, int kVec, int kCopies, bool kOrdered>
__global__ void __launch_bounds__(kBlock) histogram_kernel(HistogramArgs<K> a) {
  constexpr int kMaxP = static_cast<int>(sizeof(K));  // places one launch counts
  constexpr int kPerVec = 16 / static_cast<int>(sizeof(K));
  constexpr int kTile = kBlock * kVec * kPerVec;
  __shared__ uint32_t s_hist[kMaxP * kRadix * kCopies];

  const int tid = threadIdx.x;
  for (int i = tid; i < kMaxP * kRadix * kCopies; i += kBlock) s_hist[i] = 0u;

  int shifts[kMaxP];
  uint32_t masks[kMaxP];
#pragma unroll
  for (int j = 0; j < kMaxP; ++j) {
    const int lo = a.begin_bit + j * a.digit_bits;
    const int hi = min(lo + a.digit_bits, a.end_bit);
    shifts[j] = lo < 64 ? lo : 0;
    masks[j] = (j < a.places) ? ((1u << (hi - lo)) - 1u) : 0u;
  }
  const int places = a.places;
  uint32_t *my_hist = s_hist + (tid % kCopies);
  __syncthreads();

  auto count_key = [&](K k) {
    const K t = kOrdered ? ordered_bits(k, a.order) : k;
#pragma unroll
    for (int j = 0; j < kMaxP; ++j) {
      if (j < places) {
        const uint32_t d = static_cast<uint32_t>(t >> shifts[j]) & masks[j];
        atomicAdd(&my_hist[(j * kRadix + d) * kCopies], 1u);
      }
    }
  };

  // 32-bit keys: a wave whose 64 keys are all equal (constant or nearly
  // constant inputs) adds 64 to one counter per place from its first lane
  // instead of 64 same-address atomics per place; the test is one ballot per
  // key (measured with 8 copies in 256-thread workgroups: all-equal keys
  // 437 -> 248 us at 2^28, uniform keys unchanged, AND-skewed keys +4-7%;
  // 64-bit keys lost 28% and skip it).
  const bool wave_leader = (tid & (kWave - 1)) == 0;
  auto count_key_wave = [&](K k) {
    if constexpr (sizeof(K) != 4) {
      count_key(k);
      return;
    }
    const K k0 = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(k));
    if (__ballot(k != k0) == 0ull) {
      if (wave_leader) {
        const K t = kOrdered ? ordered_bits(k0, a.order) : k0;
#pragma unroll
        for (int j = 0; j < kMaxP; ++j) {
          if (j < places) {
            const uint32_t d = static_cast<uint32_t>(t >> shifts[j]) & masks[j];
            atomicAdd(&my_hist[(j * kRadix + d) * kCopies], static_cast<uint32_t>(kWave));
          }
        }
      }
    } else {
      count_key(k);
    }
  };

  const uint32_t n = a.n;
  const bool aligned = (reinterpret_cast<uintptr_t>(a.keys) & 15u) == 0u;
  const uint32_t stride = gridDim.x * static_cast<uint32_t>(kTile);
  uint32_t base = blockIdx.x * static_cast<uint32_t>(kTile);
  auto count_vec = [&](const uint4 &q) {  // whole tiles: every lane active
    if constexpr (sizeof(K) == 4) {
      count_key_wave(q.x);
      count_key_wave(q.y);
      count_key_wave(q.z);
      count_key_wave(q.w);
    } else {
      count_key_wave(static_cast<K>(q.x) | (static_cast<K>(q.y) << 32));
      count_key_wave(static_cast<K>(q.z) | (static_cast<K>(q.w) << 32));
    }
  };
  if (aligned) {
    // Whole tiles, software-pipelined: the next tile's loads are in flight
    // while this one is counted (n < 2^31 keeps base + stride from wrapping).
    auto whole = [&](uint32_t b) { return b < n && n - b >= static_cast<uint32_t>(kTile); };
    uint4 q[kVec];
    if (whole(base)) {
      const uint4 *v = reinterpret_cast<const uint4 *>(a.keys + base);
#pragma unroll
      for (int i = 0; i < kVec; ++i) q[i] = v[i * kBlock + tid];
    }
    while (whole(base)) {
      uint4 cur[kVec];
#pragma unroll
      for (int i = 0; i < kVec; ++i) cur[i] = q[i];
      const uint32_t next = base + stride;
      if (whole(next)) {
        const uint4 *v = reinterpret_cast<const uint4 *>(a.keys + next);
#pragma unroll
        for (int i = 0; i < kVec; ++i) q[i] = v[i * kBlock + tid];
      }
#pragma unroll
      for (int i = 0; i < kVec; ++i) count_vec(cur[i]);
      base = next;
    }
  }
  // The last, partial tile (or every tile when the keys are not 16-byte
  // aligned), one key per thread at a time.
  for (; base < n; base += stride) {
    const uint32_t end = min(n, base + static_cast<uint32_t>(kTile));
    for (uint32_t i = base + tid; i < end; i += kBlock) count_key(a.keys[i]);
  }
  __syncthreads();
  for (int i = tid; i < places * kRadix; i += kBlock) {
    uint32_t sum = 0u;
#pragma unroll
    for (int c = 0; c < kCopies; ++c) sum += s_hist[i * kCopies + c];
    if (sum != 0u) {
      if (a.hist64 != nullptr) atomicAdd(&a.hist64[i], static_cast<unsigned long long>(sum));
      else atomicAdd(&a.hist[i], sum);
    }
  }
}

// Workgroup shape: 1024 threads, two workgroups (32 waves) per CU. 32-bit
// keys keep 16 interleaved copies of their 4 x 256 counters (64 KiB of LDS),
// 64-bit keys 8 copies of 8 x 256 (64 KiB). Measured at 2^28 32-bit keys
// against 256-thread workgroups with 8 copies: uniform 251 -> 205 us, AND of
// 4 words 451 -> 238 us, all equal 246 -> 214 us; 16 copies in 256-thread
// workgroups (8 waves per CU) were slower (343 us); 2^27 64-bit keys
// 249 -> 230 us.
constexpr int kHistVec = 4;  // uint4 loads per thread per tile
constexpr int kHistBlock = 1024;
constexpr int kHistCopies32 = 16;
constexpr int kHistCopies64 = 8;

hipError_t launch_histogram(int key_bits, const void *keys, uint32_t *hist,
                            unsigned long long *hist64, uint32_t n, int begin_bit, int end_bit,
                            int places, int digit_bits, const KeyOrder &order, uint32_t grid,
                            hipStream_t stream) {
  if (key_bits == 32) {
    HistogramArgs<uint32_t> a{static_cast<const uint32_t *>(keys), hist, hist64, n, begin_bit,
                              end_bit, places, digit_bits, order};
    if (key_order_is_plain(order))
      hipLaunchKernelGGL((histogram_kernel<uint32_t, kHistBlock, kHistVec, kHistCopies32, false>),
                         dim3(grid), dim3(kHistBlock), 0, stream, a);
    else
      hipLaunchKernelGGL((histogram_kernel<uint32_t, kHistBlock, kHistVec, kHistCopies32, true>),
                         dim3(grid), dim3(kHistBlock), 0, stream, a);
  } else {
    HistogramArgs<uint64_t> a{static_cast<const uint64_t *>(keys), hist, hist64, n, begin_bit,
                              end_bit, places, digit_bits, order};
    if (key_order_is_plain(order))
      hipLaunchKernelGGL((histogram_kernel<uint64_t, kHistBlock, kHistVec, kHistCopies64, false>),
                         dim3(grid), dim3(kHistBlock), 0, stream, a);
    else
      hipLaunchKernelGGL((histogram_kernel<uint64_t, kHistBlock, kHistVec, kHistCopies64, true>),
                         dim3(grid), dim3(kHistBlock), 0, stream, a);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- exclusive sums + plan
//
// One workgroup of 256 threads: thread v owns digit v of every place. Besides
// the global bin offsets, it marks a place trivial when one bin holds all n
// keys (the pass would be the identity permutation) and lays out the buffer
// route of the executed passes. Sums are taken in 64 bits; counts and offsets
// are 32-bit words, or 64-bit ones when hist64 / offsets64 are given.
__global__ void __launch_bounds__(kRadix) scan_kernel(const uint32_t *hist,
                                                      const unsigned long long *hist64,
                                                      uint32_t *offsets,
                                                      unsigned long long *offsets64,
                                                      PassPlan *plan, int places, uint64_t n,
                                                      int alias) {
  __shared__ uint64_t s_wave_sum[kRadix / kWave];
  __shared__ uint32_t s_run[kMaxPlaces];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  for (int j = 0; j < places; ++j) {
    const uint64_t h = hist64 != nullptr ? static_cast<uint64_t>(hist64[j * kRadix + tid])
                                         : static_cast<uint64_t>(hist[j * kRadix + tid]);
    uint64_t incl = h;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint64_t t = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += t;
    }
    if (lane == kWave - 1) s_wave_sum[wave] = incl;
    const int trivial = __syncthreads_or(h == n);
    uint64_t excl = incl - h;
    for (int w = 0; w < wave; ++w) excl += s_wave_sum[w];
    if (offsets64 != nullptr) offsets64[j * kRadix + tid] = excl;
    else offsets[j * kRadix + tid] = static_cast<uint32_t>(excl);
    if (tid == 0) s_run[j] = trivial ? 0u : 1u;
    __syncthreads();  // s_wave_sum is reused by the next place
  }
  if (tid == 0) {
    PassPlan p;
    uint32_t executed = 0;
    for (int j = 0; j < places; ++j) executed += s_run[j];
    uint32_t cur = kBufIn, k = 0;
    for (int j = 0; j < kMaxPlaces; ++j) {
      p.run[j] = 0u;
      p.src[j] = kBufIn;
      p.dst[j] = kBufOut;
      if (j < places && s_run[j]) {
        ++k;
        uint32_t to;
        if (alias)  // input == output: the first pass must not write in place
          to = (k & 1u) ? kBufTmp : kBufOut;
        else        // the last executed pass writes the output
          to = ((executed - k) & 1u) ? kBufTmp : kBufOut;
        p.run[j] = 1u;
        p.src[j] = cur;
        p.dst[j] = to;
        cur = to;
      }
    }
    p.executed = executed;
    if (executed == 0u)
      p.copy_src = alias ? kNoBuffer : kBufIn;
    else
      p.copy_src = (cur == kBufOut) ? kNoBuffer : cur;
    p.lookback_error = 0u;
    for (int i = 0; i < 13; ++i) p.pad[i] = 0u;
    *plan = p;
  }
}

hipError_t launch_scan(const uint32_t *hist, const unsigned long long *hist64, uint32_t *offsets,
                       unsigned long long *offsets64, PassPlan *plan, int places, uint64_t n,
                       bool alias, hipStream_t stream) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kRadix), 0, stream, hist, hist64, offsets,
                     offsets64, plan, places, n, alias ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- copy
__global__ void __launch_bounds__(256) copy_kernel(CopyArgs a) {
  uint32_t from = kBufIn;
  if (a.plan != nullptr) {
    from = a.plan->copy_src;
    if (from == kNoBuffer) return;
  }
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  const size_t first = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  auto copy_bytes = [&](const void *s, void *d, size_t bytes) {
    if (s == d) return;
    const bool vec = ((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(d)) & 15u) == 0u;
    size_t done = 0;
    if (vec) {
      const size_t nv = bytes / 16;
      const uint4 *sv = static_cast<const uint4 *>(s);
      uint4 *dv = static_cast<uint4 *>(d);
      for (size_t i = first; i < nv; i += stride) dv[i] = sv[i];
      done = nv * 16;
    }
    const uint32_t *sw = static_cast<const uint32_t *>(s);
    uint32_t *dw = static_cast<uint32_t *>(d);
    for (size_t i = done / 4 + first; i < bytes / 4; i += stride) dw[i] = sw[i];
  };
  copy_bytes(a.keys[from], a.keys[kBufOut], static_cast<size_t>(a.n) * a.key_bytes);
  if (a.vals[from] != nullptr && a.vals[kBufOut] != nullptr)
    copy_bytes(a.vals[from], a.vals[kBufOut], static_cast<size_t>(a.n) * 4u);
}

hipError_t launch_copy(const CopyArgs &a, uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, stream, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- clear
__global__ void __launch_bounds__(256) fill_zero_kernel(uint32_t *p, size_t words) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  const size_t first = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t nv = (reinterpret_cast<uintptr_t>(p) & 15u) == 0u ? words / 4 : 0;
  uint4 *pv = reinterpret_cast<uint4 *>(p);
  for (size_t i = first; i < nv; i += stride) pv[i] = make_uint4(0u, 0u, 0u, 0u);
  for (size_t i = nv * 4 + first; i < words; i += stride) p[i] = 0u;
}

hipError_t launch_fill_zero(void *p, size_t bytes, uint32_t grid, hipStream_t stream) {
  if (bytes == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, stream,
                     static_cast<uint32_t *>(p), bytes / 4);
  return hipGetLastError();
}

}  // namespace onesweep
