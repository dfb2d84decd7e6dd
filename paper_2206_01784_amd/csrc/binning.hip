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

// Two ways to find, for every lane of a wavefront, the lanes holding the
// same digit (its "peers"), which is all the multi-split needs:
//  - kRankBallot: one ballot per digit bit; a lane ANDs each ballot or its
//    complement, by the value of its own bit (the paper's description);
//  - kRankPresence: every lane ORs its lane bit into a 64-bit presence mask
//    per digit in LDS and reads the mask back. OR is order-independent, so
//    the mask is exact whatever order the LDS serves the lanes in, and it
//    costs a few instructions per batch instead of four per digit bit.
enum RankAlgorithm : int { kRankBallot = 0, kRankPresence = 1 };

// Drop any global store whose index is not below n. Consistent counts never
// produce such an index; the check only turns a logic error into a wrong
// result instead of a memory fault.
#ifndef ONESWEEP_CHECKED_STORES
#define ONESWEEP_CHECKED_STORES 1
#endif
constexpr bool kCheckedStores = ONESWEEP_CHECKED_STORES != 0;

#ifndef ONESWEEP_LOOKBACK_WINDOW
#define ONESWEEP_LOOKBACK_WINDOW 4
#endif

// Predecessor tiles read per look-back round trip.
constexpr int kLookback = ONESWEEP_LOOKBACK_WINDOW;

// Occupancy target (waves per SIMD the register allocation must allow):
// as high as the key registers permit without spilling.
template <typename K, int kIpt>
constexpr int binning_waves_per_eu() {
  return (kIpt * sizeof(K)) <= 32 ? 8 : ((kIpt * sizeof(K)) <= 48 ? 5 : 4);
}

// Scan agent (used when BinningArgs::agents > 0). The paper's decoupled
// look-back lets every tile walk back over its predecessors' counts until it
// meets an inclusive prefix; the time a tile needs to find one grows with
// the rate at which tiles are issued, because every tile publishes its own
// prefix only after its own walk. Across the eight XCDs of MI355X the status
// words travel through the device-coherent path, which makes that walk the
// dominant cost of a pass. An agent instead computes the same chained scan
// in tile order: it reads the status rows of the next slots * kAgentRows
// tiles at once, extends the running prefix over the leading run of tiles
// that have published their counts, and writes each of those tiles'
// inclusive prefix (status G). Tiles then only wait for the word of their
// immediate predecessor. Agents take the first tickets, so they are running
// before any tile; every tile publishes its count without waiting, so the
// agent always progresses. The status words, values and final state are
// those of the paper's scheme (Figures 6 and 7f).
constexpr int kAgentRows = 16;

template <int kBlock>
__device__ void scan_agent(uint32_t *status, uint32_t tiles, uint32_t agent, uint32_t agents,
                           uint32_t *lds) {
  const int digits = kRadix / static_cast<int>(agents);  // 256, 128 or 64
  const int waves_per_slot = digits / kWave;
  const int slots = (kBlock / kWave) / waves_per_slot;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int slot = wave / waves_per_slot;
  const int local = (wave % waves_per_slot) * kWave + lane;
  const int digit = static_cast<int>(agent) * digits + local;
  uint32_t *s_valid = lds;                   // [slots][digits]
  uint32_t *s_sum = lds + slots * digits;    // [slots][digits]
  uint32_t cursor = 0u, prefix = 0u;
  while (true) {
    const uint32_t first = cursor + static_cast<uint32_t>(slot * kAgentRows);
    uint32_t st[kAgentRows];
#pragma unroll
    for (int k = 0; k < kAgentRows; ++k)
      st[k] = first + k < tiles ? load_status(&status[static_cast<size_t>(first + k) * kRadix + digit])
                                : 0u;
    uint32_t valid = 0u, sum = 0u;
    bool open = true;
#pragma unroll
    for (int k = 0; k < kAgentRows; ++k) {
      if (open && (st[k] & kFlagMask) != 0u) {
        sum += st[k] & kValueMask;
        ++valid;
      } else {
        open = false;
      }
    }
    s_valid[slot * digits + local] = valid;
    s_sum[slot * digits + local] = sum;
    __syncthreads();
    // Combine the slots in tile order up to the first slot that stopped
    // early; later slots wait for the next round.
    uint32_t running = prefix, advance = 0u, start = 0u;
    bool blocked = false, mine = false;
    for (int g = 0; g < slots; ++g) {
      if (g == slot) {
        mine = !blocked;
        start = running;
      }
      if (!blocked) {
        const uint32_t v = s_valid[g * digits + local];
        running += s_sum[g * digits + local];
        advance += v;
        blocked = v < static_cast<uint32_t>(kAgentRows);
      }
    }
    if (mine) {
      uint32_t p = start;
#pragma unroll
      for (int k = 0; k < kAgentRows; ++k) {
        if (static_cast<uint32_t>(k) < valid) {
          p += st[k] & kValueMask;
          store_status(&status[static_cast<size_t>(first + k) * kRadix + digit], kFlagG | p);
        }
      }
    }
    prefix = running;
    cursor += advance;
    if (!__syncthreads_or(cursor < tiles)) break;  // also guards the LDS reuse
    if (__builtin_amdgcn_ballot_w64(advance == 0u && cursor < tiles) != 0ull)
      __builtin_amdgcn_s_sleep(2);
  }
}

template <typename K, bool kVals, int kBlock, int kIpt, int kRank>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(binning_waves_per_eu<K, kIpt>())))
    binning_kernel(BinningArgs<K> a) {
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

  // Per-wave rank state, one entry per digit: the running count of the digit
  // in the wave (word 0) and, for kRankPresence, the 64-bit presence mask
  // (words 2-3). The region is reused for the regrouped tile afterwards.
  constexpr int kEntryWords = kRank == kRankPresence ? 4 : 1;
  constexpr size_t kKeyBytes = sizeof(K) * kTile;
  constexpr size_t kRankBytes = sizeof(uint32_t) * kWaves * kRadix * kEntryWords;
  constexpr size_t kStageBytes = kKeyBytes > kRankBytes ? kKeyBytes : kRankBytes;
  __shared__ __attribute__((aligned(16))) unsigned char s_stage[kStageBytes];
  __shared__ uint32_t s_gbase[kRadix];
  __shared__ uint32_t s_wave_sum[kRadix / kWave];
  __shared__ uint32_t s_tile;


  uint32_t *s_rank = reinterpret_cast<uint32_t *>(s_stage);
  K *s_keys = reinterpret_cast<K *>(s_stage);
  uint32_t *s_vals = reinterpret_cast<uint32_t *>(s_stage);

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int shift = a.shift;
  const int width = a.width;
  const uint32_t mask = (1u << width) - 1u;
  const uint32_t n = a.n;

  {
    uint4 *z = reinterpret_cast<uint4 *>(s_rank);
    for (int i = tid; i < static_cast<int>(kRankBytes / 16); i += kBlock)
      z[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (tid == 0) s_tile = atomicAdd(a.tile_counter, 1u);
  __syncthreads();
  const uint32_t tiles = (n + kTile - 1) / kTile;
  if (s_tile < a.agents) {  // the first tickets run the scan agents
    scan_agent<kBlock>(a.status, tiles, s_tile, a.agents, s_rank);
    return;
  }
  const uint32_t tile = s_tile - a.agents;
  const bool agent_scan = a.agents != 0u;
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

  // 2. Wave64 multi-split ranking: pos[i] becomes the key's rank among the
  // wave's earlier keys with the same digit.
  uint32_t pos[kIpt];
  const uint32_t wave_table = static_cast<uint32_t>(wave) * kRadix * kEntryWords;
#pragma unroll
  for (int i = 0; i < kIpt; ++i) {
    const uint32_t d = digit_of(key[i], shift, mask);
    const uint32_t e = wave_table + d * kEntryWords;
    uint32_t peers_lo, peers_hi;
    if constexpr (kRank == kRankPresence) {
      uint64_t *presence = reinterpret_cast<uint64_t *>(s_rank + e + 2);
      __hip_atomic_fetch_or(presence, 1ull << lane, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_WORKGROUP);
      __builtin_amdgcn_wave_barrier();
      peers_lo = s_rank[e + 2];
      peers_hi = s_rank[e + 3];
    } else {
      // miss accumulates, per lane, the lanes whose digit differs in some
      // bit: miss |= vote ^ own in one 3-input bit operation per half
      // (truth table 0xf6 = S0 | (S1 ^ S2)); peers = ~miss. Bits at or above
      // the place width are 0 in every lane and change nothing.
      uint32_t miss_lo = 0u, miss_hi = 0u;
#pragma unroll
      for (int b = 0; b < kRadixBits; ++b) {
        const int own = __builtin_amdgcn_sbfe(static_cast<int>(d), b, 1);  // 0 or -1
        uint64_t vote;
        asm volatile("v_cmp_ne_u32_e64 %0, 0, %1" : "=s"(vote) : "v"(own));
        asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xf6"
            : "=v"(miss_lo)
            : "v"(miss_lo), "s"(static_cast<uint32_t>(vote)), "v"(own));
        asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xf6"
            : "=v"(miss_hi)
            : "v"(miss_hi), "s"(static_cast<uint32_t>(vote >> 32)), "v"(own));
      }
      peers_lo = ~miss_lo;
      peers_hi = ~miss_hi;
    }
    const uint32_t prior = s_rank[e];
    pos[i] = prior + __builtin_amdgcn_mbcnt_hi(peers_hi, __builtin_amdgcn_mbcnt_lo(peers_lo, 0u));
    // Every lane of the group stores the same new count (and clears the
    // presence mask), so the result does not depend on which store lands.
    const uint32_t next = prior + static_cast<uint32_t>(__popc(peers_lo) + __popc(peers_hi));
    if constexpr (kRank == kRankPresence) {
      *reinterpret_cast<uint4 *>(s_rank + e) = make_uint4(next, 0u, 0u, 0u);
    } else {
      s_rank[e] = next;
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // 3. Per-digit sums: over waves (each wave's start inside its digit run)
  // and over digits (the run's start inside the tile).
  // With up to 8 waves the per-wave starts stay in registers; with more
  // they are written back now and adjusted by the digit's start later.
  constexpr bool kStartsInRegs = kWaves <= 8;
  uint32_t total = 0u, local_start = 0u, published = 0u;
  uint32_t wave_start[kStartsInRegs ? kWaves : 1];
  // Thread v < 256 looks back for digit v. Its first window of kLookback
  // predecessors is issued now, so the latency overlaps the local scan and
  // the regrouping.
  uint32_t window[kLookback];
  if (tid < kRadix) {
#pragma unroll
    for (int w = 0; w < kLookback; ++w) {
      const int t = static_cast<int>(tile) - 1 - w;
      window[w] = (t >= 0 && (w == 0 || !agent_scan))
                      ? load_status(&a.status[static_cast<size_t>(t) * kRadix + tid])
                      : kFlagG;
    }
    if constexpr (kStartsInRegs) {
#pragma unroll
      for (int w = 0; w < kWaves; ++w) wave_start[w] = s_rank[(w * kRadix + tid) * kEntryWords];
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t v = wave_start[w];
        wave_start[w] = total;
        total += v;
      }
    } else {
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        uint32_t &c = s_rank[(w * kRadix + tid) * kEntryWords];
        const uint32_t v = c;
        c = total;
        total += v;
      }
    }
    published = total;
    if (!full && static_cast<uint32_t>(tid) == mask) published -= kTile - tile_count;
    // 4a. Publish this tile's count (tile 0's count is already its prefix).
    // On gfx9 one counter tracks both loads and stores of a wave, so a wave
    // that waits for a load also waits until its earlier stores have been
    // written through; under a full pass of scatter traffic that takes
    // microseconds. The look-back waves therefore hand the count to the next
    // four waves, which store it and never wait on a global load afterwards.
    const uint32_t word = (tile == 0u && !agent_scan ? kFlagG : kFlagL) | published;
    if constexpr (kBlock >= 2 * kRadix)
      s_gbase[tid] = word;
    else
      store_status(&a.status[static_cast<size_t>(tile) * kRadix + tid], word);
    const uint32_t incl = wave_inclusive_sum(total);
    if (lane == kWave - 1) s_wave_sum[wave] = incl;
    local_start = incl - total;
  }
  __syncthreads();
  if constexpr (kBlock >= 2 * kRadix) {
    if (tid >= kRadix && tid < 2 * kRadix)
      store_status(&a.status[static_cast<size_t>(tile) * kRadix + (tid - kRadix)],
                   s_gbase[tid - kRadix]);
  }
  if (tid < kRadix) {
    for (int w = 0; w < wave; ++w) local_start += s_wave_sum[w];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      if constexpr (kStartsInRegs)
        s_rank[(w * kRadix + tid) * kEntryWords] = wave_start[w] + local_start;
      else
        s_rank[(w * kRadix + tid) * kEntryWords] += local_start;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kIpt; ++i)
    pos[i] += s_rank[wave_table + digit_of(key[i], shift, mask) * kEntryWords];
  __syncthreads();  // the rank tables are dead; the region now holds the tile

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
  // digit v, walking backwards until it meets an inclusive prefix, one
  // window of kLookback predecessors per round trip; tiles before the first
  // one read as an inclusive prefix of zero.
  if (tid < kRadix) {
    uint32_t exclusive = 0u;
    if (tile != 0u && agent_scan) {
      // The agent publishes the predecessor's inclusive prefix.
      uint32_t st = window[0];
      while ((st & kFlagMask) != kFlagG) {
        __builtin_amdgcn_s_sleep(1);
        st = load_status(&a.status[static_cast<size_t>(tile - 1u) * kRadix + tid]);
      }
      exclusive = st & kValueMask;
    } else if (tile != 0u) {
      int pred = static_cast<int>(tile) - 1;
      while (true) {
        bool found = false, stalled = false;
        int consumed = 0;
#pragma unroll
        for (int w = 0; w < kLookback; ++w) {
          if (!found && !stalled) {
            const uint32_t st = window[w];
            const uint32_t flag = st & kFlagMask;
            if (flag == 0u) {
              stalled = true;
            } else {
              exclusive += st & kValueMask;
              ++consumed;
              found = flag == kFlagG;
            }
          }
        }
        if (found) break;
        pred -= consumed;
        if (stalled) __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int w = 0; w < kLookback; ++w)
          window[w] = pred - w >= 0
                          ? load_status(&a.status[static_cast<size_t>(pred - w) * kRadix + tid])
                          : kFlagG;
      }
      store_status(&a.status[static_cast<size_t>(tile) * kRadix + tid],
                   kFlagG | (exclusive + published));
    }
    // Global position of the key at tile position q with digit v is
    // s_gbase[v] + q (unsigned wrap-around cancels in the sum).
    s_gbase[tid] = a.bin_offsets[tid] + exclusive - local_start;
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
      if (!kCheckedStores || g < n) dst[g] = k;
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
      if ((full || q < tile_count) && (!kCheckedStores || dst_idx[i] < n))
        vdst[dst_idx[i]] = s_vals[q];
    }
  }
}

// Instantiated shapes: (key type, values, workgroup size, items per thread,
// rank algorithm).
#define ONESWEEP_BINNING_SHAPES(X)    \
  X(uint32_t, false, 256, 16, 0)      \
  X(uint32_t, false, 512, 16, 0)      \
  X(uint32_t, false, 512, 12, 0)      \
  X(uint32_t, false, 1024, 8, 0)      \
  X(uint32_t, false, 256, 16, 1)      \
  X(uint32_t, false, 512, 16, 1)      \
  X(uint32_t, false, 512, 12, 1)      \
  X(uint32_t, false, 1024, 8, 1)      \
  X(uint32_t, true, 256, 16, 0)       \
  X(uint32_t, true, 512, 16, 0)       \
  X(uint32_t, true, 512, 12, 0)       \
  X(uint32_t, true, 1024, 8, 0)       \
  X(uint32_t, true, 256, 16, 1)       \
  X(uint32_t, true, 512, 16, 1)       \
  X(uint32_t, true, 512, 12, 1)       \
  X(uint32_t, true, 1024, 8, 1)       \
  X(uint64_t, false, 256, 16, 0)      \
  X(uint64_t, false, 512, 8, 0)       \
  X(uint64_t, false, 512, 12, 0)      \
  X(uint64_t, false, 1024, 8, 0)      \
  X(uint64_t, false, 256, 16, 1)      \
  X(uint64_t, false, 512, 8, 1)       \
  X(uint64_t, false, 512, 12, 1)      \
  X(uint64_t, false, 1024, 8, 1)      \
  X(uint64_t, true, 256, 16, 0)       \
  X(uint64_t, true, 512, 8, 0)        \
  X(uint64_t, true, 512, 12, 0)       \
  X(uint64_t, true, 1024, 8, 0)       \
  X(uint64_t, true, 256, 16, 1)       \
  X(uint64_t, true, 512, 8, 1)        \
  X(uint64_t, true, 512, 12, 1)       \
  X(uint64_t, true, 1024, 8, 1)

bool binning_shape_supported(const BinningShape &s) {
#define ONESWEEP_MATCH(K, V, B, I, R)                                                  \
  if (s.key_bits == 8 * (int)sizeof(K) && s.has_values == V && s.block == B && s.ipt == I && \
      s.rank == R)                                                                          \
    return true;
  ONESWEEP_BINNING_SHAPES(ONESWEEP_MATCH)
#undef ONESWEEP_MATCH
  return false;
}

BinningShape binning_default_shape(int key_bits, bool has_values) {
  if (key_bits == 64) return BinningShape{64, has_values, 512, 8, kRankPresence};
  return BinningShape{32, has_values, 512, 16, kRankPresence};
}

hipError_t launch_binning(const BinningShape &s, const void *args, uint32_t grid,
                          hipStream_t stream) {
#define ONESWEEP_LAUNCH(K, V, B, I, R)                                                       \
  if (s.key_bits == 8 * (int)sizeof(K) && s.has_values == V && s.block == B && s.ipt == I &&  \
      s.rank == R) {                                                                          \
    hipLaunchKernelGGL((binning_kernel<K, V, B, I, R>), dim3(grid), dim3(B), 0, stream,        \
                       *static_cast<const BinningArgs<K> *>(args));                           \
    return hipGetLastError();                                                                 \
  }
  ONESWEEP_BINNING_SHAPES(ONESWEEP_LAUNCH)
#undef ONESWEEP_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace onesweep
