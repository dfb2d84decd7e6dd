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
#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace onesweep {

// Two ways to find, for every lane of a wavefront, the lanes holding the
// same digit (its "peers"), which is all the multi-split needs:
//  - kRankBallot: one ballot per digit bit (the paper's match). A lane ORs
//    together each ballot XOR its own bit, which leaves the lanes holding
//    another digit; its peers are the other lanes. On gfx950 the OR-of-XOR
//    is one three-input bit operation per 32-lane half;
//  - kRankPresence: every lane ORs its lane bit into a 64-bit presence mask
//    per digit in LDS and reads the mask back. OR is order-independent, so
//    the mask is exact whatever order the LDS serves the lanes in, and it
//    costs a few instructions per batch instead of four per digit bit.
//  - kRankAtomic: the ballot match, but the lowest lane of each digit group
//    adds the group's size to the wave's LDS counter with an atomic that
//    returns the previous count, and the group reads it from that lane
//    afterwards. The batches' atomics do not wait on each other (a wave's
//    LDS instructions execute in program order, which keeps the counts
//    stable), so their latencies overlap instead of forming one chain of
//    read-then-write per batch.
enum RankAlgorithm : int { kRankBallot = 0, kRankPresence = 1, kRankAtomic = 2 };

// Every tile checks, once, that each digit's destination run lies inside the
// output (a look-back that gave up or inconsistent counts could place it
// elsewhere); a tile that fails writes nothing and sets bit 1 of the error
// word. With correct ranking that bounds every store. This switch adds a check
// of every single store index against n on top (debugging of the ranking).
#ifndef ONESWEEP_CHECKED_STORES
#define ONESWEEP_CHECKED_STORES 0
#endif
constexpr bool kCheckedStores = ONESWEEP_CHECKED_STORES != 0;

#ifndef ONESWEEP_LOOKBACK_WINDOW
#define ONESWEEP_LOOKBACK_WINDOW 4
#endif

// Predecessor tiles read per look-back round trip.
constexpr int kLookback = ONESWEEP_LOOKBACK_WINDOW;

// Tile positions of a thread's keys, two 16-bit positions per register (a
// tile holds at most 65536 keys). They live from the ranking to the last LDS
// regroup; packed, the 1024 x 11 tile fits 64 registers, where unpacked one
// key was spilled to scratch memory and reloaded right after a barrier, a
// memory round trip on every tile's critical path. A position is set once
// and then only grows by offsets that keep it below the tile size, so adding
// to either half never carries into the other.
template <int kN>
struct PackedPos {
  uint32_t w[(kN + 1) / 2];
  __device__ __forceinline__ void set(int i, uint32_t v) {
    if (i & 1) w[i >> 1] |= v << 16;
    else w[i >> 1] = v;
  }
  __device__ __forceinline__ void add(int i, uint32_t v) { w[i >> 1] += v << (16 * (i & 1)); }
  __device__ __forceinline__ uint32_t get(int i) const {
    return (i & 1) ? (w[i >> 1] >> 16) : (w[i >> 1] & 0xFFFFu);
  }
};

// Digit counts of one tile of a large segment, for every place at once, added
// to the segment's count rows with device-scope atomics (the counting half
// of a kBinSegCounted launch). kCopies interleaved LDS copies per counter, as
// in the upfront histogram.
constexpr int kSegCountCopies = 4;

template <typename K, bool kOrdered, int kBlock>
__device__ void count_segment_tile(const K *__restrict__ keys, const uint4 info,
                                   const SegmentTiles &seg, const KeyOrder &order,
                                   uint32_t *s_hist) {
  constexpr int kMaxP = kMaxPlaces;
  constexpr int kBatch = 8;  // independent loads in flight per thread
  const int tid = threadIdx.x;
  const int places = seg.places;
  int shifts[kMaxP];
  uint32_t masks[kMaxP];
#pragma unroll
  for (int j = 0; j < kMaxP; ++j) {
    const int lo = seg.begin_bit + j * seg.digit_bits;
    const int hi = lo + seg.digit_bits < seg.end_bit ? lo + seg.digit_bits : seg.end_bit;
    shifts[j] = j < places ? lo : 0;
    masks[j] = j < places ? ((1u << (hi - lo)) - 1u) : 0u;
  }
  for (int i = tid; i < places * kRadix * kSegCountCopies; i += kBlock) s_hist[i] = 0u;
  __syncthreads();
  uint32_t *my_hist = s_hist + (tid % kSegCountCopies);
  for (uint32_t base = 0; base < info.y; base += kBlock * kBatch) {
    K k[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const uint32_t i = base + b * kBlock + tid;
      k[b] = i < info.y ? keys[info.x + i] : K(0);
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (base + b * kBlock + tid >= info.y) continue;
      const K o = kOrdered ? ordered_bits(k[b], order) : k[b];
#pragma unroll
      for (int j = 0; j < kMaxP; ++j)
        if (j < places)
          atomicAdd(&my_hist[(j * kRadix + (static_cast<uint32_t>(o >> shifts[j]) & masks[j])) *
                             kSegCountCopies],
                    1u);
    }
  }
  __syncthreads();
  uint32_t *dst = seg.counts + static_cast<size_t>(info.w) * places * kRadix;
  for (int i = tid; i < places * kRadix; i += kBlock) {
    uint32_t c = 0u;
#pragma unroll
    for (int k = 0; k < kSegCountCopies; ++k) c += s_hist[i * kSegCountCopies + k];
    if (c != 0u) atomicAdd(&dst[i], c);
  }
}

// Occupancy target (waves per SIMD the register allocation must allow).
// 1024-thread workgroups always take 8 (64 registers): two of them per CU
// keep twice the keys in flight of one, which outweighs a few spilled
// registers (32-bit keys at 11 per thread spill 8 bytes and are the fastest
// shape at 2^28 keys; at occupancy 6 only one such workgroup fits a CU).
// Smaller workgroups: as high as the key registers permit without spilling.
template <typename K, int kBlock, int kIpt>
constexpr int binning_waves_per_eu() {
  return kBlock == 1024 || (kIpt * sizeof(K)) <= 32 ? 8 : ((kIpt * sizeof(K)) <= 48 ? 6 : 4);
}

// Element-indexed buffer stores: the memory unit forms the address from the
// base and the index times the element size, so a store takes one 32-bit
// index and no vector address arithmetic, and drops an index at or past the
// record count (the output's length). The unit's offset is 32 bits wide, so
// they serve outputs of at most 4 GiB. Word 3 of the resource: 32-bit data
// format, the value every gfx9-family buffer resource takes.
__device__ void buffer_store_i32(int32_t v, __amdgpu_buffer_rsrc_t r, int32_t index,
                                 int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.store.i32");
__device__ void buffer_store_i64(int64_t v, __amdgpu_buffer_rsrc_t r, int32_t index,
                                 int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.store.i64");
constexpr int kRsrcWord3 = 0x00020000;

// Stores of one output array: through an element-indexed buffer resource
// (kBuffered: outputs of at most 4 GiB), else plain stores (optionally
// checked). The choice is made per kernel: chosen per store, its scalar
// branches cost about 1% of a pass, and compiling the scatter twice in one
// kernel spills registers.
template <typename T, typename Idx, bool kBuffered>
struct ElementStore {
  T *base;
  Idx n;
  __amdgpu_buffer_rsrc_t rsrc;
  __device__ __forceinline__ ElementStore(T *p, Idx count) : base(p), n(count) {
    if constexpr (kBuffered)
      rsrc = __builtin_amdgcn_make_buffer_rsrc(p, static_cast<short>(sizeof(T)),
                                               static_cast<int>(count), kRsrcWord3);
  }
  __device__ __forceinline__ void put(Idx i, T v) const {
    if constexpr (kBuffered) {
      if constexpr (sizeof(T) == 4)
        buffer_store_i32(static_cast<int32_t>(v), rsrc, static_cast<int32_t>(i), 0, 0, 0);
      else
        buffer_store_i64(static_cast<int64_t>(v), rsrc, static_cast<int32_t>(i), 0, 0, 0);
    } else if (!kCheckedStores || i < n) {
      base[i] = v;
    }
  }
};

// kMode: kBinChained, one sequence with a chained scan over its tiles;
// kBinSegmented, the tiles of the large segments of a segmented sort (each
// segment its own chained scan; a tile turns its segment's digit counts of
// the place into bin starts itself); kBinSegCounted, the first place of the
// segmented sort in the same launch as the counting of every place (see
// count_segment_tile); kBinDownsweep, the scatter step of reduce-then-scan:
// every tile's exclusive prefix per digit is read from a table that the
// upsweep and tile-scan kernels filled beforehand.
// kOrdered: keys are ranked by their ordered bits (signed, floating-point or
// descending order); false for unsigned ascending sorts. Idx: type of element
// positions (uint64_t for sorts of 2^31 elements or more, or of more than
// 4 GiB of keys).
template <typename K, bool kVals, int kBlock, int kIpt, int kRank, int kMode, bool kOrdered,
          typename Idx>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(binning_waves_per_eu<K, kBlock, kIpt>())))
    binning_kernel(BinningArgs<K, Idx> a) {
  constexpr bool kCounted = kMode == kBinSegCounted;
  constexpr bool kSeg = kMode == kBinSegmented || kCounted;
  constexpr bool kRts = kMode == kBinDownsweep;
  constexpr int kWaves = kBlock / kWave;
  constexpr int kTile = kBlock * kIpt;
  constexpr int kWaveItems = kWave * kIpt;
  static_assert(kBlock >= kRadix, "one thread per digit takes part in the look-back");
  static_assert(kBlock % kWave == 0, "whole wavefronts");
  static_assert(kTile <= 65536, "tile positions are packed into 16 bits");

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
  // One-digit tiles skip the LDS regrouping and write keys and values from
  // registers. Built for 32-bit pairs only, where it is measured faster;
  // keys-only tiles gain nothing from it (the pass waits on memory, not on
  // LDS), and 64-bit pairs would spill holding their keys across the
  // look-back.
  constexpr bool kShortCircuit = sizeof(K) == 4 && kVals;
  // 64-bit keys regroup their two 32-bit halves one after the other through
  // a 4-byte-per-key buffer (values use the same buffer after them), so the
  // tile needs half the LDS and 1024 x 14 tiles keep two workgroups per CU
  // (1024 x 9 at most with 8 bytes per key): 2^27 keys, 548 -> 513 us per
  // pass, 2^27 pairs 822 -> 774 us; the second round trip costs nothing
  // measurable at equal tiles (548 against 547 us at 1024 x 9).
  constexpr bool kSplit = sizeof(K) == 8;
  // Buffer stores: kernels with 32-bit positions, whose outputs the host
  // keeps within 4 GiB (larger sorts take 64-bit positions); the segmented
  // 64-bit kernels, whose keys may pass 4 GiB, store plainly.
  constexpr bool kBuffered = sizeof(Idx) == 4 && !(kSeg && sizeof(K) == 8);
  constexpr size_t kKeyBytes = (kSplit ? 4 : sizeof(K)) * kTile;
  constexpr size_t kRankBytes = sizeof(uint32_t) * kWaves * kRadix * kEntryWords;
  constexpr size_t kTileBytes = kKeyBytes > kRankBytes ? kKeyBytes : kRankBytes;
  constexpr size_t kCountBytes =
      kCounted ? sizeof(uint32_t) * kMaxPlaces * kRadix * kSegCountCopies : 0;
  constexpr size_t kStageBytes = kTileBytes > kCountBytes ? kTileBytes : kCountBytes;
  __shared__ __attribute__((aligned(16))) unsigned char s_stage[kStageBytes];
  __shared__ Idx s_gbase[kRadix];
  __shared__ uint32_t s_wave_sum[kRadix / kWave];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_uniform;  // 1 + the tile's only digit, or 0
  __shared__ uint32_t s_outside;  // 1: a destination run leaves the output
  __shared__ uint32_t s_seg_sum[kRadix / kWave];  // segmented: digit counts per wave

  uint32_t *s_rank = reinterpret_cast<uint32_t *>(s_stage);
  K *s_keys = reinterpret_cast<K *>(s_stage);
  uint32_t *s_vals = reinterpret_cast<uint32_t *>(s_stage);

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int shift = a.shift;
  const int width = a.width;
  const uint32_t mask = (1u << width) - 1u;
  const Idx n = a.n;
  // 32-bit keys: one bit-field extract (the shift and width are uniform; the
  // compiler keeps one of them in a vector register for the whole tile).
  auto digit = [&](K k) -> uint32_t {
    const K t = kOrdered ? ordered_bits(k, a.order) : k;
    if constexpr (sizeof(K) == 4)
      return __builtin_amdgcn_ubfe(static_cast<uint32_t>(t), static_cast<uint32_t>(shift),
                                   static_cast<uint32_t>(width));
    else
      return digit_of(t, shift, mask);
  };

  // The segmented grid is sized for the most tiles the offsets could need;
  // workgroups beyond the actual count leave before taking a tile id, so the
  // ids handed out are exactly 0 .. tiles - 1 (twice that in a counted
  // launch: first the counting of every tile, then the binning of every tile).
  if constexpr (kSeg) {
    const uint32_t items = (kCounted ? 2u : 1u) * a.seg.plan->large_tiles;
    if (a.seg.plan->error || blockIdx.x >= items) return;
  }
  {
    uint4 *z = reinterpret_cast<uint4 *>(s_rank);
    for (int i = tid; i < static_cast<int>(kRankBytes / 16); i += kBlock)
      z[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (tid == 0) {
    // Tiles in the order workgroups start, in every mode: workgroups are
    // spread over the XCDs out of block-index order, and a downsweep that
    // used block indices (it needs no ordering) scatters 15-50% slower, its
    // concurrent tiles writing far-apart parts of each bin.
    s_tile = atomicAdd(a.tile_counter, 1u);
    s_uniform = 0u;
    s_outside = 0u;
  }
  __syncthreads();
  uint32_t tile = s_tile + a.tile_first;  // tickets count from the strip's start
  if constexpr (kCounted) {
    // Tickets below the tile count are counting work. Every binning tile's
    // ticket is larger than every counting ticket, so a binning tile only
    // waits on counting that workgroups already running have taken on.
    const uint32_t large_tiles = a.seg.plan->large_tiles;
    if (tile < large_tiles) {
      count_segment_tile<K, kOrdered, kBlock>(src, a.seg.tile_info[tile], a.seg, a.order,
                                              reinterpret_cast<uint32_t *>(s_stage));
      return;
    }
    tile -= large_tiles;
  }
  Idx tile_base, bin_base;
  uint32_t tile_count;
  bool first;
  uint4 seg_info = make_uint4(0u, 0u, 0u, 0u);
  if constexpr (kSeg) {
    seg_info = a.seg.tile_info[tile];
    tile_base = seg_info.x;
    tile_count = seg_info.y;
    bin_base = seg_info.z;
    first = seg_info.x == seg_info.z;
  } else {
    tile_base = static_cast<Idx>(tile) * static_cast<Idx>(kTile);
    const Idx left = n - tile_base;
    tile_count = left < static_cast<Idx>(kTile) ? static_cast<uint32_t>(left) : kTile;
    bin_base = 0u;
    first = tile == a.tile_first;
  }
  const Idx tile_end = tile_base + tile_count;
  const bool full = tile_count == static_cast<uint32_t>(kTile);

  // The bin starts of this place, loaded before the keys so that waiting for
  // them does not wait for the keys; kept in s_gbase until the look-back.
  // A segment's tile derives them from the segment's digit counts of the
  // place (seg_count, loaded here): after the key loads are issued, threads
  // 0..255 scan the counts within their wave, and each adds the lower waves'
  // totals (s_seg_sum) at the look-back.
  Idx bin_start_load = 0u;
  uint32_t seg_count = 0u;
  const uint32_t *seg_counts = nullptr;
  if constexpr (kSeg) {
    seg_counts =
        a.seg.counts + (static_cast<size_t>(seg_info.w) * a.seg.places + a.place) * kRadix;
    if constexpr (!kCounted)
      if (tid < kRadix) seg_count = seg_counts[tid];
  } else if (tid < kRadix) {
    bin_start_load = a.bin_offsets[tid];
  }
  // Segmented tiles: turn the counts into this thread's exclusive digit sum
  // within its wave. In the launch that also counts, first wait for the
  // counts: they only grow and their final values add up to the segment's
  // length, so a read of all 256 that adds up to the length has read every
  // final value (no ordering between the counters is needed, only each
  // counter's own).
  auto segment_bin_starts = [&]() {
    if constexpr (kCounted) {
      const uint32_t len = a.seg.large_len[seg_info.w];
      uint32_t rounds = 0u;
      while (true) {
        if (tid < kRadix)
          seg_count = __hip_atomic_load(const_cast<uint32_t *>(seg_counts + tid),
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t sum = tid < kRadix ? seg_count : 0u;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kWave);
        if (tid < kRadix && lane == 0) s_seg_sum[wave] = sum;
        __syncthreads();
        uint32_t total = 0u;
#pragma unroll
        for (int w = 0; w < kRadix / kWave; ++w) total += s_seg_sum[w];
        __syncthreads();
        if (total == len) break;
        if (++rounds >= a.spin_limit) {  // bounded wait: give up, record it
          if (tid == 0)
            __hip_atomic_fetch_or(a.lookback_error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    if (tid < kRadix) {
      uint32_t incl = seg_count;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += t;
      }
      if (lane == kWave - 1) s_seg_sum[wave] = incl;
      bin_start_load = incl - seg_count;
    }
  };

  // 1. Load. For ranking, a lane past the end of a ragged tile holds the key
  // whose ordered bits are all ones: its digit is the largest the place can
  // hold and it ranks after every real key, so the padding occupies the last
  // tile positions, which are never written out. Loading and ranking are
  // compiled twice: for a full tile (no bounds checks: one address and
  // immediate offsets) and for a ragged one. In a ragged keys-only tile the
  // loads are unconditional (lanes past the end load the tile's last key,
  // in bounds, and take the padding only when ranked), so no branch
  // separates the loads from the ranking and each batch waits only for its
  // own load; pairs load in two branches.
  K key[kIpt];
  const Idx wave_base = tile_base + static_cast<uint32_t>(wave * kWaveItems + lane);
  const K pad = kOrdered ? static_cast<K>(a.order.pad) : static_cast<K>(~K(0));
  PackedPos<kIpt> pos;
  const uint32_t wave_table = static_cast<uint32_t>(wave) * kRadix * kEntryWords;
  auto load_and_rank = [&](auto full_tag) {
    constexpr bool kFull = decltype(full_tag)::value;
    if constexpr (kFull) {
#pragma unroll
      for (int i = 0; i < kIpt; ++i) key[i] = src[wave_base + static_cast<uint32_t>(i * kWave)];
    } else if constexpr (kVals) {
#pragma unroll
      for (int i = 0; i < kIpt; ++i) {
        const Idx idx = wave_base + static_cast<uint32_t>(i * kWave);
        key[i] = idx < tile_end ? src[idx] : pad;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kIpt; ++i) {
        const Idx idx = wave_base + static_cast<uint32_t>(i * kWave);
        key[i] = src[idx < tile_end ? idx : tile_end - 1u];
      }
    }
    if constexpr (kSeg) segment_bin_starts();
    if (tid < kRadix) s_gbase[tid] = bin_base + bin_start_load;
    auto ranked = [&](int i) -> K {
      if constexpr (kFull) return key[i];
      else return wave_base + static_cast<uint32_t>(i * kWave) < tile_end ? key[i] : pad;
    };
    // 2. Wave64 multi-split ranking: pos[i] becomes the key's rank among the
    // wave's earlier keys with the same digit.
    if constexpr (kRank == kRankAtomic) {
      // Batch i's previous count is read back kDepth batches later, so only
      // kDepth (prior, leader) pairs are live at a time.
      constexpr int kDepth = kIpt < 3 ? kIpt : 3;
      uint32_t prior[kIpt], leader[kIpt];
#pragma unroll
      for (int i = 0; i < kIpt + kDepth; ++i) {
        if (i >= kDepth) {
          const int r = i - kDepth;
          pos.add(r, __shfl(prior[r], static_cast<int>(leader[r]), kWave));
        }
        if (i >= kIpt) continue;
        const uint32_t d = digit(ranked(i));
        uint32_t peers_lo = ~0u, peers_hi = ~0u;
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
          const int own = __builtin_amdgcn_sbfe(static_cast<int>(d), b, 1);  // 0 or -1
          const uint64_t vote = __builtin_amdgcn_ballot_w64(own != 0);
          peers_lo &= ~(static_cast<uint32_t>(vote) ^ static_cast<uint32_t>(own));
          peers_hi &= ~(static_cast<uint32_t>(vote >> 32) ^ static_cast<uint32_t>(own));
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(peers_hi, __builtin_amdgcn_mbcnt_lo(peers_lo, 0u));
        pos.set(i, below);
        leader[i] = peers_lo != 0u ? static_cast<uint32_t>(__builtin_ctz(peers_lo))
                                   : 32u + static_cast<uint32_t>(__builtin_ctz(peers_hi));
        prior[i] = 0u;
        if (below == 0u)
          prior[i] = atomicAdd(&s_rank[wave_table + d],
                               static_cast<uint32_t>(__popc(peers_lo) + __popc(peers_hi)));
      }
    } else {
#pragma unroll
      for (int i = 0; i < kIpt; ++i) {
        const uint32_t d = digit(ranked(i));
        const uint32_t e = wave_table + d * kEntryWords;
        // below: lanes under this one holding the same digit; group: all such
        // lanes of the batch.
        uint32_t below, group;
        if constexpr (kRank == kRankPresence) {
          uint64_t *presence = reinterpret_cast<uint64_t *>(s_rank + e + 2);
          __hip_atomic_fetch_or(presence, 1ull << lane, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_WORKGROUP);
          __builtin_amdgcn_wave_barrier();
          const uint32_t peers_lo = s_rank[e + 2];
          const uint32_t peers_hi = s_rank[e + 3];
          below = __builtin_amdgcn_mbcnt_hi(peers_hi, __builtin_amdgcn_mbcnt_lo(peers_lo, 0u));
          group = static_cast<uint32_t>(__popc(peers_lo) + __popc(peers_hi));
        } else {
          // The lanes whose digit differs from this lane's: per bit, the vote
          // XOR this lane's bit (all ones or zero), ORed in, one three-input
          // operation per 32-lane half (a | (b ^ c) is truth table 0xF6).
          uint32_t mis_lo = 0u, mis_hi = 0u;
#pragma unroll
          for (int b = 0; b < kRadixBits; ++b) {
            // Bits at or above the place width are 0 in every lane: the vote is
            // empty and adds nothing.
            uint32_t own = static_cast<uint32_t>(__builtin_amdgcn_sbfe(static_cast<int>(d), b, 1));
            asm volatile("" : "+v"(own));  // vote on the extracted bit: one compare
            const uint64_t vote = __builtin_amdgcn_ballot_w64(own != 0u);
            mis_lo = __builtin_amdgcn_bitop3_b32(mis_lo, static_cast<uint32_t>(vote), own, 0xF6);
            mis_hi = __builtin_amdgcn_bitop3_b32(mis_hi, static_cast<uint32_t>(vote >> 32), own, 0xF6);
          }
          below = static_cast<uint32_t>(lane) -
                  __builtin_amdgcn_mbcnt_hi(mis_hi, __builtin_amdgcn_mbcnt_lo(mis_lo, 0u));
          group = static_cast<uint32_t>(kWave - __popc(mis_lo) - __popc(mis_hi));
        }
        const uint32_t prior = s_rank[e];
        // Count the peers below this lane now: left to the scheduler, the count
        // sinks to after the last batch and keeps every batch's two lane masks
        // live, which spills keys to scratch memory.
        asm volatile("" : "+v"(below));
        pos.set(i, prior + below);
        // Every lane of the group stores the same new count (and clears the
        // presence mask), so the result does not depend on which store lands.
        const uint32_t next = prior + group;
        if constexpr (kRank == kRankPresence) {
          *reinterpret_cast<uint4 *>(s_rank + e) = make_uint4(next, 0u, 0u, 0u);
        } else {
          s_rank[e] = next;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
  };
  if (full) load_and_rank(std::true_type{});
  else load_and_rank(std::false_type{});
  __syncthreads();

  // 3. Per-digit sums: over waves (each wave's start inside its digit run)
  // and over digits (the run's start inside the tile).
  uint32_t total = 0u, local_start = 0u, published = 0u;
  if (tid < kRadix) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      uint32_t &c = s_rank[(w * kRadix + tid) * kEntryWords];
      const uint32_t v = c;
      c = total;
      total += v;
    }
    published = total;
    if (!full && static_cast<uint32_t>(tid) == mask) published -= kTile - tile_count;
    if (kShortCircuit && full && total == static_cast<uint32_t>(kTile))
      s_uniform = 1u + static_cast<uint32_t>(tid);
    // 4a. Publish this tile's count (a first tile's count is already its
    // prefix).
    if constexpr (!kRts)
      store_status(&a.status[static_cast<size_t>(tile) * kRadix + tid],
                   (first ? kFlagG : kFlagL) | published);
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
    for (int w = 0; w < kWaves; ++w) s_rank[(w * kRadix + tid) * kEntryWords] += local_start;
  }
  __syncthreads();
  if (full) {
#pragma unroll
    for (int i = 0; i < kIpt; ++i) pos.add(i, s_rank[wave_table + digit(key[i]) * kEntryWords]);
  } else {
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      const bool in = wave_base + static_cast<uint32_t>(i * kWave) < tile_end;
      pos.add(i, s_rank[wave_table + digit(in ? key[i] : pad) * kEntryWords]);
    }
  }
  __syncthreads();  // the rank tables are dead; the region now holds the tile
  const uint32_t uniform = kShortCircuit ? s_uniform : 0u;

  // 5a. Regroup the keys by digit in LDS (not needed when the tile has one
  // digit: its sorted order is its input order).
  // (Split keys: the low halves now, the high halves after the look-back.)
  uint32_t key_hi[kSplit ? kIpt : 1];
  uint32_t *s_half = reinterpret_cast<uint32_t *>(s_stage);
  if constexpr (kSplit) {
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      s_half[pos.get(i)] = static_cast<uint32_t>(key[i]);
      key_hi[i] = static_cast<uint32_t>(key[i] >> 32);
    }
  } else if (uniform == 0u) {
#pragma unroll
    for (int i = 0; i < kIpt; ++i) s_keys[pos.get(i)] = key[i];
  }

  // Values are loaded only once the keys have been written out: loaded
  // before the look-back they were held in registers across it and the key
  // scatter, which spilled (1024 x 16 pairs: 1173 -> 1086 us per pass at
  // 2^28 with the late loads; 64-bit pairs 854 -> 821 us at 2^27). The
  // segmented launch that also counts loads them early: its counting and
  // wait code leave the late loads spilling there (233 against 207 us at
  // 1024 x 16 on 20000 segments of 2^26 pairs).
  constexpr bool kLateVals = !kCounted;
  uint32_t val[kVals ? kIpt : 1];
  auto load_vals = [&]() {
    if constexpr (kVals) {
      const uint32_t *__restrict__ vsrc = a.vals[src_id];
#pragma unroll
      for (int i = 0; i < kIpt; ++i) {
        const Idx idx = wave_base + static_cast<uint32_t>(i * kWave);
        val[i] = (full || idx < tile_end) ? vsrc[idx] : 0u;
      }
    }
  };
  if constexpr (!kLateVals) load_vals();

  // 4b. Decoupled look-back: thread v sums the counts of earlier tiles for
  // digit v, walking backwards until it meets an inclusive prefix. Each round
  // trip reads a window of kLookback predecessors at once; tiles before the
  // first one read as an inclusive prefix of zero.
  if (tid < kRadix) {
    Idx bin_start = s_gbase[tid];
    if constexpr (kSeg)
      for (int w = 0; w < wave; ++w) bin_start += s_seg_sum[w];
    uint32_t exclusive = 0u;
    if constexpr (kRts) {
      // digit-major table of exclusive prefixes over tiles
      const uint32_t tiles = static_cast<uint32_t>((n + static_cast<Idx>(kTile) - 1u) / static_cast<Idx>(kTile));
      exclusive = a.status[static_cast<size_t>(tid) * tiles + tile];
    } else if (!first) {
      int pred = static_cast<int>(tile) - 1;
      const int chain_first = static_cast<int>(a.tile_first);  // 0 in a segmented sort
      uint32_t rounds = 0u;
      while (true) {
        uint32_t s[kLookback];
#pragma unroll
        for (int w = 0; w < kLookback; ++w)
          s[w] = pred - w >= chain_first
                     ? load_status(&a.status[static_cast<size_t>(pred - w) * kRadix + tid])
                     : kFlagG;
        bool found = false, stalled = false;
        int consumed = 0;
#pragma unroll
        for (int w = 0; w < kLookback; ++w) {
          if (!found && !stalled) {
            const uint32_t flag = s[w] & kFlagMask;
            if (flag == 0u) {
              stalled = true;
            } else {
              exclusive += s[w] & kValueMask;
              ++consumed;
              found = flag == kFlagG;
            }
          }
        }
        if (found) break;
        if (++rounds >= a.spin_limit) {  // bounded wait: give up, record it
          __hip_atomic_fetch_or(a.lookback_error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        pred -= consumed;
        if (stalled) __builtin_amdgcn_s_sleep(1);
      }
      store_status(&a.status[static_cast<size_t>(tile) * kRadix + tid],
                   kFlagG | (exclusive + published));
    }
    // Global position of the key at tile position q with digit v is
    // s_gbase[v] + q (unsigned wrap-around cancels in the sum). The run of
    // the tile's keys of digit v must lie in the output, and a correct run
    // never starts below the digit's tile position; a tile that fails either
    // writes nothing, as does every tile of a buffered kernel handed an
    // output over 4 GiB.
    const Idx run = bin_start + exclusive;
    const bool too_big = kBuffered && static_cast<uint64_t>(n) * sizeof(K) > (uint64_t{1} << 32);
    if (too_big || (published != 0u && (run < local_start || run > n || n - run < published))) {
      s_outside = 1u;
      __hip_atomic_fetch_or(a.lookback_error, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_gbase[tid] = run - local_start;
    // The strip's last tile hands the next strip its bin starts.
    if constexpr (kMode == kBinChained)
      if (a.next_bin_offsets != nullptr && tile + 1u == a.tile_first + gridDim.x)
        a.next_bin_offsets[tid] = bin_start + exclusive + published;
  }
  __syncthreads();
  if (s_outside != 0u) return;  // recorded above; nothing is written
  const ElementStore<K, Idx, kBuffered> out(dst, n);

  // 5b'. Short-circuit: every key of a one-digit tile goes to its bin at its
  // input position, straight from registers.
  if (uniform != 0u) {
    if constexpr (kLateVals) load_vals();
    const Idx g0 = s_gbase[uniform - 1u] + static_cast<uint32_t>(wave * kWaveItems + lane);
#pragma unroll
    for (int i = 0; i < kIpt; ++i) out.put(g0 + static_cast<uint32_t>(i * kWave), key[i]);
    if constexpr (kVals) {
      const ElementStore<uint32_t, Idx, kBuffered> vout(a.vals[dst_id], n);
#pragma unroll
      for (int i = 0; i < kIpt; ++i) vout.put(g0 + static_cast<uint32_t>(i * kWave), val[i]);
    }
    return;
  }

  // 5b. Write runs of keys to their bins. Full keys-only tiles read all their
  // keys and destinations from LDS before the first store, so the LDS
  // latencies overlap instead of alternating with the stores (pairs hold
  // their values in registers here and would spill).
  Idx dst_idx[kVals ? kIpt : 1];
  uint32_t lo_half[kSplit ? kIpt : 1];
  if constexpr (kSplit) {  // slot-order low halves, then the high halves
#pragma unroll
    for (int i = 0; i < kIpt; ++i) lo_half[i] = s_half[i * kBlock + tid];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kIpt; ++i) s_half[pos.get(i)] = key_hi[i];
    __syncthreads();
  }
  auto slot_key = [&](int i, uint32_t q) -> K {  // the key at tile position q
    if constexpr (kSplit)
      return static_cast<K>((static_cast<uint64_t>(s_half[q]) << 32) | lo_half[i]);
    else
      return s_keys[q];
  };
  if (!kVals && full) {
    K k[kIpt];
    Idx g[kIpt];
#pragma unroll
    for (int i = 0; i < kIpt; ++i) k[i] = slot_key(i, i * kBlock + tid);
#pragma unroll
    for (int i = 0; i < kIpt; ++i) g[i] = s_gbase[digit(k[i])] + static_cast<uint32_t>(i * kBlock + tid);
#pragma unroll
    for (int i = 0; i < kIpt; ++i) out.put(g[i], k[i]);
  } else {
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      const uint32_t q = i * kBlock + tid;
      if (full || q < tile_count) {
        const K k = slot_key(i, q);
        const Idx g = s_gbase[digit(k)] + q;
        out.put(g, k);
        if constexpr (kVals) dst_idx[i] = g;
      }
    }
  }

  // 5c. Values follow their keys through the same LDS positions.
  if constexpr (kVals) {
    const ElementStore<uint32_t, Idx, kBuffered> vout(a.vals[dst_id], n);
    if constexpr (kLateVals) load_vals();
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kIpt; ++i) s_vals[pos.get(i)] = val[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
      const uint32_t q = i * kBlock + tid;
      if (full || q < tile_count) vout.put(dst_idx[i], s_vals[q]);
    }
  }
}

// Instantiated shapes: (key type, values, workgroup size, items per thread,
// rank algorithm).
#define ONESWEEP_BINNING_SHAPES(X)    \
  X(uint64_t, false, 1024, 12, 0)     \
  X(uint64_t, false, 1024, 14, 0)     \
  X(uint64_t, false, 1024, 14, 1)     \
  X(uint64_t, false, 1024, 14, 2)     \
  X(uint64_t, true, 1024, 12, 0)      \
  X(uint64_t, true, 1024, 14, 0)      \
  X(uint32_t, false, 1024, 16, 0)     \
  X(uint32_t, false, 1024, 18, 0)     \
  X(uint32_t, false, 1024, 19, 0)     \
  X(uint32_t, false, 1024, 19, 1)     \
  X(uint32_t, false, 1024, 19, 2)     \
  X(uint32_t, true, 1024, 16, 0)      \
  X(uint32_t, true, 1024, 18, 0)      \
  X(uint32_t, true, 1024, 19, 0)      \
  X(uint32_t, true, 1024, 18, 1)      \
  X(uint32_t, true, 1024, 18, 2)      \
  X(uint32_t, false, 256, 8, 0)       \
  X(uint32_t, false, 256, 8, 1)       \
  X(uint32_t, true, 256, 8, 0)        \
  X(uint32_t, true, 256, 8, 1)        \
  X(uint64_t, false, 256, 8, 0)       \
  X(uint64_t, false, 256, 8, 1)       \
  X(uint64_t, true, 256, 8, 0)        \
  X(uint64_t, true, 256, 8, 1)        \
  X(uint32_t, false, 256, 16, 0)      \
  X(uint32_t, false, 512, 16, 0)      \
  X(uint32_t, false, 512, 12, 0)      \
  X(uint32_t, false, 1024, 8, 0)      \
  X(uint32_t, false, 1024, 10, 0)     \
  X(uint32_t, false, 1024, 11, 0)     \
  X(uint32_t, false, 1024, 10, 1)     \
  X(uint32_t, false, 1024, 11, 1)     \
  X(uint32_t, false, 1024, 10, 2)     \
  X(uint32_t, false, 1024, 11, 2)     \
  X(uint32_t, true, 1024, 10, 0)      \
  X(uint32_t, true, 1024, 11, 0)      \
  X(uint32_t, true, 1024, 10, 1)      \
  X(uint32_t, true, 1024, 11, 1)      \
  X(uint32_t, true, 1024, 10, 2)      \
  X(uint32_t, true, 1024, 11, 2)      \
  X(uint64_t, false, 1024, 9, 0)      \
  X(uint64_t, false, 1024, 9, 1)      \
  X(uint64_t, false, 1024, 9, 2)      \
  X(uint64_t, true, 1024, 9, 0)       \
  X(uint64_t, true, 1024, 9, 1)       \
  X(uint64_t, true, 1024, 9, 2)       \
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
  X(uint64_t, true, 1024, 8, 1)       \
  X(uint32_t, false, 256, 8, 2)       \
  X(uint32_t, false, 256, 16, 2)      \
  X(uint32_t, false, 512, 16, 2)      \
  X(uint32_t, false, 512, 12, 2)      \
  X(uint32_t, false, 1024, 8, 2)      \
  X(uint32_t, true, 256, 8, 2)        \
  X(uint32_t, true, 256, 16, 2)       \
  X(uint32_t, true, 512, 16, 2)       \
  X(uint32_t, true, 512, 12, 2)       \
  X(uint32_t, true, 1024, 8, 2)       \
  X(uint64_t, false, 256, 8, 2)       \
  X(uint64_t, false, 256, 16, 2)      \
  X(uint64_t, false, 512, 8, 2)       \
  X(uint64_t, false, 512, 12, 2)      \
  X(uint64_t, false, 1024, 8, 2)      \
  X(uint64_t, true, 256, 8, 2)        \
  X(uint64_t, true, 256, 16, 2)       \
  X(uint64_t, true, 512, 8, 2)        \
  X(uint64_t, true, 512, 12, 2)       \
  X(uint64_t, true, 1024, 8, 2)

// Shapes also built for the large segments of a segmented sort.
#define ONESWEEP_SEGMENT_BINNING_SHAPES(X) \
  X(uint32_t, false, 256, 8, 0)            \
  X(uint32_t, true, 256, 8, 0)             \
  X(uint64_t, false, 256, 8, 0)            \
  X(uint64_t, true, 256, 8, 0)             \
  X(uint32_t, false, 256, 16, 0)           \
  X(uint32_t, false, 512, 16, 0)           \
  X(uint32_t, false, 1024, 8, 0)           \
  X(uint32_t, true, 256, 16, 0)            \
  X(uint32_t, true, 512, 16, 0)            \
  X(uint32_t, true, 1024, 8, 0)            \
  X(uint64_t, false, 256, 16, 0)           \
  X(uint64_t, false, 512, 8, 0)            \
  X(uint64_t, false, 1024, 8, 0)           \
  X(uint64_t, true, 256, 16, 0)            \
  X(uint64_t, true, 512, 8, 0)             \
  X(uint64_t, true, 1024, 8, 0)            \
  X(uint32_t, false, 1024, 11, 0)          \
  X(uint32_t, true, 1024, 11, 0)           \
  X(uint32_t, false, 1024, 16, 0)          \
  X(uint32_t, true, 1024, 16, 0)           \
  X(uint32_t, false, 1024, 19, 0)          \
  X(uint32_t, true, 1024, 19, 0)           \
  X(uint64_t, false, 1024, 9, 0)           \
  X(uint64_t, true, 1024, 9, 0)            \
  X(uint64_t, false, 1024, 14, 0)          \
  X(uint64_t, true, 1024, 14, 0)

// Shapes built for the reduce-then-scan baseline (ballot ranking): the
// default shapes of every key width and value presence.
#define ONESWEEP_DOWNSWEEP_SHAPES(X) \
  X(uint64_t, false, 1024, 12, 0)    \
  X(uint64_t, false, 1024, 14, 0)    \
  X(uint64_t, true, 1024, 12, 0)     \
  X(uint64_t, true, 1024, 14, 0)     \
  X(uint32_t, false, 1024, 16, 0)    \
  X(uint32_t, true, 1024, 16, 0)     \
  X(uint32_t, false, 1024, 18, 0)    \
  X(uint32_t, false, 1024, 19, 0)    \
  X(uint32_t, true, 1024, 18, 0)     \
  X(uint32_t, true, 1024, 19, 0)     \
  X(uint32_t, false, 256, 8, 0)      \
  X(uint32_t, true, 256, 8, 0)       \
  X(uint32_t, false, 512, 16, 0)     \
  X(uint32_t, true, 512, 16, 0)      \
  X(uint32_t, false, 1024, 8, 0)     \
  X(uint32_t, true, 1024, 8, 0)      \
  X(uint32_t, false, 1024, 11, 0)    \
  X(uint32_t, true, 1024, 11, 0)     \
  X(uint64_t, false, 1024, 9, 0)     \
  X(uint64_t, true, 1024, 9, 0)      \
  X(uint64_t, false, 256, 8, 0)      \
  X(uint64_t, true, 256, 8, 0)       \
  X(uint64_t, false, 512, 8, 0)      \
  X(uint64_t, true, 512, 8, 0)       \
  X(uint64_t, false, 1024, 8, 0)     \
  X(uint64_t, true, 1024, 8, 0)

// Shapes built with 64-bit element positions for sorts of 2^31 elements or
// more: the default large-input shape of each key width and value presence.
#define ONESWEEP_WIDE_SHAPES(X)   \
  X(uint32_t, false, 1024, 19, 0) \
  X(uint32_t, true, 1024, 16, 0)  \
  X(uint32_t, true, 1024, 19, 0)  \
  X(uint64_t, false, 1024, 14, 0) \
  X(uint64_t, true, 1024, 14, 0)

#define ONESWEEP_SHAPE_IS(K, V, B, I, R) \
  (s.key_bits == 8 * (int)sizeof(K) && s.has_values == V && s.block == B && s.ipt == I && s.rank == R)

bool binning_shape_supported(const BinningShape &s, int mode, bool wide) {
#define ONESWEEP_MATCH(K, V, B, I, R) \
  if (ONESWEEP_SHAPE_IS(K, V, B, I, R)) return true;
  if (wide) {
    if (mode == kBinChained) {
      ONESWEEP_WIDE_SHAPES(ONESWEEP_MATCH)
    }
  } else if (mode == kBinSegmented || mode == kBinSegCounted) {
    ONESWEEP_SEGMENT_BINNING_SHAPES(ONESWEEP_MATCH)
  } else if (mode == kBinDownsweep) {
    ONESWEEP_DOWNSWEEP_SHAPES(ONESWEEP_MATCH)
  } else {
    ONESWEEP_BINNING_SHAPES(ONESWEEP_MATCH)
  }
#undef ONESWEEP_MATCH
  return false;
}

size_t binning_tile_items(const BinningShape &s) {
  return static_cast<size_t>(s.block) * static_cast<size_t>(s.ipt);
}

// The autotuned plain configuration: the fastest tile shape per key width,
// value presence and input size, measured on MI355X over uniform inputs of
// 2^18..2^28 keys, and over the seeded sweep of 2^17..2^28 keys of every
// distribution (500 inputs, every tile class timed). Small inputs want more,
// smaller tiles to fill 256 CUs; larger ones the largest tile that two
// 1024-thread workgroups per CU hold without spilling, since a larger tile
// spreads the look-back and the workgroup's fixed work over more keys.
// 32-bit keys (ms per sort): 1024 x 16 from 3 * 2^20 (2^22: 0.107 against
// 0.119 with 1024 x 11; the sweep's best between 2^21 and 2^22 was
// 1024 x 16 or 1024 x 11, 4% faster than 1024 x 11 alone), 1024 x 19 from
// 2^23 (2^28: 2.45 against 2.58 with 1024 x 16 and 2.95 with 1024 x 11).
// 32-bit pairs: 1024 x 11 from 2^21 (the sweep: 8% faster than 1024 x 8
// between 2^21 and 2^22), 1024 x 16 from 2^22 (2^24: 0.329 against 0.332
// with 1024 x 19), 1024 x 19 from 2^26 (2^26: 1.150 against 1.171 with
// 1024 x 16; 2^28: 4.53 against 4.61; it fits 64 registers since the stores
// go through buffer resources). 64-bit keys and pairs,
// regrouped in two 32-bit halves: 1024 x 9 from 2^21 (64-bit pairs: 1-2%
// faster than 1024 x 8 in the seeded sweep), 1024 x 12 from 2^22 and
// 1024 x 14 from 2^26 (2^27 keys: 4.36 ms against 4.41 with 1024 x 12 and
// 4.66 with 1024 x 9; a 2^27-pair pass 774 us against 784 and 822).
BinningShape binning_default_shape(int key_bits, bool has_values, size_t n) {
  if (key_bits == 64) {
    if (has_values && n < (size_t(3) << 16)) return BinningShape{64, true, 256, 8, kRankBallot};
    if (n < (size_t(1) << 19)) return BinningShape{64, has_values, 512, 8, kRankBallot};
    if (n >= (size_t(1) << 26)) return BinningShape{64, has_values, 1024, 14, kRankBallot};
    if (n >= (size_t(1) << 22)) return BinningShape{64, has_values, 1024, 12, kRankBallot};
    if (n >= (size_t(1) << 21)) return BinningShape{64, has_values, 1024, 9, kRankBallot};
    return BinningShape{64, has_values, 1024, 8, kRankBallot};
  }
  if (n < (size_t(1) << 18)) return BinningShape{32, has_values, 256, 8, kRankBallot};
  if (n < (size_t(1) << 21)) return BinningShape{32, has_values, 1024, 8, kRankBallot};
  if (has_values) {
    if (n < (size_t(1) << 22)) return BinningShape{32, true, 1024, 11, kRankBallot};
    if (n < (size_t(1) << 26)) return BinningShape{32, true, 1024, 16, kRankBallot};
    return BinningShape{32, true, 1024, 19, kRankBallot};
  }
  if (n < (size_t(3) << 20)) return BinningShape{32, false, 1024, 11, kRankBallot};
  if (n < (size_t(1) << 23)) return BinningShape{32, false, 1024, 16, kRankBallot};
  return BinningShape{32, false, 1024, 19, kRankBallot};
}

// The default tile shape of the segmented sort's large segments, measured on
// MI355X with the batched workload (20000 log-normal segments, 2^26 keys,
// eager, two streams; ms per sort): 32-bit keys 512 x 16 (0.79, against
// 0.79 with 1024 x 16, 0.82 with 1024 x 11 and 0.96 with 256 x 16), 32-bit
// pairs 1024 x 16 (1.01, against 1.06 with 1024 x 11 and 1.13 with
// 512 x 16; 1.09 against 1.17 under graph replay), 64-bit keys and pairs
// 1024 x 14 with their keys regrouped in two halves (keys 1.86 against 1.90
// with 1024 x 9 and 2.25 with 1024 x 8; pairs 2.50 against 2.61 with
// 1024 x 9 and 3.09 with 1024 x 8).
BinningShape segment_default_shape(int key_bits, bool has_values) {
  if (key_bits == 64) return BinningShape{64, has_values, 1024, 14, kRankBallot};
  return has_values ? BinningShape{32, true, 1024, 16, kRankBallot}
                    : BinningShape{32, false, 512, 16, kRankBallot};
}

hipError_t launch_binning(const BinningShape &s, int mode, const void *args, uint32_t grid,
                          hipStream_t stream, bool wide) {
#define ONESWEEP_LAUNCH_IDX(K, V, B, I, R, MODE, IDX)                                       \
  if (ONESWEEP_SHAPE_IS(K, V, B, I, R)) {                                                    \
    const BinningArgs<K, IDX> &a = *static_cast<const BinningArgs<K, IDX> *>(args);          \
    if (key_order_is_plain(a.order))                                                         \
      hipLaunchKernelGGL((binning_kernel<K, V, B, I, R, MODE, false, IDX>), dim3(grid), dim3(B), \
                         0, stream, a);                                                      \
    else                                                                                     \
      hipLaunchKernelGGL((binning_kernel<K, V, B, I, R, MODE, true, IDX>), dim3(grid), dim3(B), \
                         0, stream, a);                                                      \
    return hipGetLastError();                                                                \
  }
#define ONESWEEP_LAUNCH(K, V, B, I, R, MODE) ONESWEEP_LAUNCH_IDX(K, V, B, I, R, MODE, uint32_t)
#define ONESWEEP_LAUNCH_FLAT(K, V, B, I, R) ONESWEEP_LAUNCH(K, V, B, I, R, kBinChained)
#define ONESWEEP_LAUNCH_SEG(K, V, B, I, R) ONESWEEP_LAUNCH(K, V, B, I, R, kBinSegmented)
#define ONESWEEP_LAUNCH_SEGC(K, V, B, I, R) ONESWEEP_LAUNCH(K, V, B, I, R, kBinSegCounted)
#define ONESWEEP_LAUNCH_DOWN(K, V, B, I, R) ONESWEEP_LAUNCH(K, V, B, I, R, kBinDownsweep)
#define ONESWEEP_LAUNCH_WIDE(K, V, B, I, R) \
  ONESWEEP_LAUNCH_IDX(K, V, B, I, R, kBinChained, uint64_t)
  if (wide) {
    if (mode == kBinChained) {
      ONESWEEP_WIDE_SHAPES(ONESWEEP_LAUNCH_WIDE)
    }
  } else if (mode == kBinSegmented) {
    ONESWEEP_SEGMENT_BINNING_SHAPES(ONESWEEP_LAUNCH_SEG)
  } else if (mode == kBinSegCounted) {
    ONESWEEP_SEGMENT_BINNING_SHAPES(ONESWEEP_LAUNCH_SEGC)
  } else if (mode == kBinDownsweep) {
    ONESWEEP_DOWNSWEEP_SHAPES(ONESWEEP_LAUNCH_DOWN)
  } else {
    ONESWEEP_BINNING_SHAPES(ONESWEEP_LAUNCH_FLAT)
  }
#undef ONESWEEP_LAUNCH_WIDE
#undef ONESWEEP_LAUNCH_DOWN
#undef ONESWEEP_LAUNCH_SEGC
#undef ONESWEEP_LAUNCH_SEG
#undef ONESWEEP_LAUNCH_FLAT
#undef ONESWEEP_LAUNCH
#undef ONESWEEP_LAUNCH_IDX
  return hipErrorInvalidValue;
}

}  // namespace onesweep
