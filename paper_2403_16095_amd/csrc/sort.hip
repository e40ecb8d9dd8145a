// Depth order within each 16x16 tile -- the pre-sort of Sec. 3.1 -- as a
// segmented sort: the projection dropped every (depth | record) key into its
// tile's fixed-size bucket at an atomic slot, so one workgroup per tile now
// sorts its own bucket.
//
// Keys are depth bits << 32 | record id, unique within a tile, so the result
// is the order of (depth, record id) -- a stable depth sort of the records --
// whatever order the atomics left.  A segment of at most one key per thread
// is ranked directly (each thread counts the keys below its own, reading the
// segment from LDS by broadcast: one barrier instead of a network of them);
// segments up to kLdsKeys are sorted in LDS with a bitonic network; longer
// ones are sorted in LDS-sized chunks, merged pairwise in global memory by the
// same workgroup (merge path by binary search), ping-ponging between the two
// key buffers.
#include <algorithm>

#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kThreads = 256;
constexpr int kLdsKeys = 4096;   // 32 KB of 64-bit keys

__device__ __forceinline__ uint32_t next_pow2(uint32_t x) { return x <= 1 ? 1u : 1u << (32 - __builtin_clz(x - 1)); }

// LDS slot of key x in the bitonic sort: its low five bits XORed with the
// next five.  A compare-exchange stage of distance j has lane i read keys
// lo = 2j (i / j) + i % j and lo + j, which for j < 32 land a wave's lanes on
// the same banks several times over (SQ_LDS_BANK_CONFLICT counted 0.66
// conflict cycles per LDS instruction at the mapping size).  The swizzle is a
// permutation of every aligned block of 64 keys that puts each stage's 64
// lanes on distinct bank pairs (enumerated for 32 and 64 banks of 4 bytes and
// 512 to 4096 keys) and keeps the array dense.
__device__ __forceinline__ uint32_t swz(uint32_t x) { return x ^ ((x >> 1) & 31u); }

// Bitonic sort of s[0, p) ascending (slots swizzled by swz), p a power of
// two; all threads call it.
__device__ void bitonic_lds(uint64_t* s, uint32_t p) {
  for (uint32_t k = 2; k <= p; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < p / 2; i += kThreads) {
        const uint32_t lo = 2 * j * (i / j) + (i % j);
        const uint32_t hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint64_t a = s[swz(lo)], b = s[swz(hi)];
        if ((a > b) == up) {
          s[swz(lo)] = b;
          s[swz(hi)] = a;
        }
      }
      __syncthreads();
    }
  }
}

// Number of keys in sorted run r[0, n) that are smaller than key.
__device__ __forceinline__ uint32_t count_less(const uint64_t* r, uint32_t n, uint64_t key) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (r[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kThreads) void segment_sort_kernel(SegSortBufs b) {
  __shared__ uint64_t s[kLdsKeys];
  __shared__ uint32_t s_n;
  const uint32_t t = blockIdx.x;
  const uint64_t base = (uint64_t)t * b.cap;
  if (threadIdx.x == 0) {
    const uint32_t cnt = b.tile_count[(size_t)t * kTileCounterStride];
    const uint32_t n = min(cnt, b.cap);   // beyond the bucket only after an overflow, which is reported
    s_n = n;
    b.ranges[t] = make_uint2((uint32_t)base, (uint32_t)(base + n));
    b.tile_count[(size_t)t * kTileCounterStride] = 0u;   // reset the count for the next render
    if (t == 0) b.counters[kCntRenderPeak] = 0u;
  }
  __syncthreads();
  const uint32_t n = s_n;
  if (n == 0) return;
  uint64_t* keys = b.keys[0] + base;
  if (n <= (uint32_t)kThreads) {
    const bool mine = threadIdx.x < n;
    const uint64_t key = mine ? keys[threadIdx.x] : 0ull;
    if (mine) s[threadIdx.x] = key;
    __syncthreads();
    if (mine) {
      uint32_t rank = 0;
      for (uint32_t i = 0; i < n; ++i) rank += s[i] < key ? 1u : 0u;   // keys are unique
      b.sorted_vals[base + rank] = (uint32_t)key;
    }
    return;
  }
  if (n <= (uint32_t)kLdsKeys) {
    const uint32_t p = next_pow2(n);
    for (uint32_t i = threadIdx.x; i < p; i += kThreads) s[swz(i)] = i < n ? keys[i] : ~0ull;
    __syncthreads();
    bitonic_lds(s, p);
    for (uint32_t i = threadIdx.x; i < n; i += kThreads) b.sorted_vals[base + i] = (uint32_t)s[swz(i)];
    return;
  }
  // Long segment: sort chunks in LDS, write them back, then merge runs.
  for (uint32_t c0 = 0; c0 < n; c0 += kLdsKeys) {
    const uint32_t cn = min((uint32_t)kLdsKeys, n - c0);
    const uint32_t p = next_pow2(cn);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < p; i += kThreads) s[swz(i)] = i < cn ? keys[c0 + i] : ~0ull;
    __syncthreads();
    bitonic_lds(s, p);
    for (uint32_t i = threadIdx.x; i < cn; i += kThreads) keys[c0 + i] = s[swz(i)];
  }
  __syncthreads();
  uint64_t* src = keys;
  uint64_t* dst = b.keys[1] + base;
  for (uint32_t w = kLdsKeys; w < n; w <<= 1) {
    for (uint32_t i = threadIdx.x; i < n; i += kThreads) {
      const uint32_t run = i / (2 * w);
      const uint32_t a0 = run * 2 * w;
      const uint32_t b0 = min(n, a0 + w), b1 = min(n, a0 + 2 * w);
      const uint64_t key = src[i];
      uint32_t pos;
      if (i < b0) pos = a0 + (i - a0) + count_less(src + b0, b1 - b0, key);
      else pos = a0 + (i - b0) + count_less(src + a0, b0 - a0, key);
      dst[pos] = key;
    }
    __syncthreads();
    uint64_t* tmp = src;
    src = dst;
    dst = tmp;
  }
  for (uint32_t i = threadIdx.x; i < n; i += kThreads) b.sorted_vals[base + i] = (uint32_t)src[i];
}

__global__ __launch_bounds__(kThreads) void clear_kernel(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) p[i] = 0u;
}

// Longest-first order of the tiles for the blends: a launch with more tiles
// than fit the chip at once then starts the long ones in its first round and
// ends on short ones, instead of ending on whichever long tiles come last in
// raster order.  One workgroup, a counting sort on bins of the list length:
// 16 bins per octave (the leading bit and the next four), scanned from the
// longest bin; tiles inside a bin keep the order their atomics left, which
// changes no tile's result.
// snake (for launches whose tiles are all resident from the start): every
// other run of kOrderRound positions is reversed, so that the workgroups
// dealt one per CU take, CU by CU, a long tile of one run with a short one
// of the next, and the last, short run gives its tiles to the CU positions
// the full runs loaded least; the CUs' summed work comes out more even (a
// model of the dispatch over measured tracking lists: the fullest CU 1.16x
// the mean work longest first, 1.10x with the runs reversed, 1.06x with the
// last run placed by load).  A tile's length is then the work its four waves
// measured in the previous step (words 1..4 of its counter line; counts
// points at word 1), and each entry also takes a quadrant rotation in its top
// two bits.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBins = 16 * 33;
constexpr uint32_t kOrderRound = 256;   // compute units of the chip
constexpr int kSnakeMaxTiles = 2048;

__device__ __forceinline__ uint32_t order_bin(uint32_t n) {
  if (n == 0) return 0;
  const uint32_t lz = __builtin_clz(n);                  // leading bit at 31 - lz
  const uint32_t frac = lz <= 27 ? (n >> (27 - lz)) & 15u : (n << (lz - 27)) & 15u;   // the next four bits
  return 1u + 16u * (31u - lz) + frac;
}

// A tile's list length: from its range after the sort, or (ranges null) from
// its pair counter before a blend that sorts its own bucket, or (quads) the
// sum of the four quadrants' work.  The bin counts and the ranks must both
// come from this one function, or ranks collide and positions go unwritten.
__device__ __forceinline__ uint32_t tile_length(const uint2* ranges, const uint32_t* counts, int t, bool quads) {
  if (ranges) {
    const uint2 r = ranges[t];
    return r.y - r.x;
  }
  const uint32_t* c = counts + (size_t)t * kTileCounterStride;
  return quads ? c[0] + c[1] + c[2] + c[3] : c[0];
}

__global__ __launch_bounds__(kOrderThreads) void tile_order_kernel(const uint2* __restrict__ ranges,
                                                                   const uint32_t* __restrict__ counts, int32_t tiles,
                                                                   uint32_t* __restrict__ order, int snake) {
  __shared__ uint32_t s_bin[kOrderBins];
  __shared__ uint32_t s_wave[kOrderThreads / kWave];
  for (int i = threadIdx.x; i < kOrderBins; i += kOrderThreads) s_bin[i] = 0u;
  __syncthreads();
  for (int t = threadIdx.x; t < tiles; t += kOrderThreads)
    atomicAdd(&s_bin[order_bin(tile_length(ranges, counts, t, snake))], 1u);
  __syncthreads();
  // exclusive offsets, the longest bin first: thread k takes bin
  // kOrderBins - 1 - k (kOrderBins <= kOrderThreads)
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int bin = kOrderBins - 1 - (int)threadIdx.x;
  const uint32_t c = bin >= 0 ? s_bin[bin] : 0u;
  uint32_t inc = c;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d);
    if (lane >= d) inc += y;
  }
  if (lane == kWave - 1) s_wave[wv] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int q = 0; q < wv; ++q) base += s_wave[q];
  if (bin >= 0) s_bin[bin] = base + inc - c;
  __syncthreads();
  if (!snake) {
    for (int t = threadIdx.x; t < tiles; t += kOrderThreads)
      order[atomicAdd(&s_bin[order_bin(tile_length(ranges, counts, t, false))], 1u)] = (uint32_t)t;
    return;
  }
  // snake (tiles <= kSnakeMaxTiles): the full runs of kOrderRound positions
  // alternate direction; the last, short run's tiles (the shortest, longest
  // of them first) go to its positions in ascending order of the work the
  // full runs gave the same CU position.
  __shared__ uint32_t s_load[kOrderRound], s_perm[kOrderRound], s_ord[kSnakeMaxTiles];
  if (threadIdx.x < kOrderRound) s_load[threadIdx.x] = 0u;
  constexpr int kPer = kSnakeMaxTiles / kOrderThreads;
  uint32_t rank[kPer], len[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int t = threadIdx.x + q * kOrderThreads;
    len[q] = t < tiles ? tile_length(ranges, counts, t, true) : 0u;
    rank[q] = t < tiles ? atomicAdd(&s_bin[order_bin(len[q])], 1u) : 0u;
  }
  const uint32_t full = (uint32_t)tiles / kOrderRound * kOrderRound, rem = (uint32_t)tiles - full;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int t = threadIdx.x + q * kOrderThreads;
    if (t < tiles && rank[q] < full) {
      const uint32_t run = rank[q] / kOrderRound, j = rank[q] % kOrderRound;
      const uint32_t pos = (run & 1u) ? run * kOrderRound + kOrderRound - 1u - j : rank[q];
      s_ord[pos] = (uint32_t)t;
      atomicAdd(&s_load[pos % kOrderRound], len[q]);
    }
  }
  __syncthreads();
  if (threadIdx.x < rem) {   // rank of the position by (load, position)
    const uint32_t j = threadIdx.x, key = s_load[j];
    uint32_t r = 0;
    for (uint32_t i = 0; i < rem; ++i) r += (s_load[i] < key || (s_load[i] == key && i < j)) ? 1u : 0u;
    s_perm[r] = j;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int t = threadIdx.x + q * kOrderThreads;
    if (t < tiles && rank[q] >= full) s_ord[full + s_perm[rank[q] - full]] = (uint32_t)t;
  }
  __syncthreads();
  // The workgroups at positions c, c + 256, ... run on one CU, the r-th of
  // them with its waves on that CU's SIMDs in the order kSimdOf[(w + r) & 3]
  // (the dispatcher's rule, up to a renaming of the SIMDs).  Each CU's
  // workgroups in turn take the quadrant rotation that keeps its busiest
  // SIMD least busy.
  constexpr uint32_t kSimdOf[4] = {0, 2, 1, 3};
  if (threadIdx.x < kOrderRound) {
    uint32_t load[4] = {0u, 0u, 0u, 0u};
    uint32_t r = 0;
    for (uint32_t p = threadIdx.x; p < (uint32_t)tiles; p += kOrderRound, ++r) {
      const uint32_t t = s_ord[p];
      uint32_t qw[4];
      for (int k = 0; k < 4; ++k) qw[k] = counts[(size_t)t * kTileCounterStride + k];
      uint32_t best = 0xFFFFFFFFu, pick = 0;
      for (uint32_t rr = 0; rr < 4; ++rr) {
        uint32_t trial[4] = {load[0], load[1], load[2], load[3]};
        for (uint32_t w = 0; w < 4; ++w) trial[kSimdOf[(w + r) & 3]] += qw[(w + rr) & 3];
        const uint32_t m = max(max(trial[0], trial[1]), max(trial[2], trial[3]));
        if (m < best) {
          best = m;
          pick = rr;
        }
      }
      for (uint32_t w = 0; w < 4; ++w) load[kSimdOf[(w + r) & 3]] += qw[(w + pick) & 3];
      order[p] = t | (pick << 30);
    }
  }
}

__global__ __launch_bounds__(kThreads) void restore_counts_kernel(uint32_t* tile_count, const uint2* ranges,
                                                                  int32_t tiles) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t < tiles) {
    const uint2 r = ranges[t];
    tile_count[(size_t)t * kTileCounterStride] = r.y - r.x;
  }
}

}  // namespace

void launch_clear_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>(1024, (n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(clear_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, p, n);
}

void launch_tile_order(const uint2* ranges, const uint32_t* counts, int32_t tiles, uint32_t* order, hipStream_t s,
                       bool snake) {
  if (tiles <= 0) return;
  static_assert(kOrderBins <= kOrderThreads, "one bin per thread in the scan");
  hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(kOrderThreads), 0, s, ranges, counts, tiles, order,
                     snake && tiles <= kSnakeMaxTiles ? 1 : 0);
}

void launch_restore_counts(uint32_t* tile_count, const uint2* ranges, int32_t tiles, hipStream_t s) {
  if (tiles <= 0) return;
  hipLaunchKernelGGL(restore_counts_kernel, dim3((unsigned)((tiles + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     s, tile_count, ranges, tiles);
}

void launch_segment_sort(const SegSortBufs& b, int32_t total_tiles, hipStream_t s) {
  if (total_tiles <= 0) return;
  hipLaunchKernelGGL(segment_sort_kernel, dim3(total_tiles), dim3(kThreads), 0, s, b);
}

}  // namespace cgsr
