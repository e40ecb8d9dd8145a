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
constexpr int kOrderThreads = 1024;
constexpr int kOrderBins = 16 * 33;
constexpr uint32_t kOrderRound = 256;   // compute units of the chip

__device__ __forceinline__ uint32_t order_bin(uint32_t n) {
  if (n == 0) return 0;
  const uint32_t lz = __builtin_clz(n);                  // leading bit at 31 - lz
  const uint32_t frac = lz <= 27 ? (n >> (27 - lz)) & 15u : (n << (lz - 27)) & 15u;   // the next four bits
  return 1u + 16u * (31u - lz) + frac;
}

// A tile's list length: from its range after the sort, or (ranges null) from
// its pair counter before a blend that sorts its own bucket.
__device__ __forceinline__ uint32_t tile_length(const uint2* ranges, const uint32_t* counts, int t) {
  if (ranges) {
    const uint2 r = ranges[t];
    return r.y - r.x;
  }
  return counts[(size_t)t * kTileCounterStride];
}

// s_bin holds each bin's count on entry and its first position, the longest
// bin first, on return: thread k scans bin kOrderBins - 1 - k.
__device__ __forceinline__ void bin_offsets_longest_first(uint32_t* s_bin, uint32_t* s_wave) {
  static_assert(kOrderBins <= kOrderThreads, "one bin per thread in the scan");
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
}

__global__ __launch_bounds__(kOrderThreads) void tile_order_kernel(const uint2* __restrict__ ranges,
                                                                   const uint32_t* __restrict__ counts, int32_t tiles,
                                                                   uint32_t* __restrict__ order) {
  __shared__ uint32_t s_bin[kOrderBins];
  __shared__ uint32_t s_wave[kOrderThreads / kWave];
  for (int i = threadIdx.x; i < kOrderBins; i += kOrderThreads) s_bin[i] = 0u;
  __syncthreads();
  for (int t = threadIdx.x; t < tiles; t += kOrderThreads)
    atomicAdd(&s_bin[order_bin(tile_length(ranges, counts, t))], 1u);
  __syncthreads();
  bin_offsets_longest_first(s_bin, s_wave);
  for (int t = threadIdx.x; t < tiles; t += kOrderThreads)
    order[atomicAdd(&s_bin[order_bin(tile_length(ranges, counts, t))], 1u)] = (uint32_t)t;
}

// The kept order of a launch whose tiles are all resident from the start
// (tiles <= kKeptOrderMaxTiles).  A tile's length is the work its four waves
// measured in the previous step: quads[t * kTileCounterStride + k] for
// quadrant k (words 1..4 of its counter line), read once into LDS.  Longest
// first as above, then every other run of kOrderRound positions reversed, so
// that the workgroups dealt one per CU take, CU by CU, a long tile of one run
// with a short one of the next, and the last, short run's tiles (the
// shortest, longest of them first) go to its positions in ascending order of
// the work the full runs gave the same CU position; the CUs' summed work
// comes out more even (a model of the dispatch over measured tracking lists:
// the fullest CU 1.16x the mean work longest first, 1.10x with the runs
// reversed, 1.06x with the last run placed by load).  Each entry then takes a
// quadrant rotation in its top two bits (below).
__global__ __launch_bounds__(kOrderThreads) void tile_order_kept_kernel(const uint32_t* __restrict__ quads,
                                                                        int32_t tiles, uint32_t* __restrict__ order) {
  __shared__ uint32_t s_bin[kOrderBins];
  __shared__ uint32_t s_wave[kOrderThreads / kWave];
  __shared__ uint4 s_quad[kKeptOrderMaxTiles];
  __shared__ uint32_t s_load[kOrderRound], s_perm[kOrderRound], s_ord[kKeptOrderMaxTiles];
  constexpr int kPer = kKeptOrderMaxTiles / kOrderThreads;
  for (int i = threadIdx.x; i < kOrderBins; i += kOrderThreads) s_bin[i] = 0u;
  if (threadIdx.x < kOrderRound) s_load[threadIdx.x] = 0u;
  uint4 qw[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {   // every load in flight at once
    const int t = threadIdx.x + q * kOrderThreads;
    const uint32_t* c = quads + (size_t)t * kTileCounterStride;
    qw[q] = t < tiles ? make_uint4(c[0], c[1], c[2], c[3]) : make_uint4(0u, 0u, 0u, 0u);
  }
  __syncthreads();
  uint32_t len[kPer], rank[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int t = threadIdx.x + q * kOrderThreads;
    len[q] = qw[q].x + qw[q].y + qw[q].z + qw[q].w;
    if (t < tiles) {
      s_quad[t] = qw[q];
      atomicAdd(&s_bin[order_bin(len[q])], 1u);
    }
  }
  __syncthreads();
  bin_offsets_longest_first(s_bin, s_wave);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int t = threadIdx.x + q * kOrderThreads;
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
  {   // rank of each last-run position by (load, position): four lanes per position
    static_assert(kOrderThreads == 4 * kOrderRound, "four lanes rank each position");
    const uint32_t j = threadIdx.x >> 2, part = threadIdx.x & 3u;
    uint32_t r = 0;
    if (j < rem) {
      const uint32_t key = s_load[j];
#pragma unroll 4
      for (uint32_t i = part; i < rem; i += 4) r += (s_load[i] < key || (s_load[i] == key && i < j)) ? 1u : 0u;
    }
    r += __shfl_xor(r, 1);
    r += __shfl_xor(r, 2);
    if (j < rem && part == 0) s_perm[r] = j;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int t = threadIdx.x + q * kOrderThreads;
    if (t < tiles && rank[q] >= full) s_ord[full + s_perm[rank[q] - full]] = (uint32_t)t;
  }
  __syncthreads();
  // The workgroups at positions c, c + 256, ... run on one CU, the r-th of
  // them with its wave w on that CU's SIMD kSimdOf[(w + r) & 3] (the
  // dispatcher's rule, up to a renaming of the SIMDs).  Wave w takes
  // quadrant (w + rot) & 3, so SIMD s gets quadrant (kSimdOf[s] + d) & 3 with
  // d = rot - r (kSimdOf is its own inverse).  Each CU's workgroups in turn
  // take the d, the first of equals, that keeps the CU's busiest SIMD least
  // busy.
  if (threadIdx.x < kOrderRound) {
    constexpr uint32_t kSimdOf[4] = {0, 2, 1, 3};
    uint32_t load[4] = {0u, 0u, 0u, 0u};
    uint32_t r = 0;
    for (uint32_t p = threadIdx.x; p < (uint32_t)tiles; p += kOrderRound, ++r) {
      const uint32_t t = s_ord[p];
      const uint4 w4 = s_quad[t];
      const uint32_t qw[4] = {w4.x, w4.y, w4.z, w4.w};
      uint32_t trial[4][4];   // [d][s]
      uint32_t best = 0xFFFFFFFFu, pick = 0;
#pragma unroll
      for (uint32_t d = 0; d < 4; ++d) {
#pragma unroll
        for (uint32_t s4 = 0; s4 < 4; ++s4) trial[d][s4] = load[s4] + qw[(kSimdOf[s4] + d) & 3];
        const uint32_t m = max(max(trial[d][0], trial[d][1]), max(trial[d][2], trial[d][3]));
        pick = m < best ? d : pick;
        best = m < best ? m : best;
      }
#pragma unroll
      for (uint32_t s4 = 0; s4 < 4; ++s4)
        load[s4] = pick == 0 ? trial[0][s4] : pick == 1 ? trial[1][s4] : pick == 2 ? trial[2][s4] : trial[3][s4];
      order[p] = t | (((pick + r) & 3u) << 30);
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

void launch_tile_order(const uint2* ranges, const uint32_t* counts, int32_t tiles, uint32_t* order, hipStream_t s) {
  if (tiles <= 0) return;
  hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(kOrderThreads), 0, s, ranges, counts, tiles, order);
}

void launch_tile_order_kept(const uint32_t* quads, int32_t tiles, uint32_t* order, hipStream_t s) {
  if (tiles <= 0 || tiles > kKeptOrderMaxTiles) return;   // callers keep within the limit
  hipLaunchKernelGGL(tile_order_kept_kernel, dim3(1), dim3(kOrderThreads), 0, s, quads, tiles, order);
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
