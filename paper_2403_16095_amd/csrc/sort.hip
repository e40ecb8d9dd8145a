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

// Bitonic sort of s[0, p) ascending, p a power of two; all threads call it.
__device__ void bitonic_lds(uint64_t* s, uint32_t p) {
  for (uint32_t k = 2; k <= p; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < p / 2; i += kThreads) {
        const uint32_t lo = 2 * j * (i / j) + (i % j);
        const uint32_t hi = lo + j;
        const bool up = (lo & k) == 0;
        const uint64_t a = s[lo], b = s[hi];
        if ((a > b) == up) {
          s[lo] = b;
          s[hi] = a;
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
    for (uint32_t i = threadIdx.x; i < p; i += kThreads) s[i] = i < n ? keys[i] : ~0ull;
    __syncthreads();
    bitonic_lds(s, p);
    for (uint32_t i = threadIdx.x; i < n; i += kThreads) b.sorted_vals[base + i] = (uint32_t)s[i];
    return;
  }
  // Long segment: sort chunks in LDS, write them back, then merge runs.
  for (uint32_t c0 = 0; c0 < n; c0 += kLdsKeys) {
    const uint32_t cn = min((uint32_t)kLdsKeys, n - c0);
    const uint32_t p = next_pow2(cn);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < p; i += kThreads) s[i] = i < cn ? keys[c0 + i] : ~0ull;
    __syncthreads();
    bitonic_lds(s, p);
    for (uint32_t i = threadIdx.x; i < cn; i += kThreads) keys[c0 + i] = s[i];
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
