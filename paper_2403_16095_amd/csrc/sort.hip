// Stable LSD radix sort of the (tile | depth, record) pairs -- the depth
// pre-sort of Sec. 3.1, done per 16x16 tile -- and the per-tile range pass.
//
// Each 8-bit pass is two launches: a per-workgroup digit histogram, and a
// scatter whose workgroups each derive their own output offsets from the whole
// histogram table (no single-workgroup scan in between).  The pair count lives
// in device memory, so grids are sized to the capacity and workgroups past the
// work exit at once; nothing is read back to the host.
#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;                      // keys per lane per sub-tile
constexpr int kWaveSpan = kWave * kItems;       // 1024 keys per wave per sub-tile
constexpr int kSubTile = kThreads * kItems;     // 4096 keys per workgroup per sub-tile
constexpr int kRadix = 256;

struct Geometry {
  uint32_t count, blocks, chunk;
};

__device__ __forceinline__ Geometry geometry(const uint32_t* counters, int64_t cap, int max_blocks) {
  Geometry g;
  const int64_t k = min((int64_t)counters[kCntPairs], cap);
  g.count = (uint32_t)k;
  const uint32_t want = (g.count + kSubTile - 1) / kSubTile;
  g.blocks = max(1u, min((uint32_t)max_blocks, want));
  g.chunk = (g.count + g.blocks - 1) / g.blocks;
  return g;
}

// Lanes of this wave holding the same 8-bit digit (restricted to valid lanes).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool set = (d >> bit) & 1u;
    const uint64_t b = __ballot(set);
    m &= set ? b : ~b;
  }
  return m;
}

__global__ __launch_bounds__(kThreads) void hist_kernel(SortBufs b, int shift, int src) {
  __shared__ uint32_t h[4][kRadix];
  const Geometry geo = geometry(b.counters, b.cap, b.max_blocks);
  if (blockIdx.x >= geo.blocks) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) h[w][lane * 4 + k] = 0u;
  const uint32_t begin = blockIdx.x * geo.chunk;
  const uint32_t end = min(geo.count, begin + geo.chunk);
  const uint64_t* keys = b.keys[src];
  // Each wave walks its own stride of 64 keys; same-digit lanes are counted by
  // their leader so a skewed digit costs one LDS update per wave, not 64.
  for (uint32_t base = begin + w * kWave; base < end; base += kThreads) {
    const uint32_t idx = base + lane;
    const bool valid = idx < end;
    const uint32_t d = valid ? (uint32_t)(keys[idx] >> shift) & 0xFFu : 0u;
    const uint64_t peers = match_digit(d, valid);
    if (valid && lane == (int)__builtin_ctzll(peers)) h[w][d] += (uint32_t)__builtin_popcountll(peers);
  }
  __syncthreads();
  const int d = threadIdx.x;
  b.hist[blockIdx.x * kRadix + d] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

__device__ uint32_t exclusive_scan_256(uint32_t x, uint32_t* lds4) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d);
    if (lane >= d) inc += y;
  }
  if (lane == 63) lds4[w] = inc;
  __syncthreads();
  uint32_t base = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) base += (k < w) ? lds4[k] : 0u;
  __syncthreads();
  return base + inc - x;
}

__global__ __launch_bounds__(kThreads) void scatter_kernel(SortBufs b, int shift, int src) {
  __shared__ uint32_t s_base[kRadix];
  __shared__ uint32_t s_wcnt[4][kRadix];
  __shared__ uint32_t s_scan[4];
  const Geometry geo = geometry(b.counters, b.cap, b.max_blocks);
  if (blockIdx.x >= geo.blocks) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

  // Output offset of each digit for this workgroup: all keys with a smaller
  // digit, plus keys with this digit in earlier workgroups.
  {
    const int d = threadIdx.x;
    uint32_t tot = 0, before = 0;
    for (uint32_t bb = 0; bb < geo.blocks; ++bb) {
      const uint32_t c = b.hist[bb * kRadix + d];
      tot += c;
      before += bb < blockIdx.x ? c : 0u;
    }
    s_base[d] = exclusive_scan_256(tot, s_scan) + before;
  }

  const uint64_t* __restrict__ kin = b.keys[src];
  const uint32_t* __restrict__ vin = b.vals[src];
  uint64_t* __restrict__ kout = b.keys[src ^ 1];
  uint32_t* __restrict__ vout = b.vals[src ^ 1];
  const uint32_t begin = blockIdx.x * geo.chunk;
  const uint32_t end = min(geo.count, begin + geo.chunk);
  const uint64_t lt_mask = (1ull << lane) - 1ull;

  for (uint32_t start = begin; start < end; start += kSubTile) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s_wcnt[w][lane * 4 + k] = 0u;
    uint64_t key[kItems];
    uint32_t val[kItems];
    uint32_t rank[kItems];
    // Stable ranks within this wave's 1024 consecutive keys.
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t idx = start + w * kWaveSpan + r * kWave + lane;
      const bool valid = idx < end;
      key[r] = valid ? kin[idx] : 0ull;
      val[r] = valid ? vin[idx] : 0u;
      const uint32_t d = (uint32_t)(key[r] >> shift) & 0xFFu;
      const uint64_t peers = match_digit(d, valid);
      const uint32_t before = s_wcnt[w][d];
      rank[r] = before + (uint32_t)__builtin_popcountll(peers & lt_mask);
      if (valid && lane == (int)__builtin_ctzll(peers)) s_wcnt[w][d] = before + (uint32_t)__builtin_popcountll(peers);
    }
    __syncthreads();
    {
      const int d = threadIdx.x;
      const uint32_t c0 = s_wcnt[0][d], c1 = s_wcnt[1][d], c2 = s_wcnt[2][d], c3 = s_wcnt[3][d];
      const uint32_t base = s_base[d];
      s_wcnt[0][d] = base;
      s_wcnt[1][d] = base + c0;
      s_wcnt[2][d] = base + c0 + c1;
      s_wcnt[3][d] = base + c0 + c1 + c2;
      s_base[d] = base + c0 + c1 + c2 + c3;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t idx = start + w * kWaveSpan + r * kWave + lane;
      if (idx < end) {
        const uint32_t d = (uint32_t)(key[r] >> shift) & 0xFFu;
        const uint32_t pos = s_wcnt[w][d] + rank[r];
        kout[pos] = key[r];
        vout[pos] = val[r];
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void ranges_kernel(const uint64_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ counters, int64_t cap,
                                                          uint2* __restrict__ ranges) {
  const uint32_t k = (uint32_t)min((int64_t)counters[kCntPairs], cap);
  for (uint32_t idx = blockIdx.x * kThreads + threadIdx.x; idx < k; idx += gridDim.x * kThreads) {
    const uint32_t t = (uint32_t)(keys[idx] >> 32);
    if (idx == 0 || (uint32_t)(keys[idx - 1] >> 32) != t) ranges[t].x = idx;
    if (idx == k - 1 || (uint32_t)(keys[idx + 1] >> 32) != t) ranges[t].y = idx + 1;
  }
}

}  // namespace

void launch_sort(const SortBufs& b, int key_bits, hipStream_t s, int* result_buffer) {
  int src = 0;
  for (int shift = 0; shift < key_bits; shift += 8) {
    hipLaunchKernelGGL(hist_kernel, dim3(b.max_blocks), dim3(kThreads), 0, s, b, shift, src);
    hipLaunchKernelGGL(scatter_kernel, dim3(b.max_blocks), dim3(kThreads), 0, s, b, shift, src);
    src ^= 1;
  }
  *result_buffer = src;
}

void launch_ranges(const uint64_t* keys, const uint32_t* counters, int64_t cap, uint2* ranges, hipStream_t s) {
  hipLaunchKernelGGL(ranges_kernel, dim3(1024), dim3(kThreads), 0, s, keys, counters, cap, ranges);
}

}  // namespace cgsr
