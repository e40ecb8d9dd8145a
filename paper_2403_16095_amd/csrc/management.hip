// Gaussian management (Sec. 3.3): spawning Gaussians from the pixels a render
// leaves unobserved (rendered opacity below psi) using their colour and depth,
// order-preserving compaction of the set (removal), and the clone / split
// densification the paper keeps from splatting.
//
// All three are ranked selections: every item (candidate pixel or Gaussian)
// carries up to three flags, and each flagged item needs its rank among the
// items of its kind in item order, so the output order is deterministic.
// Three launches: per-workgroup counts (ballot and popcount), one workgroup
// scanning the counts into offsets and totals, then every workgroup emitting
// its items at rank = workgroup offset + preceding waves + lane rank (mbcnt).
#include <algorithm>
#include <mutex>

#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kScanThreads = 1024;
constexpr int kCompactItems = 1024;   // Gaussians per compaction workgroup

struct Ranked {
  uint32_t* counts;   // [kRankKinds][blocks]: counts, then exclusive offsets
  uint32_t* totals;   // [kRankKinds]
  int64_t blocks;
};

template <class Op>
__global__ __launch_bounds__(kThreads) void ranked_count_kernel(Op op, int64_t n, Ranked r) {
  __shared__ uint32_t s_cnt[kRankKinds][kWaves];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const uint32_t f = i < n ? op.flags(i) : 0u;
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
  for (int k = 0; k < kRankKinds; ++k) {
    const uint64_t m = __ballot((f >> k) & 1u);
    if (lane == 0) s_cnt[k][w] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < kRankKinds) {
    uint32_t t = 0;
    for (int q = 0; q < kWaves; ++q) t += s_cnt[threadIdx.x][q];
    r.counts[threadIdx.x * r.blocks + blockIdx.x] = t;
  }
}

// One workgroup: exclusive scan of each of kKinds kinds' workgroup counts,
// each lane taking a contiguous run of workgroups.
template <int kKinds>
__global__ __launch_bounds__(kScanThreads) void ranked_scan_kernel(Ranked r) {
  __shared__ uint32_t s_w[kScanThreads / kWave];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int64_t per = (r.blocks + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = std::min<int64_t>(r.blocks, (int64_t)threadIdx.x * per);
  const int64_t b1 = std::min<int64_t>(r.blocks, b0 + per);
  for (int k = 0; k < kKinds; ++k) {
    uint32_t* c = r.counts + k * r.blocks;
    uint32_t run = 0;
    for (int64_t b = b0; b < b1; ++b) run += c[b];
    uint32_t inc = run;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d);
      if (lane >= d) inc += y;
    }
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (int q = 0; q < kScanThreads / kWave; ++q) {
      base += q < w ? s_w[q] : 0u;
      total += s_w[q];
    }
    uint32_t acc = base + inc - run;
    for (int64_t b = b0; b < b1; ++b) {
      const uint32_t t = c[b];
      c[b] = acc;
      acc += t;
    }
    if (threadIdx.x == 0) r.totals[k] = total;
    __syncthreads();
  }
}

template <class Op>
__global__ __launch_bounds__(kThreads) void ranked_emit_kernel(Op op, int64_t n, Ranked r) {
  __shared__ uint32_t s_cnt[kRankKinds][kWaves];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const uint32_t f = i < n ? op.flags(i) : 0u;
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint32_t rank[kRankKinds];
#pragma unroll
  for (int k = 0; k < kRankKinds; ++k) {
    const uint64_t m = __ballot((f >> k) & 1u);
    rank[k] = (uint32_t)mask_rank(m);
    if (lane == 0) s_cnt[k][w] = (uint32_t)__popcll(m);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRankKinds; ++k) {
    uint32_t base = r.counts[k * r.blocks + blockIdx.x];
    for (int q = 0; q < w; ++q) base += s_cnt[k][q];
    rank[k] += base;
  }
  if (f) op.emit(i, f, rank, r.totals);
}

// Copies Gaussian i of src to slot j of dst (every array of the set).
__device__ __forceinline__ void copy_gaussian(const GaussArrays& src, const GaussArrays& dst, int64_t i, int64_t j,
                                              int colour_w) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    dst.means[3 * j + c] = src.means[3 * i + c];
    dst.log_scales[3 * j + c] = src.log_scales[3 * i + c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) dst.quats[4 * j + c] = src.quats[4 * i + c];
  dst.opacity_logits[j] = src.opacity_logits[i];
  const float* cs = src.sh ? src.sh : src.rgb;
  float* cd = src.sh ? dst.sh : dst.rgb;
  for (int c = 0; c < colour_w; ++c) cd[(int64_t)colour_w * j + c] = cs[(int64_t)colour_w * i + c];
}

// Candidate pixel c of a stride grid gw wide spawns when its sensor depth is
// positive and (with an opacity map) its rendered opacity is below psi.
struct SpawnOp {
  GaussArrays dst;
  int64_t n, capacity;
  int width, stride, gw, K;   // K: SH coefficients per channel, 0 = rgb
  float fx, fy, cx, cy, psi, init_logit;
  const float* pose;          // device [12]: R row-major, t
  const float *color, *depth, *opacity;
  int64_t hw;

  __device__ uint32_t flags(int64_t c) const {
    const int64_t p = (c / gw) * stride * (int64_t)width + (c % gw) * stride;
    const float D = depth[p];
    return (D > 0.f && (!opacity || opacity[p] < psi)) ? 1u : 0u;
  }

  __device__ void emit(int64_t c, uint32_t, const uint32_t* rank, const uint32_t*) const {
    const int64_t j = n + rank[0];
    if (j >= capacity) return;
    const int u = (int)(c % gw) * stride, v = (int)(c / gw) * stride;
    const int64_t p = (int64_t)v * width + u;
    const float D = depth[p];
    // back-projection of the pixel centre at depth D, then X = R^T (p - t)
    const float q0 = D * ((float)u - cx) / fx - pose[9];
    const float q1 = D * ((float)v - cy) / fy - pose[10];
    const float q2 = D - pose[11];
    const float ls = logf(D / (0.5f * (fx + fy)));
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      dst.means[3 * j + r] = pose[r] * q0 + pose[3 + r] * q1 + pose[6 + r] * q2;
      dst.log_scales[3 * j + r] = ls;
    }
    dst.quats[4 * j] = 1.f;
    dst.quats[4 * j + 1] = dst.quats[4 * j + 2] = dst.quats[4 * j + 3] = 0.f;
    dst.opacity_logits[j] = init_logit;
    if (K == 0) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) dst.rgb[3 * j + ch] = color[ch * hw + p];
    } else {
      // degree-0 harmonic Y_00 = 1 / sqrt(4 pi): colour = 1/2 + Y_00 k_0
      constexpr float kSqrt4Pi = 3.5449077018110318f;
      float* sh = dst.sh + (int64_t)3 * K * j;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) sh[ch] = (color[ch * hw + p] - 0.5f) * kSqrt4Pi;
      for (int k = 3; k < 3 * K; ++k) sh[k] = 0.f;
    }
  }
};

// Compaction streams the set array by array.  A workgroup owns a chunk of
// kCompactItems consecutive Gaussians: it ranks the chunk's kept ones in LDS
// (one block scan, each thread ranking kCompactPerThread consecutive items),
// then, for every array of w floats per Gaussian, reads the chunk's w x
// kCompactItems floats as 16-byte loads in address order and writes each
// kept float to its output row.  Kept Gaussians are contiguous in the output,
// so lanes write consecutive addresses too: both sides are coalesced whatever
// the width, instead of one lane walking one Gaussian's floats.
constexpr int kCompactThreads = 256;
constexpr int kCompactPerThread = 4;
constexpr int kCompactUnroll = 4;   // 16-byte loads in flight per thread
constexpr uint32_t kDropped = 0xFFFFFFFFu;

struct CompactArray {
  const float* src;
  float* dst;
  uint32_t width;
  uint32_t magic;   // floor(2^32 / width) + 1 (width >= 2): row = umulhi(f, magic)
};
constexpr int kMaxCompactArrays = 6 + kMaxExtraArrays;

struct CompactJob {
  int64_t n;
  const uint8_t* keep;
  uint32_t* counts;   // [chunks]: kept per chunk, then exclusive offsets
  uint32_t* total;    // [1]
  int64_t chunks;
  int n_arrays;
  CompactArray a[kMaxCompactArrays];
};

__global__ __launch_bounds__(kCompactThreads) void compact_count_kernel(CompactJob j) {
  __shared__ uint32_t s_w[kCompactThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kCompactItems;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kCompactPerThread; ++k) {
    const int64_t i = base + k * kCompactThreads + threadIdx.x;
    c += (i < j.n && j.keep[i]) ? 1u : 0u;
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) c += __shfl_xor(c, d);
  if (threadIdx.x % kWave == 0) s_w[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int q = 0; q < kCompactThreads / kWave; ++q) t += s_w[q];
    j.counts[blockIdx.x] = t;
  }
}

// Row of float f (0 <= f < kCompactItems * w) of a chunk: f / w, by a
// multiply-high with magic = floor(2^32 / w) + 1, exact while f (w - 2^32 mod
// w) < 2^32, which f < kCompactItems w with w < 2048 guarantees.
__device__ __forceinline__ uint32_t row_of(uint32_t f, const CompactArray& a) {
  if (a.width == 1) return f;
  if (a.width < 2048) return __umulhi(f, a.magic);
  return f / a.width;
}

__device__ __forceinline__ void put(const CompactArray& a, const uint32_t* s_rank, uint32_t f, float v) {
  const uint32_t r = row_of(f, a);
  const uint32_t out = s_rank[r];
  if (out != kDropped) a.dst[(int64_t)out * a.width + (f - r * a.width)] = v;
}

__global__ __launch_bounds__(kCompactThreads) void compact_emit_kernel(CompactJob j) {
  __shared__ uint32_t s_rank[kCompactItems];   // output row of each item of the chunk, or kDropped
  __shared__ uint32_t s_w[kCompactThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kCompactItems;
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  uint32_t f[kCompactPerThread], c = 0;
#pragma unroll
  for (int k = 0; k < kCompactPerThread; ++k) {
    const int64_t i = base + kCompactPerThread * t + k;
    f[k] = (i < j.n && j.keep[i]) ? 1u : 0u;
    c += f[k];
  }
  uint32_t inc = c;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d);
    if (lane >= d) inc += y;
  }
  if (lane == kWave - 1) s_w[w] = inc;
  __syncthreads();
  uint32_t row = j.counts[blockIdx.x] + inc - c;
  for (int q = 0; q < w; ++q) row += s_w[q];
#pragma unroll
  for (int k = 0; k < kCompactPerThread; ++k) s_rank[kCompactPerThread * t + k] = f[k] ? row++ : kDropped;
  __syncthreads();
  const uint32_t items = (uint32_t)std::min<int64_t>(kCompactItems, j.n - base);
  for (int ai = 0; ai < j.n_arrays; ++ai) {
    const CompactArray a = j.a[ai];
    const float* src = a.src + base * a.width;
    const uint32_t len = items * a.width;
    uint32_t done = 0;
    if ((reinterpret_cast<uintptr_t>(a.src) & 15u) == 0) {
      // a chunk starts at a multiple of kCompactItems * w floats, so its
      // 16-byte loads stay aligned when the array is
      const uint32_t nv = len / 4;
      const float4* src4 = reinterpret_cast<const float4*>(src);
      for (uint32_t q0 = t; q0 < nv; q0 += kCompactThreads * kCompactUnroll) {
        float4 v[kCompactUnroll];
#pragma unroll
        for (int u = 0; u < kCompactUnroll; ++u) {
          const uint32_t q = q0 + u * kCompactThreads;
          v[u] = q < nv ? src4[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kCompactUnroll; ++u) {
          const uint32_t q = q0 + u * kCompactThreads;
          if (q < nv) {
            put(a, s_rank, 4 * q, v[u].x);
            put(a, s_rank, 4 * q + 1, v[u].y);
            put(a, s_rank, 4 * q + 2, v[u].z);
            put(a, s_rank, 4 * q + 3, v[u].w);
          }
        }
      }
      done = nv * 4;
    }
    for (uint32_t q = done + t; q < len; q += kCompactThreads) put(a, s_rank, q, src[q]);
  }
}

// Flags: 1 kept (not split), 2 clone, 4 split.
struct DensifyOp {
  GaussArrays src, dst;
  int colour_w;
  int64_t capacity;
  const float* grad_accum;
  const uint32_t* count;
  float threshold, dense_scale;
  const float* normals;   // [n][2][3]

  __device__ uint32_t flags(int64_t i) const {
    const uint32_t c = count[i];
    const float stat = c ? grad_accum[i] / (float)c : 0.f;
    if (!(stat >= threshold)) return 1u;
    const float* ls = src.log_scales + 3 * i;
    const float smax = expf(fmaxf(ls[0], fmaxf(ls[1], ls[2])));
    return smax <= dense_scale ? (1u | 2u) : 4u;
  }

  __device__ void emit(int64_t i, uint32_t f, const uint32_t* rank, const uint32_t* totals) const {
    if ((f & 1u) && rank[0] < capacity) copy_gaussian(src, dst, i, rank[0], colour_w);
    if ((f & 2u) && totals[0] + rank[1] < capacity) copy_gaussian(src, dst, i, totals[0] + rank[1], colour_w);
    if (!(f & 4u)) return;
    // two halves at mu + R diag(s) z_k, scales / 1.6, the rest copied
    const float4 q = make_float4(src.quats[4 * i], src.quats[4 * i + 1], src.quats[4 * i + 2], src.quats[4 * i + 3]);
    const float inv = 1.0f / sqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
    const float w = q.x * inv, x = q.y * inv, y = q.z * inv, z = q.w * inv;
    const float Rq[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                         2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                         2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
    float s[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] = expf(src.log_scales[3 * i + c]);
    const float ldiv = logf(1.6f);
    for (int k = 0; k < 2; ++k) {
      const int64_t j = (int64_t)totals[0] + totals[1] + 2 * (int64_t)rank[2] + k;
      if (j >= capacity) break;
      copy_gaussian(src, dst, i, j, colour_w);
      const float* zk = normals + 6 * i + 3 * k;
      const float a0 = s[0] * zk[0], a1 = s[1] * zk[1], a2 = s[2] * zk[2];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        dst.means[3 * j + r] = src.means[3 * i + r] + (Rq[3 * r] * a0 + Rq[3 * r + 1] * a1 + Rq[3 * r + 2] * a2);
        dst.log_scales[3 * j + r] = src.log_scales[3 * i + r] - ldiv;
      }
    }
  }
};

template <class Op>
hipError_t run_ranked(const Op& op, int64_t n, uint32_t* totals_host, hipStream_t s) {
  const int64_t blocks = std::max<int64_t>(1, (n + kThreads - 1) / kThreads);
  uint32_t* buf = nullptr;
  hipError_t e = hipMallocAsync((void**)&buf, sizeof(uint32_t) * (size_t)(kRankKinds * blocks + kRankKinds), s);
  if (e != hipSuccess) return e;
  Ranked r{buf, buf + kRankKinds * blocks, blocks};
  hipLaunchKernelGGL(ranked_count_kernel<Op>, dim3((unsigned)blocks), dim3(kThreads), 0, s, op, n, r);
  hipLaunchKernelGGL(ranked_scan_kernel<kRankKinds>, dim3(1), dim3(kScanThreads), 0, s, r);
  hipLaunchKernelGGL(ranked_emit_kernel<Op>, dim3((unsigned)blocks), dim3(kThreads), 0, s, op, n, r);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(totals_host, r.totals, sizeof(uint32_t) * kRankKinds, hipMemcpyDeviceToHost, s);
  const hipError_t f = hipFreeAsync(buf, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e != hipSuccess ? e : f;
}

}  // namespace

hipError_t run_spawn(const GaussArrays& dst, int64_t n, int64_t capacity, const ViewInfo& cam, const float* pose,
                     const float* color, const float* depth, const float* opacity, float psi, int stride,
                     float init_logit, int K, uint32_t* total, hipStream_t s) {
  SpawnOp op;
  op.dst = dst;
  op.n = n;
  op.capacity = capacity;
  op.width = cam.width;
  op.stride = stride;
  op.gw = (cam.width + stride - 1) / stride;
  const int gh = (cam.height + stride - 1) / stride;
  op.K = K;
  op.fx = cam.fx;
  op.fy = cam.fy;
  op.cx = cam.cx;
  op.cy = cam.cy;
  op.psi = psi;
  op.init_logit = init_logit;
  op.pose = pose;
  op.color = color;
  op.depth = depth;
  op.opacity = opacity;
  op.hw = (int64_t)cam.width * cam.height;
  uint32_t t[kRankKinds];
  const hipError_t e = run_ranked(op, (int64_t)op.gw * gh, t, s);
  *total = t[0];
  return e;
}

namespace {

// Fills the job's array list from the set and the extra arrays.
CompactJob compact_job(int64_t n, const uint8_t* keep, const GaussArrays& src, const GaussArrays& dst, int colour_w,
                       const ExtraArrays& extra) {
  CompactJob j{};
  j.n = n;
  j.keep = keep;
  j.chunks = (n + kCompactItems - 1) / kCompactItems;
  auto add = [&](const float* sp, float* dp, int w) {
    CompactArray& a = j.a[j.n_arrays++];
    a.src = sp;
    a.dst = dp;
    a.width = (uint32_t)w;
    a.magic = w >= 2 ? (uint32_t)((1ull << 32) / (uint64_t)w + 1ull) : 0u;
  };
  add(src.means, dst.means, 3);
  add(src.log_scales, dst.log_scales, 3);
  add(src.quats, dst.quats, 4);
  add(src.opacity_logits, dst.opacity_logits, 1);
  add(src.sh ? src.sh : src.rgb, src.sh ? dst.sh : dst.rgb, colour_w);
  for (int e = 0; e < extra.n; ++e) add(extra.src[e], extra.dst[e], extra.width[e]);
  return j;
}

// Count, scan and emit with the caller's scratch (chunks + 1 words), then
// the kept count to the host.
hipError_t launch_compact(CompactJob j, uint32_t* scratch, uint32_t* total, hipStream_t s) {
  j.counts = scratch;
  j.total = scratch + j.chunks;
  const Ranked r{j.counts, j.total, j.chunks};
  hipLaunchKernelGGL(compact_count_kernel, dim3((unsigned)j.chunks), dim3(kCompactThreads), 0, s, j);
  hipLaunchKernelGGL(ranked_scan_kernel<1>, dim3(1), dim3(kScanThreads), 0, s, r);
  hipLaunchKernelGGL(compact_emit_kernel, dim3((unsigned)j.chunks), dim3(kCompactThreads), 0, s, j);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(total, j.total, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  return e;
}

}  // namespace

hipError_t run_compact(int64_t n, const uint8_t* keep, const GaussArrays& src, const GaussArrays& dst, int colour_w,
                       const ExtraArrays& extra, uint32_t* total, hipStream_t s) {
  *total = 0;
  if (n <= 0) return hipSuccess;
  const CompactJob j = compact_job(n, keep, src, dst, colour_w, extra);
  uint32_t* buf = nullptr;
  hipError_t e = hipMallocAsync((void**)&buf, sizeof(uint32_t) * (size_t)(j.chunks + 1), s);
  if (e != hipSuccess) return e;
  e = launch_compact(j, buf, total, s);
  const hipError_t f = hipFreeAsync(buf, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e != hipSuccess ? e : f;
}

// Scratch of the allocation-free compaction: one counter per chunk of
// kCompactItems Gaussians plus the total, for up to kNoAllocMaxN Gaussians
// (256 KB).  Every GPU the library runs on holds its own copy until the
// process ends.  In host code the name is only a stand-in for the device
// address, which scratch_address() takes from hipGetSymbolAddress once per
// device and keeps.
constexpr int64_t kNoAllocChunks = kNoAllocMaxN / kCompactItems;
static __device__ __align__(256) uint32_t scratch[kNoAllocChunks + 64];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch (the current device's).
hipError_t scratch_address(uint32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

hipError_t run_compact_noalloc(int64_t n, const uint8_t* keep, const GaussArrays& src, const GaussArrays& dst,
                               int colour_w, const ExtraArrays& extra, uint32_t* total, hipStream_t s) {
  *total = 0;
  if (n <= 0) return hipSuccess;
  if (n > kNoAllocMaxN) return hipErrorInvalidValue;
  uint32_t* buf = nullptr;
  hipError_t e = scratch_address(&buf);
  if (e != hipSuccess) return e;
  // every counter the kernels read is written first by this call's count
  // and scan launches, so nothing is cleared
  e = launch_compact(compact_job(n, keep, src, dst, colour_w, extra), buf, total, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

hipError_t run_densify(int64_t n, const float* grad_accum, const uint32_t* count, float threshold, float dense_scale,
                       const float* normals, const GaussArrays& src, const GaussArrays& dst, int colour_w,
                       int64_t capacity, uint32_t* totals, hipStream_t s) {
  DensifyOp op{src, dst, colour_w, capacity, grad_accum, count, threshold, dense_scale, normals};
  return run_ranked(op, n, totals, s);
}

}  // namespace cgsr
