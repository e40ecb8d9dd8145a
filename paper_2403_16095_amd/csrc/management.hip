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

#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kScanThreads = 1024;

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

// One workgroup: exclusive scan of each kind's workgroup counts, each lane
// taking a contiguous run of workgroups.
__global__ __launch_bounds__(kScanThreads) void ranked_scan_kernel(Ranked r) {
  __shared__ uint32_t s_w[kScanThreads / kWave];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int64_t per = (r.blocks + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = std::min<int64_t>(r.blocks, (int64_t)threadIdx.x * per);
  const int64_t b1 = std::min<int64_t>(r.blocks, b0 + per);
  for (int k = 0; k < kRankKinds; ++k) {
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

struct CompactOp {
  GaussArrays src, dst;
  int colour_w;
  const uint8_t* keep;
  ExtraArrays extra;

  __device__ uint32_t flags(int64_t i) const { return keep[i] ? 1u : 0u; }

  __device__ void emit(int64_t i, uint32_t, const uint32_t* rank, const uint32_t*) const {
    const int64_t j = rank[0];
    copy_gaussian(src, dst, i, j, colour_w);
    for (int e = 0; e < extra.n; ++e) {
      const int w = extra.width[e];
      for (int c = 0; c < w; ++c) extra.dst[e][(int64_t)w * j + c] = extra.src[e][(int64_t)w * i + c];
    }
  }
};

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
  hipLaunchKernelGGL(ranked_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, r);
  hipLaunchKernelGGL(ranked_emit_kernel<Op>, dim3((unsigned)blocks), dim3(kThreads), 0, s, op, n, r);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(totals_host, r.totals, sizeof(uint32_t) * kRankKinds, hipMemcpyDeviceToHost, s);
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

hipError_t run_compact(int64_t n, const uint8_t* keep, const GaussArrays& src, const GaussArrays& dst, int colour_w,
                       const ExtraArrays& extra, uint32_t* total, hipStream_t s) {
  CompactOp op{src, dst, colour_w, keep, extra};
  uint32_t t[kRankKinds];
  const hipError_t e = run_ranked(op, n, t, s);
  *total = t[0];
  return e;
}

hipError_t run_densify(int64_t n, const float* grad_accum, const uint32_t* count, float threshold, float dense_scale,
                       const float* normals, const GaussArrays& src, const GaussArrays& dst, int colour_w,
                       int64_t capacity, uint32_t* totals, hipStream_t s) {
  DensifyOp op{src, dst, colour_w, capacity, grad_accum, count, threshold, dense_scale, normals};
  return run_ranked(op, n, totals, s);
}

}  // namespace cgsr
