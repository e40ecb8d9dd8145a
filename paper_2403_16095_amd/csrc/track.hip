// Sequential-tracking glue kept on the device so a whole tracking iteration
// can be replayed from a HIP graph: gradient images of the tracking loss
// (Eq. 19 from Eq. 14 and 16) and the Adam step plus retraction on the pose
// (Eq. 20).  Also the counters behind cgsr_get_stats, and the per-Gaussian
// uncertainty finalisation and pruning of Sec. 3.2 (Eq. 13).
#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float sgn(float x) { return (float)((x > 0.f) - (x < 0.f)); }

__global__ __launch_bounds__(kThreads) void tracking_loss_kernel(int w, int h, const float* __restrict__ color,
                                                                 const float* __restrict__ depth,
                                                                 const float* __restrict__ tcolor,
                                                                 const float* __restrict__ tdepth, float lc, float ld,
                                                                 float* __restrict__ dcolor,
                                                                 float* __restrict__ ddepth, float* loss) {
  __shared__ float s_part[4];
  const int64_t hw = (int64_t)w * h;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const float inv = 1.0f / (float)hw;
  float l = 0.f;
  if (i < hw) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float diff = color[c * hw + i] - tcolor[c * hw + i];
      dcolor[c * hw + i] = lc * inv * sgn(diff);
      l += fabsf(diff);
    }
    l *= lc;
    const float dd = depth[i] - tdepth[i];
    ddepth[i] = ld * inv * sgn(dd);
    l = (l + ld * fabsf(dd)) * inv;
  }
  if (!loss) return;
  const float t = wave_sum(l);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, s_part[0] + s_part[1] + s_part[2] + s_part[3]);
}

// Mapping loss L = mean_n |I^ - I|_1 + mean_n U |D^ - D|, per pixel.
__global__ __launch_bounds__(kThreads) void mapping_loss_kernel(int w, int h, const float* __restrict__ color,
                                                                const float* __restrict__ depth,
                                                                const float* __restrict__ unc,
                                                                const float* __restrict__ tcolor,
                                                                const float* __restrict__ tdepth,
                                                                float* __restrict__ dcolor, float* __restrict__ ddepth,
                                                                float* __restrict__ dunc, float* loss) {
  __shared__ float s_part[4];
  const int64_t hw = (int64_t)w * h;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const float inv = 1.0f / (float)hw;
  float l = 0.f;
  if (i < hw) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float diff = color[c * hw + i] - tcolor[c * hw + i];
      dcolor[c * hw + i] = inv * sgn(diff);
      l += fabsf(diff);
    }
    const float dd = depth[i] - tdepth[i];
    ddepth[i] = inv * unc[i] * sgn(dd);
    dunc[i] = inv * fabsf(dd);
    l = (l + unc[i] * fabsf(dd)) * inv;
  }
  if (!loss) return;
  const float t = wave_sum(l);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, s_part[0] + s_part[1] + s_part[2] + s_part[3]);
}

// One wave per view, lane k on component k: Adam step and retraction
// (adam_retract_wave), then the gradient buffer is cleared for the next
// iteration.
__global__ __launch_bounds__(64) void pose_adam_kernel(float* poses, float* dposes, float* adam, AdamParams ap) {
  const int v = blockIdx.x, k = threadIdx.x;
  float g = 0.f;
  if (k < 6) {
    g = dposes[6 * v + k];
    dposes[6 * v + k] = 0.f;
  }
  adam_retract_wave(poses + 12 * v, adam + 16 * v, g, ap);
}

// nu_i = nu_sum_i / (M_1 + ... + M_k) (Eq. 13), 0 for a Gaussian that
// dominates no pixel; nu_i > tau lowers its opacity logit to low_logit (it is
// never raised).  One block-reduced atomic counts the pruned Gaussians.
__global__ __launch_bounds__(kThreads) void nu_prune_kernel(int64_t n, const float* __restrict__ nu_sum,
                                                            const uint32_t* __restrict__ nu_count, float tau,
                                                            float low_logit, float* __restrict__ opacity_logits,
                                                            float* __restrict__ nu, uint32_t* n_pruned) {
  __shared__ uint32_t s_part[kThreads / 64];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  uint32_t pruned = 0;
  if (i < n) {
    const uint32_t c = nu_count[i];
    const float v = c ? nu_sum[i] / (float)c : 0.f;
    if (nu) nu[i] = v;
    if (v > tau) {
      pruned = 1;
      if (opacity_logits) opacity_logits[i] = fminf(opacity_logits[i], low_logit);
    }
  }
  if (!n_pruned) return;
  const uint64_t mask = __ballot(pruned);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = (uint32_t)__popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < kThreads / 64; ++k) t += s_part[k];
    if (t) atomicAdd(n_pruned, t);
  }
}

// One Adam step (Kingma and Ba, with bias correction) on element e of the
// concatenated parameter groups: widths 3, 3, 4, 1 and the colour width per
// Gaussian.
__global__ __launch_bounds__(kThreads) void gaussian_adam_kernel(int64_t n, GaussianAdam a, float* moments,
                                                                 const uint32_t* step) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t total = (11 + (int64_t)a.colour_width) * n;
  if (e >= total) return;
  // group of e: boundaries 3n, 6n, 10n, 11n, total
  int grp;
  int64_t base;
  if (e < 3 * n) { grp = 0; base = 0; }
  else if (e < 6 * n) { grp = 1; base = 3 * n; }
  else if (e < 10 * n) { grp = 2; base = 6 * n; }
  else if (e < 11 * n) { grp = 3; base = 10 * n; }
  else { grp = 4; base = 11 * n; }
  float* p = a.param[grp];
  float* gp = a.grad[grp];
  const int64_t k = e - base;
  // SH coefficients past the three of degree 0 take their own rate
  const float lr = grp == 4 && k % a.colour_width >= 3 ? a.lr_sh_rest : a.lr[grp];
  const float t = (float)(*step + 1u);
  const float g = gp[k];
  gp[k] = 0.f;
  float* m = moments + e;
  float* v = moments + total + e;
  const float mm = a.beta1 * *m + (1.f - a.beta1) * g;
  const float vv = a.beta2 * *v + (1.f - a.beta2) * g * g;
  *m = mm;
  *v = vv;
  const float c1 = 1.f - powf(a.beta1, t), c2 = 1.f - powf(a.beta2, t);
  p[k] -= lr * (mm / c1) / (sqrtf(vv / c2) + a.eps);
}

__global__ void increment_kernel(uint32_t* step) { *step += 1u; }

__global__ __launch_bounds__(kThreads) void stats_kernel(const uint32_t* __restrict__ tiles, int64_t m,
                                                         const uint4* __restrict__ ps,
                                                         const uint2* __restrict__ count, int64_t pixels,
                                                         const uint2* __restrict__ ranges, int64_t n_tiles,
                                                         unsigned long long* out) {
  unsigned long long vis = 0, ev = 0, bl = 0, wk = 0, pairs = 0, peak = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < m; i += (int64_t)gridDim.x * kThreads)
    vis += tiles[i] != 0u;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < pixels; i += (int64_t)gridDim.x * kThreads) {
    ev += ps[i].w;
    wk += count[i].y;
    bl += count[i].x;
  }
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n_tiles; i += (int64_t)gridDim.x * kThreads) {
    const unsigned long long n = ranges[i].y - ranges[i].x;
    pairs += n;
    peak = n > peak ? n : peak;
  }
  // These counters are read rarely; one atomic per lane keeps the code short.
  if (vis) atomicAdd(out, vis);
  if (ev) atomicAdd(out + 1, ev);
  if (bl) atomicAdd(out + 2, bl);
  if (wk) atomicAdd(out + 3, wk);
  if (pairs) atomicAdd(out + 4, pairs);
  if (peak) atomicMax(out + 5, peak);
}

}  // namespace

void launch_tracking_loss(int w, int h, const float* color, const float* depth, const float* tcolor,
                          const float* tdepth, float lc, float ld, float* dcolor, float* ddepth, float* loss,
                          hipStream_t s) {
  const int64_t hw = (int64_t)w * h;
  hipLaunchKernelGGL(tracking_loss_kernel, dim3((unsigned)((hw + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     w, h, color, depth, tcolor, tdepth, lc, ld, dcolor, ddepth, loss);
}

void launch_mapping_loss(int w, int h, const float* color, const float* depth, const float* unc,
                         const float* tcolor, const float* tdepth, float* dcolor, float* ddepth, float* dunc,
                         float* loss, hipStream_t s) {
  const int64_t hw = (int64_t)w * h;
  hipLaunchKernelGGL(mapping_loss_kernel, dim3((unsigned)((hw + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     w, h, color, depth, unc, tcolor, tdepth, dcolor, ddepth, dunc, loss);
}

void launch_nu_prune(int64_t n, const float* nu_sum, const uint32_t* nu_count, float tau, float low_logit,
                     float* opacity_logits, float* nu, uint32_t* n_pruned, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(nu_prune_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, n,
                     nu_sum, nu_count, tau, low_logit, opacity_logits, nu, n_pruned);
}

void launch_gaussian_adam(int64_t n, const GaussianAdam& a, float* moments, uint32_t* step, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(gaussian_adam_kernel,
                       dim3((unsigned)(((11 + (int64_t)a.colour_width) * n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, n, a, moments, (const uint32_t*)step);
  hipLaunchKernelGGL(increment_kernel, dim3(1), dim3(1), 0, s, step);
}

void launch_pose_adam(int n_views, float* poses, float* dposes, float* adam, const AdamParams& ap, hipStream_t s) {
  hipLaunchKernelGGL(pose_adam_kernel, dim3((unsigned)n_views), dim3(64), 0, s, poses, dposes, adam, ap);
}

void launch_stats(const uint32_t* tiles, int64_t m, const uint4* pixel_state, const uint2* pixel_count,
                  int64_t pixels, const uint2* ranges, int64_t n_tiles, unsigned long long* out6, hipStream_t s) {
  hipLaunchKernelGGL(stats_kernel, dim3(256), dim3(kThreads), 0, s, tiles, m, pixel_state, pixel_count, pixels,
                     ranges, n_tiles, out6);
}

}  // namespace cgsr
