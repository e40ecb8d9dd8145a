// The mapping objective, Eq. 18: per-pixel gradient images of its image
// terms and the per-Gaussian gradient of its scale term.
//
//   colour L1 (Eq. 14), depth L1 (Eq. 16), alpha-depth / median-depth
//   alignment (Eq. 12, pixels that have a median), geometry variance
//   mean |U| (Eq. 11)                          -> objective_pixel_kernel
//   1 - SSIM (Eq. 15): 11x11 Gaussian window (sigma 1.5), zero padding,
//   C1 = 0.01^2, C2 = 0.03^2, mean over channels and pixels
//                                              -> ssim_forward_kernel,
//                                                 ssim_backward_kernel
//   isotropy (Eq. 17) over the view's visible Gaussians
//                                              -> iso_count_kernel,
//                                                 iso_grad_kernel
//
// SSIM is a separable stencil: both SSIM kernels stage a 26x26 halo tile of
// their inputs in LDS (zero outside the image), run the 11 horizontal taps
// into LDS and then the 11 vertical taps per output pixel.  The forward
// keeps, per pixel and channel, the derivatives of the local SSIM value S
// with respect to the local moments mu_x, E[x^2] and E[xy]; the gradient
// with respect to pixel p is then the same window applied to those three
// maps (the window is symmetric, so the adjoint is the window itself):
//   dS_mean/dx_p = (1/N) [G*P1 + 2 x_p G*P2 + y_p G*P3](p).
#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kT = 16;            // output tile edge
constexpr int kR = 5;             // window radius (11 taps)
constexpr int kE = kT + 2 * kR;   // staged edge with halo
constexpr int kThreads = kT * kT;
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

// Normalised 11-tap Gaussian of standard deviation 1.5, computed on the host
// in double and passed by value.
struct Window {
  float w[2 * kR + 1];
};

__device__ __forceinline__ float sgn(float x) { return (float)((x > 0.f) - (x < 0.f)); }

__device__ __forceinline__ float block_sum(float v, float* s_part) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = 0.f;
  if (threadIdx.x == 0)
    for (int k = 0; k < kThreads / 64; ++k) t += s_part[k];
  return t;
}

// Gradient images of the L1, alignment and variance terms (written, not
// added) and their losses.  Also adds the constant w_ssim of 1 - SSIM.
__global__ __launch_bounds__(kThreads) void objective_pixel_kernel(
    int w, int h, const float* __restrict__ color, const float* __restrict__ depth,
    const float* __restrict__ median, const float* __restrict__ unc, const float* __restrict__ tcolor,
    const float* __restrict__ tdepth, float w_color, float w_geo, float w_align, float w_var, float w_ssim,
    float* __restrict__ dcolor, float* __restrict__ ddepth, float* __restrict__ dmedian,
    float* __restrict__ dunc, float* loss) {
  __shared__ float s_part[kThreads / 64];
  const int64_t hw = (int64_t)w * h;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const float inv = 1.0f / (float)hw;
  float l = 0.f;
  if (i < hw) {
    if (dcolor) {
      float lc = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float e = color[c * hw + i] - tcolor[c * hw + i];
        dcolor[c * hw + i] = w_color * inv * sgn(e);
        lc += fabsf(e);
      }
      l += w_color * lc;
    }
    float gd = 0.f;
    if (ddepth) {
      const float eg = depth[i] - tdepth[i];
      gd = w_geo * inv * sgn(eg);
      l += w_geo * fabsf(eg);
    }
    if (median) {
      // a pixel without a median Gaussian (median depth 0) adds nothing
      const float Dm = median[i];
      const float ea = Dm > 0.f ? depth[i] - Dm : 0.f;
      gd += w_align * inv * sgn(ea);
      if (dmedian) dmedian[i] = -w_align * inv * sgn(ea);
      l += w_align * fabsf(ea);
    }
    if (ddepth) ddepth[i] = gd;
    if (dunc) {
      const float U = unc[i];
      dunc[i] = w_var * inv * sgn(U);
      l += w_var * fabsf(U);
    }
    l *= inv;
  }
  if (!loss) return;
  float t = block_sum(l, s_part);
  if (threadIdx.x == 0) {
    if (blockIdx.x == 0) t += w_ssim;
    if (t != 0.f) atomicAdd(loss, t);
  }
}

// Stage a kE x kE tile of a plane (origin ox - kR, oy - kR), zero outside.
__device__ __forceinline__ void stage_plane(const float* __restrict__ src, int w, int h, int ox, int oy,
                                            float (*dst)[kE]) {
  for (int k = threadIdx.x; k < kE * kE; k += kThreads) {
    const int ly = k / kE, lx = k % kE;
    const int gx = ox - kR + lx, gy = oy - kR + ly;
    dst[ly][lx] = (gx >= 0 && gx < w && gy >= 0 && gy < h) ? src[(int64_t)gy * w + gx] : 0.f;
  }
}

// blockIdx.z = channel.  Writes P1 = dS/dmu_x, P2 = dS/dE[x^2], P3 = dS/dE[xy]
// into part[(3c + k) * hw + pixel] and adds -w_ssim * sum S / N to *loss.
__global__ __launch_bounds__(kThreads) void ssim_forward_kernel(int w, int h, const float* __restrict__ x,
                                                                const float* __restrict__ y, Window win,
                                                                float w_ssim, float* __restrict__ part,
                                                                float* loss) {
  __shared__ float sx[kE][kE];
  __shared__ float sy[kE][kE];
  __shared__ float hsum[5][kE][kT];
  __shared__ float s_part[kThreads / 64];
  const int64_t hw = (int64_t)w * h;
  const int c = blockIdx.z;
  const int ox = blockIdx.x * kT, oy = blockIdx.y * kT;
  stage_plane(x + c * hw, w, h, ox, oy, sx);
  stage_plane(y + c * hw, w, h, ox, oy, sy);
  __syncthreads();
  for (int k = threadIdx.x; k < kE * kT; k += kThreads) {
    const int ly = k / kT, lx = k % kT;
    float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
    for (int t = 0; t < 2 * kR + 1; ++t) {
      const float xv = sx[ly][lx + t], yv = sy[ly][lx + t], g = win.w[t];
      a = __builtin_fmaf(g, xv, a);
      b = __builtin_fmaf(g, yv, b);
      aa = __builtin_fmaf(g, xv * xv, aa);
      bb = __builtin_fmaf(g, yv * yv, bb);
      ab = __builtin_fmaf(g, xv * yv, ab);
    }
    hsum[0][ly][lx] = a;
    hsum[1][ly][lx] = b;
    hsum[2][ly][lx] = aa;
    hsum[3][ly][lx] = bb;
    hsum[4][ly][lx] = ab;
  }
  __syncthreads();
  const int tx = threadIdx.x % kT, ty = threadIdx.x / kT;
  float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
  for (int t = 0; t < 2 * kR + 1; ++t) {
    const float g = win.w[t];
    mx = __builtin_fmaf(g, hsum[0][ty + t][tx], mx);
    my = __builtin_fmaf(g, hsum[1][ty + t][tx], my);
    exx = __builtin_fmaf(g, hsum[2][ty + t][tx], exx);
    eyy = __builtin_fmaf(g, hsum[3][ty + t][tx], eyy);
    exy = __builtin_fmaf(g, hsum[4][ty + t][tx], exy);
  }
  const int px = ox + tx, py = oy + ty;
  float S = 0.f;
  if (px < w && py < h) {
    const float a1 = 2.f * mx * my + kC1;
    const float a2 = 2.f * (exy - mx * my) + kC2;
    const float b1 = mx * mx + my * my + kC1;
    const float b2 = (exx - mx * mx) + (eyy - my * my) + kC2;
    S = (a1 * a2) / (b1 * b2);
    const float p1 = S * (2.f * my / a1 - 2.f * my / a2 - 2.f * mx / b1 + 2.f * mx / b2);
    const float p2 = -S / b2;
    const float p3 = 2.f * S / a2;
    const int64_t q = (int64_t)py * w + px;
    part[(3 * c + 0) * hw + q] = p1;
    part[(3 * c + 1) * hw + q] = p2;
    part[(3 * c + 2) * hw + q] = p3;
  }
  if (!loss) return;
  const float t = block_sum(S, s_part);
  if (threadIdx.x == 0 && t != 0.f) atomicAdd(loss, -w_ssim * t / (3.f * (float)hw));
}

// dcolor += -w_ssim / N (G*P1 + 2 x G*P2 + y G*P3), N = 3 H W.
__global__ __launch_bounds__(kThreads) void ssim_backward_kernel(int w, int h, const float* __restrict__ x,
                                                                 const float* __restrict__ y, Window win,
                                                                 float w_ssim, const float* __restrict__ part,
                                                                 float* __restrict__ dcolor) {
  __shared__ float sp[3][kE][kE];
  __shared__ float hsum[3][kE][kT];
  const int64_t hw = (int64_t)w * h;
  const int c = blockIdx.z;
  const int ox = blockIdx.x * kT, oy = blockIdx.y * kT;
#pragma unroll
  for (int k = 0; k < 3; ++k) stage_plane(part + (3 * c + k) * hw, w, h, ox, oy, sp[k]);
  __syncthreads();
  for (int k = threadIdx.x; k < kE * kT; k += kThreads) {
    const int ly = k / kT, lx = k % kT;
    float a = 0.f, b = 0.f, d = 0.f;
#pragma unroll
    for (int t = 0; t < 2 * kR + 1; ++t) {
      const float g = win.w[t];
      a = __builtin_fmaf(g, sp[0][ly][lx + t], a);
      b = __builtin_fmaf(g, sp[1][ly][lx + t], b);
      d = __builtin_fmaf(g, sp[2][ly][lx + t], d);
    }
    hsum[0][ly][lx] = a;
    hsum[1][ly][lx] = b;
    hsum[2][ly][lx] = d;
  }
  __syncthreads();
  const int tx = threadIdx.x % kT, ty = threadIdx.x / kT;
  const int px = ox + tx, py = oy + ty;
  if (px >= w || py >= h) return;
  float g1 = 0.f, g2 = 0.f, g3 = 0.f;
#pragma unroll
  for (int t = 0; t < 2 * kR + 1; ++t) {
    const float g = win.w[t];
    g1 = __builtin_fmaf(g, hsum[0][ty + t][tx], g1);
    g2 = __builtin_fmaf(g, hsum[1][ty + t][tx], g2);
    g3 = __builtin_fmaf(g, hsum[2][ty + t][tx], g3);
  }
  const int64_t q = (int64_t)py * w + px;
  const float xv = x[c * hw + q], yv = y[c * hw + q];
  const float dS = g1 + 2.f * xv * g2 + yv * g3;
  dcolor[c * hw + q] += -w_ssim * dS / (3.f * (float)hw);
}

// Visible Gaussians per view: those whose binning rectangle reaches the image
// (tiles[m] > 0 for record m = view * N + i).
__global__ __launch_bounds__(kThreads) void iso_count_kernel(int64_t n, const uint32_t* __restrict__ tiles,
                                                             uint32_t* counts) {
  __shared__ uint32_t s_part[kThreads / 64];
  const int v = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool vis = i < n && tiles[(int64_t)v * n + i] != 0u;
  const uint64_t mask = __ballot(vis);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = (uint32_t)__popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < kThreads / 64; ++k) t += s_part[k];
    if (t) atomicAdd(counts + v, t);
  }
}

// Eq. 17: r = max s / min s = exp(max l - min l) (first axis on ties);
// the term is max(r, eps) - eps, its gradient r (e_max - e_min) when r > eps.
__global__ __launch_bounds__(kThreads) void iso_grad_kernel(int64_t n, const uint32_t* __restrict__ tiles,
                                                            const uint32_t* __restrict__ counts,
                                                            const float* __restrict__ log_scales, float w_iso,
                                                            float eps, float* dlog_scales, float* loss) {
  __shared__ float s_part[kThreads / 64];
  const int v = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const uint32_t cnt = counts[v];
  float l = 0.f;
  if (i < n && cnt && tiles[(int64_t)v * n + i] != 0u) {
    const float l0 = log_scales[3 * i], l1 = log_scales[3 * i + 1], l2 = log_scales[3 * i + 2];
    int imax = 0, imin = 0;
    float vmax = l0, vmin = l0;
    if (l1 > vmax) { vmax = l1; imax = 1; }
    if (l2 > vmax) { vmax = l2; imax = 2; }
    if (l1 < vmin) { vmin = l1; imin = 1; }
    if (l2 < vmin) { vmin = l2; imin = 2; }
    const float r = expf(vmax - vmin);
    const float scale = w_iso / (float)cnt;
    l = scale * (fmaxf(r, eps) - eps);
    if (dlog_scales && r > eps && imax != imin) {
      unsafeAtomicAdd(dlog_scales + 3 * i + imax, scale * r);
      unsafeAtomicAdd(dlog_scales + 3 * i + imin, -scale * r);
    }
  }
  if (!loss) return;
  const float t = block_sum(l, s_part);
  if (threadIdx.x == 0 && t != 0.f) atomicAdd(loss + v, t);
}

Window make_window() {
  Window win;
  double g[2 * kR + 1], s = 0.0;
  for (int t = 0; t <= 2 * kR; ++t) {
    const double d = t - kR;
    g[t] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    s += g[t];
  }
  for (int t = 0; t <= 2 * kR; ++t) win.w[t] = (float)(g[t] / s);
  return win;
}

}  // namespace

void launch_objective_view(const ObjectiveView& o, const ObjectiveWeights& wt, float* ssim_part, hipStream_t s) {
  const int64_t hw = (int64_t)o.width * o.height;
  if (hw <= 0) return;
  hipLaunchKernelGGL(objective_pixel_kernel, dim3((unsigned)((hw + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     o.width, o.height, o.color, o.depth, o.median, o.unc, o.tcolor, o.tdepth, wt.color, wt.geo,
                     wt.align, wt.var, o.dcolor ? wt.ssim : 0.f, o.dcolor, o.ddepth, o.dmedian, o.dunc, o.loss);
  if (o.dcolor && wt.ssim != 0.f) {
    const Window win = make_window();
    const dim3 grid((o.width + kT - 1) / kT, (o.height + kT - 1) / kT, 3);
    hipLaunchKernelGGL(ssim_forward_kernel, grid, dim3(kThreads), 0, s, o.width, o.height, o.color, o.tcolor, win,
                       wt.ssim, ssim_part, o.loss);
    hipLaunchKernelGGL(ssim_backward_kernel, grid, dim3(kThreads), 0, s, o.width, o.height, o.color, o.tcolor, win,
                       wt.ssim, ssim_part, o.dcolor);
  }
}

void launch_iso(int64_t n, int n_views, const uint32_t* tiles, uint32_t* counts, const float* log_scales, float w_iso,
                float eps, float* dlog_scales, float* loss, hipStream_t s) {
  launch_clear_u32(counts, n_views, s);
  if (n <= 0) return;
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads), n_views);
  hipLaunchKernelGGL(iso_count_kernel, grid, dim3(kThreads), 0, s, n, tiles, counts);
  hipLaunchKernelGGL(iso_grad_kernel, grid, dim3(kThreads), 0, s, n, tiles, counts, log_scales, w_iso, eps,
                     dlog_scales, loss);
}

}  // namespace cgsr
