// Sequential-tracking glue kept on the device so a whole tracking iteration
// can be replayed from a HIP graph: gradient images of the tracking loss
// (Eq. 19 from Eq. 14 and 16) and the Adam step plus retraction on the pose
// (Eq. 20).  Also the counters behind cgsr_get_stats.
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

// One lane per view.  Adam on the tangent vector xi = (rho, phi) whose value is
// zero at the current pose, so the step is delta = -lr m_hat / (sqrt(v_hat) + eps);
// then T <- exp(delta^) T with the closed-form SE(3) exponential.
__global__ void pose_adam_kernel(int n_views, float* poses, float* dposes, float* adam, float lr_rho, float lr_phi,
                                 float b1, float b2, float eps) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_views) return;
  float* st = adam + 16 * v;
  const float step = st[12] + 1.f;
  st[12] = step;
  const float c1 = 1.f - powf(b1, step), c2 = 1.f - powf(b2, step);
  float d[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float g = dposes[6 * v + k];
    dposes[6 * v + k] = 0.f;
    const float m = b1 * st[k] + (1.f - b1) * g;
    const float s = b2 * st[6 + k] + (1.f - b2) * g * g;
    st[k] = m;
    st[6 + k] = s;
    const float lr = k < 3 ? lr_rho : lr_phi;
    d[k] = -lr * (m / c1) / (sqrtf(s / c2) + eps);
  }
  // exp of (rho, phi): R = I + A K + B K^2, V = I + B K + C K^2, K = [phi]x.
  const float p0 = d[3], p1 = d[4], p2 = d[5];
  const float th2 = p0 * p0 + p1 * p1 + p2 * p2;
  float A, Bc, Cc;
  if (th2 < 1e-8f) {
    A = 1.f - th2 / 6.f;
    Bc = 0.5f - th2 / 24.f;
    Cc = 1.f / 6.f - th2 / 120.f;
  } else {
    const float th = sqrtf(th2);
    A = sinf(th) / th;
    Bc = (1.f - cosf(th)) / th2;
    Cc = (th - sinf(th)) / (th2 * th);
  }
  const float K[9] = {0.f, -p2, p1, p2, 0.f, -p0, -p1, p0, 0.f};
  float K2[9], R[9], V[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) K2[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float I = (k % 4 == 0) ? 1.f : 0.f;
    R[k] = I + A * K[k] + Bc * K2[k];
    V[k] = I + Bc * K[k] + Cc * K2[k];
  }
  float* P = poses + 12 * v;
  float Rn[9], tn[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) Rn[3 * r + c] = R[3 * r] * P[c] + R[3 * r + 1] * P[3 + c] + R[3 * r + 2] * P[6 + c];
    tn[r] = R[3 * r] * P[9] + R[3 * r + 1] * P[10] + R[3 * r + 2] * P[11] + V[3 * r] * d[0] + V[3 * r + 1] * d[1] +
            V[3 * r + 2] * d[2];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) P[k] = Rn[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) P[9 + k] = tn[k];
}

__global__ __launch_bounds__(kThreads) void stats_kernel(const uint32_t* __restrict__ tiles, int64_t m,
                                                         const uint4* __restrict__ ps,
                                                         const uint32_t* __restrict__ count, int64_t pixels,
                                                         unsigned long long* out) {
  unsigned long long vis = 0, ev = 0, bl = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < m; i += (int64_t)gridDim.x * kThreads)
    vis += tiles[i] != 0u;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < pixels; i += (int64_t)gridDim.x * kThreads) {
    ev += ps[i].w;
    bl += count[i];
  }
  // These counters are read rarely; one atomic per lane keeps the code short.
  if (vis) atomicAdd(out, vis);
  if (ev) atomicAdd(out + 1, ev);
  if (bl) atomicAdd(out + 2, bl);
}

}  // namespace

void launch_tracking_loss(int w, int h, const float* color, const float* depth, const float* tcolor,
                          const float* tdepth, float lc, float ld, float* dcolor, float* ddepth, float* loss,
                          hipStream_t s) {
  const int64_t hw = (int64_t)w * h;
  hipLaunchKernelGGL(tracking_loss_kernel, dim3((unsigned)((hw + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     w, h, color, depth, tcolor, tdepth, lc, ld, dcolor, ddepth, loss);
}

void launch_pose_adam(int n_views, float* poses, float* dposes, float* adam, float lr_rho, float lr_phi, float b1,
                      float b2, float eps, hipStream_t s) {
  hipLaunchKernelGGL(pose_adam_kernel, dim3(1), dim3(64), 0, s, n_views, poses, dposes, adam, lr_rho, lr_phi, b1,
                     b2, eps);
}

void launch_stats(const uint32_t* tiles, int64_t m, const uint4* pixel_state, const uint32_t* pixel_count,
                  int64_t pixels, unsigned long long* out3, hipStream_t s) {
  hipLaunchKernelGGL(stats_kernel, dim3(256), dim3(kThreads), 0, s, tiles, m, pixel_state, pixel_count, pixels,
                     out3);
}

}  // namespace cgsr
