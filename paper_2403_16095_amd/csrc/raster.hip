// Tile blending, forward (Sec. 3.1 Eq. 3-9, Sec. 3.2 Eq. 10) and backward.
//
// One 256-lane workgroup per 16x16 tile, one pixel per lane; each wave owns
// an 8x8 quadrant so its lanes see nearby pixels and leave together.  The
// tile's depth-ordered records are staged through LDS 256 at a time (see
// stage_record); every lane then reads the same LDS address, a broadcast free
// of bank conflicts.  A pair below the skip threshold costs one base-2
// exponent and a compare; only blended pairs evaluate exp2.
//
// Tracking mode (kTrack) forms the gradient images of the tracking loss
// (Eq. 19: L1 colour, Eq. 14, and L1 depth, Eq. 16) at the end of the
// forward, straight from the blended values in registers, and keeps them in
// a per-pixel buffer for the backward instead of writing maps.
#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kThreads = kTilePixels;
constexpr int kBatch = 256;

struct PixelCoord {
  int px, py;
  bool inside;
};

__device__ __forceinline__ PixelCoord pixel_of_lane(const ViewInfo& cam, int gtile) {
  const int lt = gtile - cam.tile_base;
  const int tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  PixelCoord c;
  c.px = tx * kTile + (w & 1) * 8 + (l & 7);
  c.py = ty * kTile + (w >> 1) * 8 + (l >> 3);
  c.inside = c.px < cam.width && c.py < cam.height;
  return c;
}

__device__ __forceinline__ float sgn(float x) { return (float)((x > 0.f) - (x < 0.f)); }

template <bool kTrack>
__global__ __launch_bounds__(kThreads) void raster_forward_kernel(RasterBufs b) {
  __shared__ float4 sA[kBatch];
  __shared__ float4 sB[kBatch];
  __shared__ float4 sC[kBatch];
  const int gtile = blockIdx.x;
  const int v = view_of_tile(b.views, gtile);
  const ViewIO io = b.views.io[v];
  const ViewInfo cam = io.info;
  const PixelCoord pc = pixel_of_lane(cam, gtile);
  const int64_t pix = (int64_t)pc.py * cam.width + pc.px;
  const float dobs = (io.depth_obs && pc.inside) ? io.depth_obs[pix] : 0.f;
  const uint2 range = b.ranges[gtile];
  const float fx = (float)pc.px, fy = (float)pc.py;

  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, O = 0.f, U = 0.f, Dmed = 0.f;
  int med = -1;
  uint32_t last = 0, evaluated = range.y - range.x, blended = 0;
  bool done = !pc.inside;
  for (uint32_t base = range.x; base < range.y; base += kBatch) {
    const int n = (int)min((uint32_t)kBatch, range.y - base);
    __syncthreads();
    if ((int)threadIdx.x < n) {
      const uint32_t m = b.vals[base + threadIdx.x];
      stage_record(b.rec + (int64_t)kRecF4 * m, sA[threadIdx.x], sB[threadIdx.x], sC[threadIdx.x]);
    }
    __syncthreads();
    if (!done) {
      const uint32_t off = base - range.x;
      for (int j = 0; j < n; ++j) {
        const float4 A = sA[j];
        const float4 B = sB[j];
        float dx, dy;
        const float e = pair_exponent(A, B, fx, fy, dx, dy);
        if (e < B.w) continue;
        const float alpha = fminf(kAlphaMax, B.y * __builtin_amdgcn_exp2f(e));
        const float Tn = T * (1.f - alpha);
        if (Tn < kTStop) {
          done = true;
          evaluated = off + j + 1;
          break;
        }
        const float wgt = alpha * T;
        const float4 Cc = sC[j];
        C0 = __builtin_fmaf(wgt, Cc.x, C0);
        C1 = __builtin_fmaf(wgt, Cc.y, C1);
        C2 = __builtin_fmaf(wgt, Cc.z, C2);
        D = __builtin_fmaf(wgt, B.z, D);
        O += wgt;
        if (!kTrack) {
          const float dz = B.z - dobs;
          U = __builtin_fmaf(wgt * dz, dz, U);
        }
        if (med < 0 && Tn < kTMedian) {
          med = (int)(off + j);
          Dmed = B.z;
        }
        T = Tn;
        last = off + j + 1;
        ++blended;
      }
    }
    if (__syncthreads_count(done) == kThreads) break;
  }
  const int64_t hw = (int64_t)cam.width * cam.height;
  if (kTrack) {
    // dL/dcolour and dL/ddepth of L = lc mean_n |I^ - I|_1 + ld mean_n |D^ - D|.
    float l = 0.f;
    if (pc.inside) {
      const float inv = 1.0f / (float)hw;
      const float e0 = C0 - io.t_color[pix], e1 = C1 - io.t_color[hw + pix], e2 = C2 - io.t_color[2 * hw + pix];
      const float ed = D - io.t_depth[pix];
      const float lc = b.lambda_color * inv, ld = b.lambda_depth * inv;
      b.pixel_grad[cam.pixel_base + pix] = make_float4(lc * sgn(e0), lc * sgn(e1), lc * sgn(e2), ld * sgn(ed));
      l = lc * (fabsf(e0) + fabsf(e1) + fabsf(e2)) + ld * fabsf(ed);
    }
    if (b.loss) {
      const float t = wave_sum(l);
      if ((threadIdx.x & 63) == 0 && t != 0.f) atomicAdd(b.loss + v, t);
    }
  }
  if (!pc.inside) return;
  if (io.color) {
    io.color[pix] = C0;
    io.color[hw + pix] = C1;
    io.color[2 * hw + pix] = C2;
  }
  if (io.depth) io.depth[pix] = D;
  if (io.opacity) io.opacity[pix] = O;
  if (io.depth_median) io.depth_median[pix] = Dmed;
  if (io.uncertainty) io.uncertainty[pix] = U;
  b.pixel_state[cam.pixel_base + pix] = make_uint4(__float_as_uint(T), last, (uint32_t)med, evaluated);
  b.pixel_count[cam.pixel_base + pix] = blended;
}

// Back-to-front over each pixel's blended run.  With the normalised "behind"
// sums Bx = sum_{k>j} w_k x_k / T_{j+1}, dL/dalpha_j = T_j sum_x g_x (x_j - Bx),
// and Bx <- alpha_j x_j + (1 - alpha_j) Bx moves the sums one Gaussian forward;
// T_j = T_{j+1} / (1 - alpha_j) recovers the transmittance from the final one.
// kParams adds the opacity and colour gradients (mapping); kTrack takes the
// upstream gradients from the tracking forward (colour and depth only).
template <bool kParams, bool kTrack>
__global__ __launch_bounds__(kThreads) void raster_backward_kernel(RasterBufs b) {
  __shared__ float4 sA[kBatch];
  __shared__ float4 sB[kBatch];
  __shared__ float4 sC[kBatch];
  __shared__ uint32_t sM[kBatch];
  __shared__ uint32_t s_max;
  const int gtile = blockIdx.x;
  const int v = view_of_tile(b.views, gtile);
  const ViewIO io = b.views.io[v];
  const ViewInfo cam = io.info;
  const PixelCoord pc = pixel_of_lane(cam, gtile);
  const int64_t pix = (int64_t)pc.py * cam.width + pc.px;
  const int64_t hw = (int64_t)cam.width * cam.height;
  const uint2 range = b.ranges[gtile];
  const int lane = threadIdx.x & 63;

  float T = 1.f;
  uint32_t walked = 0;
  int med = -1;
  float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gd = 0.f, go = 0.f, gm = 0.f, gu = 0.f, dobs = 0.f;
  if (pc.inside) {
    const uint4 ps = b.pixel_state[cam.pixel_base + pix];
    T = __uint_as_float(ps.x);
    walked = ps.y;
    med = (int)ps.z;
    if (kTrack) {
      const float4 g4 = b.pixel_grad[cam.pixel_base + pix];
      gc0 = g4.x;
      gc1 = g4.y;
      gc2 = g4.z;
      gd = g4.w;
    } else {
      if (io.g_color) {
        gc0 = io.g_color[pix];
        gc1 = io.g_color[hw + pix];
        gc2 = io.g_color[2 * hw + pix];
      }
      if (io.g_depth) gd = io.g_depth[pix];
      if (io.g_opacity) go = io.g_opacity[pix];
      if (io.g_median) gm = io.g_median[pix];
      if (io.g_uncertainty) gu = io.g_uncertainty[pix];
      if (io.depth_obs) dobs = io.depth_obs[pix];
    }
  }
  if (threadIdx.x == 0) s_max = 0u;
  __syncthreads();
  if (walked) atomicMax(&s_max, walked);
  __syncthreads();
  const int nmax = (int)s_max;
  const float fx = (float)pc.px, fy = (float)pc.py;

  float Bc0 = 0.f, Bc1 = 0.f, Bc2 = 0.f, Bd = 0.f, Bo = 0.f, Bu = 0.f;
  for (int end = nmax; end > 0; end -= kBatch) {
    const int start = max(0, end - kBatch);
    const int n = end - start;
    __syncthreads();
    if ((int)threadIdx.x < n) {
      const uint32_t m = b.vals[range.x + start + threadIdx.x];
      sM[threadIdx.x] = m;
      stage_record(b.rec + (int64_t)kRecF4 * m, sA[threadIdx.x], sB[threadIdx.x], sC[threadIdx.x]);
    }
    __syncthreads();
    for (int j = n - 1; j >= 0; --j) {
      const int pos = start + j;
      const float4 A = sA[j];
      const float4 B = sB[j];
      float dx, dy;
      const float e = pair_exponent(A, B, fx, fy, dx, dy);
      const bool active = pos < (int)walked && e >= B.w;
      float gmx = 0.f, gmy = 0.f, ga = 0.f, gb = 0.f, gcc = 0.f, gop = 0.f, gdd = 0.f;
      float gr = 0.f, gg = 0.f, gbl = 0.f;
      if (active) {
        const float4 Cc = sC[j];
        const float g = __builtin_amdgcn_exp2f(e);
        const float raw = B.y * g;
        const float alpha = fminf(kAlphaMax, raw);
        const float oma = 1.f - alpha;
        const float Tj = T * __builtin_amdgcn_rcpf(oma);
        const float wgt = alpha * Tj;
        float dsum = gc0 * (Cc.x - Bc0) + gc1 * (Cc.y - Bc1) + gc2 * (Cc.z - Bc2) + gd * (B.z - Bd);
        Bc0 = __builtin_fmaf(alpha, Cc.x, oma * Bc0);
        Bc1 = __builtin_fmaf(alpha, Cc.y, oma * Bc1);
        Bc2 = __builtin_fmaf(alpha, Cc.z, oma * Bc2);
        Bd = __builtin_fmaf(alpha, B.z, oma * Bd);
        float dz = 0.f;
        if (!kTrack) {
          dz = B.z - dobs;
          const float u = dz * dz;
          dsum += go * (1.f - Bo) + gu * (u - Bu);
          Bo = __builtin_fmaf(alpha, 1.f, oma * Bo);
          Bu = __builtin_fmaf(alpha, u, oma * Bu);
        }
        const float dalpha = Tj * dsum;
        T = Tj;
        const bool capped = raw > kAlphaMax;
        const float dpower = capped ? 0.f : dalpha * raw;   // alpha = opacity * exp(power)
        // power = -(a dx^2 + 2 b dx dy + c dy^2) / 2, with the staged
        // qa = -a/2 log2 e etc.: d power/d mu = ln2 (2 qa dx + qb dy, qb dx + 2 qc dy)
        gmx = dpower * kLn2 * __builtin_fmaf(2.f * A.z, dx, A.w * dy);
        gmy = dpower * kLn2 * __builtin_fmaf(A.w, dx, 2.f * B.x * dy);
        ga = -0.5f * dpower * dx * dx;
        gb = -dpower * dx * dy;
        gcc = -0.5f * dpower * dy * dy;
        gdd = wgt * gd;
        if (!kTrack) gdd += 2.f * wgt * dz * gu + (pos == med ? gm : 0.f);
        if (kParams) {
          gop = capped ? 0.f : dalpha * g;
          gr = wgt * gc0;
          gg = wgt * gc1;
          gbl = wgt * gc2;
        }
      }
      if (__ballot(active)) {
        const uint32_t m = sM[j];
        float* dst = b.rec_grad + (int64_t)kGradStride * m;
        const float s0 = wave_sum(gmx), s1 = wave_sum(gmy), s2 = wave_sum(ga), s3 = wave_sum(gb);
        const float s4 = wave_sum(gcc), s6 = wave_sum(gdd);
        if (kParams) {
          const float s5 = wave_sum(gop), s7 = wave_sum(gr), s8 = wave_sum(gg), s9 = wave_sum(gbl);
          float val = s0;
          val = lane == 1 ? s1 : val;
          val = lane == 2 ? s2 : val;
          val = lane == 3 ? s3 : val;
          val = lane == 4 ? s4 : val;
          val = lane == 5 ? s5 : val;
          val = lane == 6 ? s6 : val;
          val = lane == 7 ? s7 : val;
          val = lane == 8 ? s8 : val;
          val = lane == 9 ? s9 : val;
          if (lane < 10) unsafeAtomicAdd(dst + lane, val);
        } else {
          float val = s0;
          val = lane == 1 ? s1 : val;
          val = lane == 2 ? s2 : val;
          val = lane == 3 ? s3 : val;
          val = lane == 4 ? s4 : val;
          val = lane == 5 ? s6 : val;
          if (lane < 6) unsafeAtomicAdd(dst + (lane == 5 ? 6 : lane), val);
        }
      }
    }
  }
}

}  // namespace

void launch_raster_forward(const RasterBufs& b, bool track, hipStream_t s) {
  if (b.total_tiles <= 0) return;
  if (track)
    hipLaunchKernelGGL(raster_forward_kernel<true>, dim3(b.total_tiles), dim3(kThreads), 0, s, b);
  else
    hipLaunchKernelGGL(raster_forward_kernel<false>, dim3(b.total_tiles), dim3(kThreads), 0, s, b);
}

void launch_raster_backward(const RasterBufs& b, bool param_grads, bool track, hipStream_t s) {
  if (b.total_tiles <= 0) return;
  if (track)
    hipLaunchKernelGGL((raster_backward_kernel<false, true>), dim3(b.total_tiles), dim3(kThreads), 0, s, b);
  else if (param_grads)
    hipLaunchKernelGGL((raster_backward_kernel<true, false>), dim3(b.total_tiles), dim3(kThreads), 0, s, b);
  else
    hipLaunchKernelGGL((raster_backward_kernel<false, false>), dim3(b.total_tiles), dim3(kThreads), 0, s, b);
}

}  // namespace cgsr
