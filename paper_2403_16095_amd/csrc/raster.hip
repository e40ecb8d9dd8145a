// Tile blending, forward (Sec. 3.1 Eq. 3-9, Sec. 3.2 Eq. 10) and backward.
//
// One workgroup per 16x16 tile.  A lane owns kPPL pixels (1, 2 or 4), so a
// tile takes 256 / kPPL lanes; pixel q of the tile lies in the 8x8 quadrant
// q / 64, and lane t owns pixels t, t + L, t + 2L, ... (L lanes), so a wave's
// pixels are whole quadrants and leave together.  The tile's depth-ordered
// records are staged through LDS 256 at a time (see stage_record); every lane
// then reads the same LDS address, a broadcast free of bank conflicts, and
// uses it for all of its pixels.  A pair below the skip threshold costs one
// base-2 exponent and a compare; only blended pairs evaluate exp2.
//
// kNu (mapping renders) also keeps, per pixel, the blended Gaussian of
// largest weight alpha T -- the pixel is "dominated" by it (Sec. 3.2,
// Eq. 13) -- and at the end adds w (D - d)^2 and 1 to that Gaussian's
// uncertainty sum and count when the pixel has a sensor depth D > 0.
//
// Tracking mode (kTrack) forms the gradient images of the tracking loss
// (Eq. 19: L1 colour, Eq. 14, and L1 depth, Eq. 16) at the end of the
// forward, straight from the blended values in registers, and keeps them in
// a per-pixel buffer for the backward instead of writing maps.
#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kBatch = 256;
constexpr uint32_t kNone = 0xffffffffu;

struct PixelCoord {
  int px, py;   // absolute pixel
  int ox, oy;   // tile origin
  bool inside;
};

// Pixel q (0..255) of tile gtile: quadrant q / 64, row-major 8x8 inside it.
__device__ __forceinline__ PixelCoord pixel_of(const ViewInfo& cam, int gtile, int q) {
  const int lt = gtile - cam.tile_base;
  const int tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
  const int w = q >> 6, l = q & 63;
  PixelCoord c;
  c.ox = tx * kTile;
  c.oy = ty * kTile;
  c.px = c.ox + (w & 1) * 8 + (l & 7);
  c.py = c.oy + (w >> 1) * 8 + (l >> 3);
  c.inside = c.px < cam.width && c.py < cam.height;
  return c;
}

__device__ __forceinline__ float2 tile_origin(const ViewInfo& cam, int gtile) {
  const int lt = gtile - cam.tile_base;
  return make_float2((float)((lt % cam.tiles_x) * kTile), (float)((lt / cam.tiles_x) * kTile));
}

__device__ __forceinline__ float sgn(float x) { return (float)((x > 0.f) - (x < 0.f)); }

template <int kPPL, bool kTrack, bool kNu>
__global__ __launch_bounds__(kTilePixels / kPPL) void raster_forward_kernel(RasterBufs b) {
  constexpr int L = kTilePixels / kPPL;
  __shared__ float4 sA[kBatch];
  __shared__ float4 sB[kBatch];
  __shared__ float4 sC[kBatch];
  __shared__ uint32_t sM[kNu ? kBatch : 1];
  const int gtile = blockIdx.x;
  const int v = view_of_tile(b.views, gtile);
  const ViewIO io = b.views.io[v];
  const ViewInfo cam = io.info;
  const float2 org = tile_origin(cam, gtile);
  const uint2 range = b.ranges[gtile];
  const int64_t hw = (int64_t)cam.width * cam.height;

  float fx[kPPL], fy[kPPL], dobs[kPPL], T[kPPL], C0[kPPL], C1[kPPL], C2[kPPL], D[kPPL], O[kPPL], U[kPPL],
      Dmed[kPPL];
  int64_t pix[kPPL];
  int med[kPPL];
  uint32_t last[kPPL], evaluated[kPPL], blended[kPPL];
  float wdom[kPPL], ddom[kPPL];   // kNu: largest weight so far and its depth
  uint32_t dom[kPPL];             // kNu: its record id, kNone if none
  bool inside[kPPL], done[kPPL];
  bool lane_done = true;
#pragma unroll
  for (int k = 0; k < kPPL; ++k) {
    const PixelCoord pc = pixel_of(cam, gtile, k * L + threadIdx.x);
    fx[k] = (float)(pc.px - pc.ox);
    fy[k] = (float)(pc.py - pc.oy);
    inside[k] = pc.inside;
    pix[k] = (int64_t)pc.py * cam.width + pc.px;
    dobs[k] = (!kTrack && io.depth_obs && pc.inside) ? io.depth_obs[pix[k]] : 0.f;
    T[k] = 1.f;
    C0[k] = C1[k] = C2[k] = D[k] = O[k] = U[k] = Dmed[k] = 0.f;
    med[k] = -1;
    last[k] = 0;
    blended[k] = 0;
    wdom[k] = ddom[k] = 0.f;
    dom[k] = kNone;
    evaluated[k] = range.y - range.x;
    done[k] = !pc.inside;
    lane_done = lane_done && done[k];
  }
  for (uint32_t base = range.x; base < range.y; base += kBatch) {
    const int n = (int)min((uint32_t)kBatch, range.y - base);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += L) {
      const uint32_t m = b.vals[base + i];
      if (kNu) sM[i] = m;
      stage_record(b.rec + (int64_t)kRecF4 * m, org.x, org.y, sA[i], sB[i], sC[i]);
    }
    __syncthreads();
    // The wave walks the whole batch while any of its lanes still blends;
    // lanes that are done ride along predicated off.  (A vote every few
    // records to leave early cost more issue slots than it saved: at tracking
    // sizes most pixels never reach the stop threshold.)
    if (__ballot(!lane_done) != 0ull) {
      const uint32_t off = base - range.x;
      for (int j = 0; j < n; ++j) {
        const float4 A = sA[j];
        const float4 B = sB[j];
        const float4 Cc = sC[j];
        // Straight-line, predicated per lane: a lane that skips (alpha below
        // 1/255, or already done) adds exact zeros, so the results are those
        // of the branching form, without exec-mask bookkeeping per record.
#pragma unroll
        for (int k = 0; k < kPPL; ++k) {
          float dx, dy, tq;
          const float e = pair_exponent(A, B, fx[k], fy[k], dx, dy, tq);
          const bool hit = !done[k] && e >= B.w;
          const float alpha = fminf(kAlphaMax, B.y * __builtin_amdgcn_exp2f(e));
          const float Tn = T[k] * (1.f - alpha);
          const bool stop = hit && Tn < kTStop;
          const bool blend = hit && !stop;
          done[k] = done[k] || stop;
          evaluated[k] = stop ? off + j + 1 : evaluated[k];
          const float wgt = blend ? alpha * T[k] : 0.f;
          C0[k] = __builtin_fmaf(wgt, Cc.x, C0[k]);
          C1[k] = __builtin_fmaf(wgt, Cc.y, C1[k]);
          C2[k] = __builtin_fmaf(wgt, Cc.z, C2[k]);
          D[k] = __builtin_fmaf(wgt, B.z, D[k]);
          O[k] += wgt;
          if (!kTrack) {
            const float dz = B.z - dobs[k];
            U[k] = __builtin_fmaf(wgt * dz, dz, U[k]);
          }
          const bool first_med = blend && med[k] < 0 && Tn < kTMedian;
          med[k] = first_med ? (int)(off + j) : med[k];
          Dmed[k] = first_med ? B.z : Dmed[k];
          if (kNu) {
            const bool more = blend && wgt > wdom[k];   // strict: the first of equal maxima
            wdom[k] = more ? wgt : wdom[k];
            ddom[k] = more ? B.z : ddom[k];
            dom[k] = more ? sM[j] : dom[k];
          }
          T[k] = blend ? Tn : T[k];
          last[k] = blend ? off + j + 1 : last[k];
          blended[k] += blend ? 1u : 0u;
        }
      }
      bool all = true;
#pragma unroll
      for (int k = 0; k < kPPL; ++k) all = all && done[k];
      lane_done = all;
    }
    if (__syncthreads_count(lane_done) == L) break;
  }
  if (kTrack) {
    // dL/dcolour and dL/ddepth of L = lc mean_n |I^ - I|_1 + ld mean_n |D^ - D|.
    float l = 0.f;
    const float inv = 1.0f / (float)hw;
    const float lc = b.lambda_color * inv, ld = b.lambda_depth * inv;
#pragma unroll
    for (int k = 0; k < kPPL; ++k) {
      if (!inside[k]) continue;
      const int64_t p = pix[k];
      const float e0 = C0[k] - io.t_color[p], e1 = C1[k] - io.t_color[hw + p], e2 = C2[k] - io.t_color[2 * hw + p];
      const float ed = D[k] - io.t_depth[p];
      b.pixel_grad[cam.pixel_base + p] = make_float4(lc * sgn(e0), lc * sgn(e1), lc * sgn(e2), ld * sgn(ed));
      l += lc * (fabsf(e0) + fabsf(e1) + fabsf(e2)) + ld * fabsf(ed);
    }
    if (b.loss) {
      const float t = wave_sum(l);
      if ((threadIdx.x & 63) == 0 && t != 0.f) atomicAdd(b.loss + v, t);
    }
  }
#pragma unroll
  for (int k = 0; k < kPPL; ++k) {
    if (!inside[k]) continue;
    const int64_t p = pix[k];
    if (io.color) {
      io.color[p] = C0[k];
      io.color[hw + p] = C1[k];
      io.color[2 * hw + p] = C2[k];
    }
    if (io.depth) io.depth[p] = D[k];
    if (io.opacity) io.opacity[p] = O[k];
    if (io.depth_median) io.depth_median[p] = Dmed[k];
    if (io.uncertainty) io.uncertainty[p] = U[k];
    b.pixel_state[cam.pixel_base + p] = make_uint4(__float_as_uint(T[k]), last[k], (uint32_t)med[k], evaluated[k]);
    b.pixel_count[cam.pixel_base + p] = blended[k];
    if (kNu) {
      // record id m = view * N + Gaussian index
      const int gi = dom[k] == kNone ? -1 : (int)(dom[k] - (uint32_t)v * (uint32_t)b.views.n_gauss);
      if (io.dominant) io.dominant[p] = gi;
      if (gi >= 0 && dobs[k] > 0.f && b.nu_sum) {
        const float e = dobs[k] - ddom[k];
        unsafeAtomicAdd(b.nu_sum + gi, wdom[k] * e * e);
        atomicAdd(b.nu_count + gi, 1u);
      }
    }
  }
}

// Back-to-front over each pixel's blended run.  With the normalised "behind"
// sums Bx = sum_{k>j} w_k x_k / T_{j+1}, dL/dalpha_j = T_j sum_x g_x (x_j - Bx),
// and Bx <- alpha_j x_j + (1 - alpha_j) Bx moves the sums one Gaussian forward;
// T_j = T_{j+1} / (1 - alpha_j) recovers the transmittance from the final one.
// A lane first sums its pixels' contributions to a Gaussian, then the wave
// reduces all of the Gaussian's gradient terms together (wave_sum_many) and
// issues one atomic instruction.  kParams adds the
// opacity and colour gradients (mapping); kTrack takes the upstream
// gradients from the tracking forward (colour and depth only).
template <int kPPL, bool kParams, bool kTrack>
__global__ __launch_bounds__(kTilePixels / kPPL) void raster_backward_kernel(RasterBufs b) {
  constexpr int L = kTilePixels / kPPL;
  __shared__ float4 sA[kBatch];
  __shared__ float4 sB[kBatch];
  __shared__ float4 sC[kBatch];
  __shared__ uint32_t sM[kBatch];
  __shared__ uint32_t s_max;
  const int gtile = blockIdx.x;
  const int v = view_of_tile(b.views, gtile);
  const ViewIO io = b.views.io[v];
  const ViewInfo cam = io.info;
  const float2 org = tile_origin(cam, gtile);
  const int64_t hw = (int64_t)cam.width * cam.height;
  const uint2 range = b.ranges[gtile];
  const int lane = threadIdx.x & 63;

  float fx[kPPL], fy[kPPL], T[kPPL], gc0[kPPL], gc1[kPPL], gc2[kPPL], gd[kPPL], go[kPPL], gm[kPPL], gu[kPPL],
      dobs[kPPL];
  float Bc0[kPPL], Bc1[kPPL], Bc2[kPPL], Bd[kPPL], Bo[kPPL], Bu[kPPL];
  int walked[kPPL], med[kPPL];
  uint32_t lane_max = 0;
#pragma unroll
  for (int k = 0; k < kPPL; ++k) {
    const PixelCoord pc = pixel_of(cam, gtile, k * L + threadIdx.x);
    const int64_t pix = (int64_t)pc.py * cam.width + pc.px;
    fx[k] = (float)(pc.px - pc.ox);
    fy[k] = (float)(pc.py - pc.oy);
    T[k] = 1.f;
    walked[k] = 0;
    med[k] = -1;
    gc0[k] = gc1[k] = gc2[k] = gd[k] = go[k] = gm[k] = gu[k] = dobs[k] = 0.f;
    Bc0[k] = Bc1[k] = Bc2[k] = Bd[k] = Bo[k] = Bu[k] = 0.f;
    if (pc.inside) {
      const uint4 ps = b.pixel_state[cam.pixel_base + pix];
      T[k] = __uint_as_float(ps.x);
      walked[k] = (int)ps.y;
      med[k] = (int)ps.z;
      if (kTrack) {
        const float4 g4 = b.pixel_grad[cam.pixel_base + pix];
        gc0[k] = g4.x;
        gc1[k] = g4.y;
        gc2[k] = g4.z;
        gd[k] = g4.w;
      } else {
        if (io.g_color) {
          gc0[k] = io.g_color[pix];
          gc1[k] = io.g_color[hw + pix];
          gc2[k] = io.g_color[2 * hw + pix];
        }
        if (io.g_depth) gd[k] = io.g_depth[pix];
        if (io.g_opacity) go[k] = io.g_opacity[pix];
        if (io.g_median) gm[k] = io.g_median[pix];
        if (io.g_uncertainty) gu[k] = io.g_uncertainty[pix];
        if (io.depth_obs) dobs[k] = io.depth_obs[pix];
      }
      lane_max = max(lane_max, (uint32_t)walked[k]);
    }
  }
  if (threadIdx.x == 0) s_max = 0u;
  __syncthreads();
  if (lane_max) atomicMax(&s_max, lane_max);
  __syncthreads();
  const int nmax = (int)s_max;

  for (int end = nmax; end > 0; end -= kBatch) {
    const int start = max(0, end - kBatch);
    const int n = end - start;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += L) {
      const uint32_t m = b.vals[range.x + start + i];
      sM[i] = m;
      stage_record(b.rec + (int64_t)kRecF4 * m, org.x, org.y, sA[i], sB[i], sC[i]);
    }
    __syncthreads();
    for (int j = n - 1; j >= 0; --j) {
      const int pos = start + j;
      const float4 A = sA[j];
      const float4 B = sB[j];
      float u1 = 0.f, u2 = 0.f, sxx = 0.f, sxy = 0.f, syy = 0.f, gop = 0.f, gdd = 0.f;
      float gr = 0.f, gg = 0.f, gbl = 0.f;
      bool any = false;
      const float4 Cc = sC[j];
      // Straight-line, predicated per lane: a lane that did not blend this
      // record (past its last blended one, or alpha below 1/255) takes
      // alpha = 0, which leaves T and the behind sums exactly unchanged and
      // adds exact zeros to every gradient term.
#pragma unroll
      for (int k = 0; k < kPPL; ++k) {
        float dx, dy, tq;
        const float e = pair_exponent(A, B, fx[k], fy[k], dx, dy, tq);
        const bool hit = pos < walked[k] && e >= B.w;
        any = any || hit;
        const float g = __builtin_amdgcn_exp2f(e);
        const float raw = B.y * g;
        const float alpha = hit ? fminf(kAlphaMax, raw) : 0.f;
        const float oma = 1.f - alpha;
        const float Tj = T[k] * __builtin_amdgcn_rcpf(oma);
        const float wgt = alpha * Tj;
        float dsum = gc0[k] * (Cc.x - Bc0[k]) + gc1[k] * (Cc.y - Bc1[k]) + gc2[k] * (Cc.z - Bc2[k]) +
                     gd[k] * (B.z - Bd[k]);
        Bc0[k] = __builtin_fmaf(alpha, Cc.x, oma * Bc0[k]);
        Bc1[k] = __builtin_fmaf(alpha, Cc.y, oma * Bc1[k]);
        Bc2[k] = __builtin_fmaf(alpha, Cc.z, oma * Bc2[k]);
        Bd[k] = __builtin_fmaf(alpha, B.z, oma * Bd[k]);
        float dz = 0.f;
        if (!kTrack) {
          dz = B.z - dobs[k];
          const float u = dz * dz;
          dsum += go[k] * (1.f - Bo[k]) + gu[k] * (u - Bu[k]);
          Bo[k] = __builtin_fmaf(alpha, 1.f, oma * Bo[k]);
          Bu[k] = __builtin_fmaf(alpha, u, oma * Bu[k]);
        }
        const float dalpha = Tj * dsum;
        T[k] = Tj;
        const bool live = hit && !(raw > kAlphaMax);   // a capped alpha has no gradient
        const float dpower = live ? dalpha * raw : 0.f;   // alpha = opacity * exp(power)
        // power = -(a dx^2 + 2 b dx dy + c dy^2) / 2 = ln2 (qa t^2 + qc dy^2)
        // with t = dx + k dy, so d power/d mu = 2 ln2 (qa t, qa k t + qc dy)
        // and d power/d(a, b, c) = -(dx^2 / 2, dx dy, dy^2 / 2).  The factors
        // that belong to the record (qa, k, qc, the constants) are applied
        // once after the wave reduction; lanes only accumulate
        // u1 = sum dpower t, u2 = sum dpower dy and the second moments.
        const float pdx = dpower * dx, pdy = dpower * dy;
        u1 = __builtin_fmaf(dpower, tq, u1);
        u2 += pdy;
        sxx = __builtin_fmaf(pdx, dx, sxx);
        sxy = __builtin_fmaf(pdx, dy, sxy);
        syy = __builtin_fmaf(pdy, dy, syy);
        gdd += wgt * gd[k];
        if (!kTrack) gdd += 2.f * wgt * dz * gu[k] + ((hit && pos == med[k]) ? gm[k] : 0.f);
        if (kParams) {
          gop += live ? dalpha * g : 0.f;
          gr += wgt * gc0[k];
          gg += wgt * gc1[k];
          gbl += wgt * gc2[k];
        }
      }
      if (__ballot(any)) {
        const uint32_t m = sM[j];
        float* dst = b.rec_grad + (int64_t)kGradStride * m;
        // values 0-4 (u1, u2, sxx, sxy, syy) become the gradients of mu x,
        // mu y and the conic (a, b, c); the rest pass through.
        auto finish = [&](int idx, float t) {
          const float U1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, t), 0));
          const float c2 = 2.f * kLn2;
          float out = t;
          out = idx == 0 ? c2 * A.z * t : out;
          out = idx == 1 ? c2 * __builtin_fmaf(A.z * A.w, U1, B.x * t) : out;
          out = (idx == 2 || idx == 4) ? -0.5f * t : out;
          out = idx == 3 ? -t : out;
          return out;
        };
        if (kParams) {
          // slots 0-9: mu x, mu y, conic a, b, c, opacity, depth, colour
          const float vals[10] = {u1, u2, sxx, sxy, syy, gop, gdd, gr, gg, gbl};
          const float t = wave_sum_many<16>(vals);
          const int idx = reduced_value_index<16>(lane);
          const float out = finish(idx, t);
          if ((lane & 3) == 0 && idx < 10) unsafeAtomicAdd(dst + idx, out);
        } else {
          const float vals[6] = {u1, u2, sxx, sxy, syy, gdd};
          const float t = wave_sum_many<8>(vals);
          const int idx = reduced_value_index<8>(lane);
          const float out = finish(idx, t);
          if ((lane & 7) == 0 && idx < 6) unsafeAtomicAdd(dst + (idx == 5 ? 6 : idx), out);
        }
      }
    }
  }
}

template <int kPPL>
void launch_fwd(const RasterBufs& b, bool track, hipStream_t s) {
  const dim3 grid(b.total_tiles), block(kTilePixels / kPPL);
  if (track) hipLaunchKernelGGL((raster_forward_kernel<kPPL, true, false>), grid, block, 0, s, b);
  else if (b.nu) hipLaunchKernelGGL((raster_forward_kernel<kPPL, false, true>), grid, block, 0, s, b);
  else hipLaunchKernelGGL((raster_forward_kernel<kPPL, false, false>), grid, block, 0, s, b);
}

template <int kPPL>
void launch_bwd(const RasterBufs& b, bool params, bool track, hipStream_t s) {
  const dim3 grid(b.total_tiles), block(kTilePixels / kPPL);
  if (track) hipLaunchKernelGGL((raster_backward_kernel<kPPL, false, true>), grid, block, 0, s, b);
  else if (params) hipLaunchKernelGGL((raster_backward_kernel<kPPL, true, false>), grid, block, 0, s, b);
  else hipLaunchKernelGGL((raster_backward_kernel<kPPL, false, false>), grid, block, 0, s, b);
}

}  // namespace

void launch_raster_forward(const RasterBufs& b, bool track, int ppl, hipStream_t s) {
  if (b.total_tiles <= 0) return;
  if (ppl == 4) launch_fwd<4>(b, track, s);
  else if (ppl == 2) launch_fwd<2>(b, track, s);
  else launch_fwd<1>(b, track, s);
}

void launch_raster_backward(const RasterBufs& b, bool param_grads, bool track, int ppl, hipStream_t s) {
  if (b.total_tiles <= 0) return;
  if (ppl == 4) launch_bwd<4>(b, param_grads, track, s);
  else if (ppl == 2) launch_bwd<2>(b, param_grads, track, s);
  else launch_bwd<1>(b, param_grads, track, s);
}

}  // namespace cgsr
