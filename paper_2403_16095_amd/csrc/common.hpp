// Device-side definitions shared by the cgsr kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cgsr.h"

namespace cgsr {

// Readings of constants the paper leaves to the 3-D Gaussian splatting
// rasterizer it builds on (Sec. 3.1); the CPU oracle states the same values.
constexpr float kNearZ = 0.2f;              // cull at camera z <= this
constexpr float kTanClamp = 1.3f;           // J uses x/z clamped to 1.3 x half FOV
constexpr float kDilation = 0.3f;           // added to the 2-D covariance diagonal
constexpr float kAlphaMax = 0.99f;          // alpha cap
constexpr float kAlphaMin = 1.0f / 255.0f;  // alpha below this is skipped
constexpr float kTStop = 1.0e-4f;           // stop before T would fall below this
constexpr float kTMedian = 0.5f;            // Eq. 8
constexpr float kBinR2Rel = 1.0f + 1.0f / 128.0f;  // binning-rectangle margins
constexpr float kBinR2Abs = 1.0f / 256.0f;

constexpr int kTile = 16;                   // tile edge in pixels
constexpr int kTilePixels = kTile * kTile;  // one workgroup per tile, one pixel per lane
constexpr int kWave = 64;

// Per-view camera constants.
struct ViewInfo {
  int32_t width, height;
  float fx, fy, cx, cy;
  int32_t tiles_x, tiles_y;
  int32_t tile_base;   // first global tile index of this view
  int32_t pixel_base;  // first global pixel index of this view
};

// One entry of a per-view table in device memory: the camera plus the
// device pointers of that view's images (forward) or gradients (backward).
// Tables are uploaded only when their contents change, which keeps kernel
// arguments small and lets a steady loop be captured into a graph.
struct ViewIO {
  ViewInfo info;
  const float* depth_obs;   // [H][W] or null
  float* color;             // [3][H][W] or null
  float* depth;
  float* opacity;
  float* depth_median;
  float* uncertainty;
  const float* g_color;     // upstream gradients (backward)
  const float* g_depth;
  const float* g_opacity;
  const float* g_median;
  const float* g_uncertainty;
};

struct ViewTable {
  const ViewIO* io;   // [n] device
  int32_t n;          // views
  int32_t n_gauss;    // Gaussians per view (records are view-major)
};

// Projected record, 3 x float4 per (view, Gaussian):
//   a = (mu_x, mu_y, conic_a, conic_b)
//   b = (conic_c, opacity, depth, r)
//   c = (g, b, 0, 0)
constexpr int kRecF4 = 3;

// Per-record gradient accumulator with respect to the projected quantities:
//   0,1 mu   2,3,4 conic (a, b, c)   5 opacity   6 depth   7,8,9 colour
constexpr int kGradStride = 12;  // floats per record (48 B, 16-B aligned)

// alpha of a (Gaussian, pixel) pair, Eq. 5 with the 3DGS conventions.  Used by
// the forward and the backward pass with identical operation order, so both
// take the same skip, cap and stop decisions (the library is built without
// floating-point contraction; every fused multiply-add here is explicit).
struct PairAlpha {
  float dx, dy;   // mu - pixel
  float g;        // exp(power)
  float raw;      // opacity * g (before the cap)
};

__device__ __forceinline__ PairAlpha pair_alpha(float mux, float muy, float ca, float cb, float cc,
                                                float opac, float px, float py) {
  PairAlpha r;
  r.dx = mux - px;
  r.dy = muy - py;
  const float q = __builtin_fmaf(ca * r.dx, r.dx, __builtin_fmaf(cc * r.dy, r.dy, 2.0f * cb * r.dx * r.dy));
  r.g = __expf(-0.5f * q);
  r.raw = opac * r.g;
  return r;
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_move(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kCtrl, kRowMask, 0xF,
                                                               false));
}

// Sum over the 64 lanes of a wave with DPP row operations; every lane must be
// active.  Returns the total (wave-uniform).
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_move<0x140, 0xF>(v);  // row_mirror
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of a 64-bit wave mask below this lane.
__device__ __forceinline__ int mask_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ __forceinline__ uint32_t float_key(float z) { return __float_as_uint(z); }

__device__ __forceinline__ int view_of_tile(const ViewTable& vt, int gtile) {
  int v = 0;
  while (v + 1 < vt.n && gtile >= vt.io[v + 1].info.tile_base) ++v;
  return v;
}

}  // namespace cgsr
