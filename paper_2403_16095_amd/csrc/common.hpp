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
  int32_t* dominant;        // [H][W] Gaussian of largest weight (Eq. 13) or -1, or null
  const float* g_color;     // upstream gradients (backward)
  const float* g_depth;
  const float* g_opacity;
  const float* g_median;
  const float* g_uncertainty;
  const float* t_color;     // tracking targets: [3][H][W] colour and [H][W] depth
  const float* t_depth;
};

struct ViewTable {
  const ViewIO* io;   // [n] device, followed by one word: the hash of the uploaded table
  int32_t n;          // views
  int32_t n_gauss;    // Gaussians per view (records are view-major)
  uint32_t hash;      // the hash of the table this launch was set up with
};


// Projected record, 3 x float4 per (view, Gaussian):
//   a = (mu_x, mu_y, a, k)                  mu = float nearest the mean
//   b = (c', opacity, depth, r)
//   c = (g, b, mu_x lo, mu_y lo)             the mean is mu + lo
// The conic (a, b, c) enters as the completed square
//   a dx^2 + 2 b dx dy + c dy^2 = a (dx + k dy)^2 + c' dy^2,
//   k = b / a,  c' = c - b^2 / a = 1 / Sigma2d_yy,
// whose two terms are non-negative: the expanded form cancels for thin,
// tilted footprints (|2 b dx dy| ~ a dx^2 + c dy^2), and float rounding of its
// large terms then reached 1e-4 of the exponent.  Both k and c' come from the
// double-precision projection.
constexpr int kRecF4 = 3;

// Per-record gradient accumulator with respect to the projected quantities:
//   0,1 mu   2,3,4 conic (a, b, c)   5 opacity   6 depth   7,8,9 colour
constexpr int kGradStride = 12;  // floats per record (48 B, 16-B aligned)

// A record as the blend kernels stage it in LDS, once per (tile, record):
//   a = (mu_x, mu_y, qa, k)        mean relative to the tile origin (ox, oy),
//                                  qa = -a/2 log2(e)
//   b = (qc, opacity, depth, pos)  qc = -c'/2 log2(e); pos: the staging's
//   c = (r, g, b, id)              list position and record id (int bits)
// so that the exponent of Eq. 5 in base 2 is qa (dx + k dy)^2 + qc dy^2, and
// alpha = opacity 2^exponent (skipped below 1/255, capped at 0.99).  The
// forward and the backward stage and evaluate with these same functions (the
// library is built without floating-point contraction, every fused
// multiply-add is explicit), so they take identical skip, cap and stop
// decisions.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Pixel coordinates inside the blend kernels are relative to the tile origin
// too, so dx and dy carry no rounding from large absolute coordinates: the
// float part minus the origin is exact when the mean lies within a factor of
// two of the origin (and rounds by an ulp of the difference otherwise, where
// only wide Gaussians, with small conics, reach the tile); the low part adds
// the rest.
__device__ __forceinline__ void stage_record(const float4* __restrict__ rec, float ox, float oy, float4& A, float4& B,
                                             float4& C) {
  const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2];
  A = make_float4((r0.x - ox) + r2.z, (r0.y - oy) + r2.w, (-0.5f * kLog2e) * r0.z, r0.w);
  B = make_float4((-0.5f * kLog2e) * r1.x, r1.y, r1.z, 0.f);
  C = make_float4(r1.w, r2.x, r2.y, 0.f);
}

// Whether a staged record (A, B) can reach alpha >= 1/255 anywhere on the
// square of pixel centres [x0, x0 + span] x [y0, y0 + span], tile-relative.
// The base-2 exponent of Eq. 5 is a concave quadratic in the pixel position,
// so its maximum over the square (taken continuous, which bounds every
// pixel's) is 0 at the mean when the square holds it and otherwise lies on an
// edge, where it is a one-dimensional maximum clamped to the edge.  A record
// is kept unless it falls short by kCellMargin (base-2 units: alpha a factor
// 1.007 below the threshold), far more than the rounding of the per-pixel
// evaluation, so a dropped record is one every pixel of the square would skip
// and the blends give the same results without it.
constexpr float kCellMargin = 0.01f;
__device__ __forceinline__ bool box_reached(const float4& A, const float4& B, float x0, float y0, float span) {
  const float dx0 = A.x - (x0 + span), dx1 = A.x - x0, dy0 = A.y - (y0 + span), dy1 = A.y - y0;
  if (dx0 <= 0.f && dx1 >= 0.f && dy0 <= 0.f && dy1 >= 0.f) return true;
  const float qa = A.z, k = A.w, qc = B.x;   // exponent qa t^2 + qc dy^2, t = dx + k dy
  auto expo = [&](float dx, float dy) {
    const float t = __builtin_fmaf(k, dy, dx);
    return __builtin_fmaf(qa, t * t, qc * (dy * dy));
  };
  // edges dy = dy0, dy1: t = 0 at dx = -k dy
  float best = fmaxf(expo(fminf(fmaxf(-k * dy0, dx0), dx1), dy0), expo(fminf(fmaxf(-k * dy1, dx0), dx1), dy1));
  // edges dx = dx0, dx1: the exponent is largest at dy = sl dx
  const float sl = -(qa * k) / __builtin_fmaf(qa * k, k, qc);
  best = fmaxf(best, expo(dx0, fminf(fmaxf(sl * dx0, dy0), dy1)));
  best = fmaxf(best, expo(dx1, fminf(fmaxf(sl * dx1, dy0), dy1)));
  return B.y * __builtin_amdgcn_exp2f(best + kCellMargin) >= kAlphaMin;
}

// Base-2 exponent of a staged record at pixel centre (px, py); dx, dy = mu - p
// and t = dx + k dy.
__device__ __forceinline__ float pair_exponent(const float4& A, const float4& B, float px, float py, float& dx,
                                               float& dy, float& t) {
  dx = A.x - px;
  dy = A.y - py;
  t = __builtin_fmaf(A.w, dy, dx);
  return __builtin_fmaf(A.z, t * t, B.x * (dy * dy));
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

// Sums K per-lane values (K <= NV, NV = 8 or 16) over the 64 lanes of a wave
// at once, by halving the lanes per value while doubling the values per
// register: a gfx950 permlane32 swap pairs the two wave halves, a permlane16
// swap pairs rows, row_ror:8 pairs the halves of each row (and, for NV = 16,
// row_half_mirror pairs the quarters), and the remaining DPP butterflies
// finish each value inside a group of 64 / NV lanes.  About NV + 2 log2(64 /
// NV) adds and swaps instead of K full six-step reductions.  Every lane must be
// active.  Returns, in each lane, the total of value reduced_value_index<NV>
// (lane), which is the same for the 64 / NV lanes of a group.
template <int NV>
__device__ __forceinline__ constexpr int reduced_value_index(int lane) {
  const int r = lane >> 4;
  const int qb = NV == 16 ? 2 * ((lane >> 2) & 1) + ((lane >> 3) & 1) : ((lane >> 3) & 1);
  return 2 * (2 * qb + (r & 1)) + (r >> 1);
}

// The swaps are written as inline assembly: this compiler's optimiser folds
// the two results of its permlane-swap builtins into one (the IR adds the
// first result to itself), which would silently drop half of every sum.  The
// s_nop pairs give the wait states a VALU write needs before a permlane reads
// the register, and a permlane write before the next VALU reads it.  The
// swaps of one reduction level touch different registers, so they share one
// block and one pair of s_nop (up to four swaps a block).
#define CGSR_PERMLANE_SWAPS(op, n)                                                                     \
  if constexpr (n == 1) {                                                                              \
    asm volatile("s_nop 1\n\t" op " %0, %1\n\ts_nop 1" : "+v"(x[0]), "+v"(y[0]));                      \
  } else if constexpr (n == 2) {                                                                       \
    asm volatile("s_nop 1\n\t" op " %0, %1\n\t" op " %2, %3\n\ts_nop 1"                                \
                 : "+v"(x[0]), "+v"(y[0]), "+v"(x[1]), "+v"(y[1]));                                    \
  } else if constexpr (n == 3) {                                                                       \
    asm volatile("s_nop 1\n\t" op " %0, %1\n\t" op " %2, %3\n\t" op " %4, %5\n\ts_nop 1"              \
                 : "+v"(x[0]), "+v"(y[0]), "+v"(x[1]), "+v"(y[1]), "+v"(x[2]), "+v"(y[2]));            \
  } else {                                                                                             \
    asm volatile("s_nop 1\n\t" op " %0, %1\n\t" op " %2, %3\n\t" op " %4, %5\n\t" op " %6, %7\n\ts_nop 1" \
                 : "+v"(x[0]), "+v"(y[0]), "+v"(x[1]), "+v"(y[1]), "+v"(x[2]), "+v"(y[2]), "+v"(x[3]),  \
                   "+v"(y[3]));                                                                        \
  }

// x[i] <-> y[i] across the wave halves (lanes 32-63 of x with 0-31 of y).
template <int N>
__device__ __forceinline__ void swap_halves32(float* x, float* y) {
  static_assert(N >= 1, "at least one pair");
  CGSR_PERMLANE_SWAPS("v_permlane32_swap_b32", (N < 4 ? N : 4))
  if constexpr (N > 4) swap_halves32<N - 4>(x + 4, y + 4);
}

// The same across the 16-lane rows (rows 1 and 3 of x with rows 0 and 2 of y).
template <int N>
__device__ __forceinline__ void swap_halves16(float* x, float* y) {
  static_assert(N >= 1, "at least one pair");
  CGSR_PERMLANE_SWAPS("v_permlane16_swap_b32", (N < 4 ? N : 4))
  if constexpr (N > 4) swap_halves16<N - 4>(x + 4, y + 4);
}
#undef CGSR_PERMLANE_SWAPS

template <int NV, int K>
__device__ __forceinline__ float wave_sum_many(const float (&v)[K]) {
  static_assert((NV == 8 || NV == 16) && K <= NV, "8 or 16 slots");
  const int lane = __lane_id();
  // first level: value pairs (2p, 2p + 1) that hold a value, swapped and added
  constexpr int P32 = (K + 1) / 2;
  float x[P32], y[P32];
#pragma unroll
  for (int p = 0; p < P32; ++p) {
    x[p] = v[2 * p];
    y[p] = 2 * p + 1 < K ? v[2 * p + 1] : 0.f;
  }
  swap_halves32<P32>(x, y);
  float a[NV / 2];
#pragma unroll
  for (int p = 0; p < NV / 2; ++p) a[p] = p < P32 ? x[p] + y[p] : 0.f;   // both slots empty beyond
  // second level: pairs (a[2q], a[2q + 1]) that hold a value
  constexpr int P16 = (K + 3) / 4;
  float x2[P16], y2[P16];
#pragma unroll
  for (int q = 0; q < P16; ++q) {
    x2[q] = a[2 * q];
    y2[q] = a[2 * q + 1];
  }
  swap_halves16<P16>(x2, y2);
  float b[NV / 4];
#pragma unroll
  for (int q = 0; q < NV / 4; ++q) b[q] = q < P16 ? x2[q] + y2[q] : 0.f;
  float c[NV / 8];
  const bool hi8 = lane & 8;
#pragma unroll
  for (int t = 0; t < NV / 8; ++t) {
    const float send = hi8 ? b[2 * t] : b[2 * t + 1];
    const float keep = hi8 ? b[2 * t + 1] : b[2 * t];
    c[t] = keep + dpp_move<0x128, 0xF>(send);                     // row_ror:8
  }
  float d;
  if constexpr (NV == 16) {
    const bool hi4 = lane & 4;
    const float send = hi4 ? c[0] : c[1];
    const float keep = hi4 ? c[1] : c[0];
    d = keep + dpp_move<0x141, 0xF>(send);                        // row_half_mirror
  } else {
    d = c[0];
    d += dpp_move<0x141, 0xF>(d);
  }
  d += dpp_move<0x4E, 0xF>(d);                                    // quad_perm [2,3,0,1]
  d += dpp_move<0xB1, 0xF>(d);                                    // quad_perm [1,0,3,2]
  return d;
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

struct AdamParams {
  float lr_rho, lr_phi, beta1, beta2, eps;
};

// One Adam step (bias-corrected) on a pose's tangent vector xi = (rho, phi),
// whose value is zero at the current pose, so the step is
// delta = -lr m_hat / (sqrt(v_hat) + eps); then the left retraction
// T <- exp(delta^) T with the closed-form SE(3) exponential.  One wave per
// pose: lane k < 6 holds gradient component g and updates its own moments;
// lane 0 writes the pose.  P: pose[12] (row-major R, t); st: m[6], v[6], step
// count, 1 - beta1^step, 1 - beta2^step (all zero before the first step: the
// bias corrections are kept as running values, c <- beta c + 1 - beta).
__device__ inline void adam_retract_wave(float* P, float* st, float g, const AdamParams& ap) {
  const int k = __lane_id();
  const float step = st[12] + 1.f;
  const float c1 = __builtin_fmaf(ap.beta1, st[13], 1.f - ap.beta1);
  const float c2 = __builtin_fmaf(ap.beta2, st[14], 1.f - ap.beta2);
  float d = 0.f;
  if (k < 6) {
    const float m = ap.beta1 * st[k] + (1.f - ap.beta1) * g;
    const float s = ap.beta2 * st[6 + k] + (1.f - ap.beta2) * g * g;
    st[k] = m;
    st[6 + k] = s;
    const float lr = k < 3 ? ap.lr_rho : ap.lr_phi;
    d = -lr * (m / c1) / (sqrtf(s / c2) + ap.eps);
  }
  float dl[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) dl[j] = __shfl(d, j);
  if (k != 0) return;
  st[12] = step;
  st[13] = c1;
  st[14] = c2;
  // exp of (rho, phi): R = I + A K + B K^2, V = I + B K + C K^2, K = [phi]x.
  const float p0 = dl[3], p1 = dl[4], p2 = dl[5];
  const float th2 = p0 * p0 + p1 * p1 + p2 * p2;
  // Below 0.1 rad (every step of a converging solve) the series, whose next
  // terms are under 1e-9; the closed forms there lose digits to cancellation.
  float A, Bc, Cc;
  if (th2 < 1e-2f) {
    A = 1.f - th2 / 6.f * (1.f - th2 / 20.f);
    Bc = 0.5f - th2 / 24.f * (1.f - th2 / 30.f);
    Cc = 1.f / 6.f - th2 / 120.f * (1.f - th2 / 42.f);
  } else {
    const float th = sqrtf(th2);
    float sn, cs;
    sincosf(th, &sn, &cs);
    A = sn / th;
    Bc = (1.f - cs) / th2;
    Cc = (th - sn) / (th2 * th);
  }
  const float K[9] = {0.f, -p2, p1, p2, 0.f, -p0, -p1, p0, 0.f};
  float K2[9], R[9], V[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) K2[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
  for (int q = 0; q < 9; ++q) {
    const float I = (q % 4 == 0) ? 1.f : 0.f;
    R[q] = I + A * K[q] + Bc * K2[q];
    V[q] = I + Bc * K[q] + Cc * K2[q];
  }
  float Rn[9], tn[3];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) Rn[3 * r + c] = R[3 * r] * P[c] + R[3 * r + 1] * P[3 + c] + R[3 * r + 2] * P[6 + c];
    tn[r] = R[3 * r] * P[9] + R[3 * r + 1] * P[10] + R[3 * r + 2] * P[11] + V[3 * r] * dl[0] + V[3 * r + 1] * dl[1] +
            V[3 * r + 2] * dl[2];
  }
  for (int q = 0; q < 9; ++q) P[q] = Rn[q];
  for (int q = 0; q < 3; ++q) P[9 + q] = tn[q];
}

}  // namespace cgsr
