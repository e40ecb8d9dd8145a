// Per-(view, Gaussian) projection (Sec. 3.1, Eq. 1-2), pair emission into
// fixed-size per-tile buckets for the tile sort (no global scan: a returning
// atomic on the tile's count is the pair's slot; pairs whose Gaussian reaches
// alpha >= 1/255 on no pixel of the tile are not emitted), and the chain rule back from
// the projected quantities to the Gaussian parameters and the camera pose.
//
// Grid layout: blockIdx.y = view, blockIdx.x covers the Gaussians, so every
// workgroup sees one view and reads its camera from the view table with
// uniform (scalar) loads.  Records are view-major: m = view * n + i.
#include <algorithm>

#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kThreads = 256;

// Rotation matrix (row-major) of the unit quaternion (w, x, y, z).
__device__ __forceinline__ void quat_rot(double w, double x, double y, double z, double R[9]) {
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Everything the forward and backward projection share.  The projection's
// linear algebra is evaluated in double precision: it costs a few hundred
// operations per Gaussian, and single precision would leave pixel-space means
// near x = 1000 with ~1e-4 px of rounding, which the exponent of Eq. 5
// amplifies by the conic times the offset from the mean, and conics of thin
// footprints with the cancellation of their 2x2 determinant (which also
// amplifies any rounding of the scales, so exp of the log-scales is double
// too).  The opacity sigmoid and the rectangle's log are single precision:
// they enter linearly or against a relative margin.
struct Proj {
  double qn[4], qinv;    // unit quaternion and 1/|q|
  double R[9];           // rotation of the ellipsoid
  double s[3];           // scales
  double p[3];           // camera-space mean
  double Sc[6];          // camera covariance W Sigma W^T: 00 01 02 11 12 22
  double J00, J02, J11, J12;
  int clampx, clampy;
  double tx, ty;         // (possibly clamped) tangents used in J
  double cov[3];         // Sigma2d xx, xy, yy (dilated)
  double conic[3];
  double opacity;
};

// The parameters of Eq. 1-2 of one Gaussian, read together: the culling
// tests of project_core then wait for one memory round trip, not one per
// parameter (the compiler keeps loads behind the branches they follow).
struct GaussianIn {
  float4 q;
  float ls[3], X[3];
  float opacity_logit;
};

__device__ __forceinline__ GaussianIn load_gaussian(const GaussianPtrs& g, int64_t i) {
  GaussianIn in;
  in.q = reinterpret_cast<const float4*>(g.quats)[i];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    in.ls[k] = g.log_scales[3 * i + k];
    in.X[k] = g.means[3 * i + k];
  }
  in.opacity_logit = g.opacity_logits[i];
  return in;
}

// Eq. 1-2 for a Gaussian (parameters in) under pose P.  Returns false if the
// Gaussian is culled (non-finite or zero quaternion, behind the near plane,
// opacity under 1/255, singular 2-D covariance).
__device__ bool project_core(const GaussianIn& in, const float* P, const ViewInfo& cam, Proj& o) {
  double W[9], t[3];   // the pose, read before the first test as well
#pragma unroll
  for (int k = 0; k < 9; ++k) W[k] = P[k];
#pragma unroll
  for (int r = 0; r < 3; ++r) t[r] = P[9 + r];
  const double q0 = in.q.x, q1 = in.q.y, q2 = in.q.z, q3 = in.q.w;
  const double qn2 = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
  if (!(qn2 > 0.0) || !(qn2 < 1.0e300)) return false;
  o.qinv = 1.0 / sqrt(qn2);
  o.qn[0] = q0 * o.qinv; o.qn[1] = q1 * o.qinv; o.qn[2] = q2 * o.qinv; o.qn[3] = q3 * o.qinv;
  quat_rot(o.qn[0], o.qn[1], o.qn[2], o.qn[3], o.R);
  o.s[0] = exp((double)in.ls[0]); o.s[1] = exp((double)in.ls[1]); o.s[2] = exp((double)in.ls[2]);
  const double X0 = in.X[0], X1 = in.X[1], X2 = in.X[2];
#pragma unroll
  for (int r = 0; r < 3; ++r) o.p[r] = W[3 * r] * X0 + W[3 * r + 1] * X1 + W[3 * r + 2] * X2 + t[r];
  const double z = o.p[2];
  if (!(z > (double)kNearZ)) return false;
  o.opacity = 1.0f / (1.0f + expf(-in.opacity_logit));
  if (!(o.opacity >= (double)kAlphaMin)) return false;
  // Sigma = (R S)(R S)^T, then Sc = W Sigma W^T with W the camera rotation.
  double M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[3 * r + k] = o.R[3 * r + k] * o.s[k];
  double WM[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) WM[3 * r + k] = W[3 * r] * M[k] + W[3 * r + 1] * M[3 + k] + W[3 * r + 2] * M[6 + k];
  auto dot3 = [&](int r, int c) {
    return WM[3 * r] * WM[3 * c] + WM[3 * r + 1] * WM[3 * c + 1] + WM[3 * r + 2] * WM[3 * c + 2];
  };
  o.Sc[0] = dot3(0, 0); o.Sc[1] = dot3(0, 1); o.Sc[2] = dot3(0, 2);
  o.Sc[3] = dot3(1, 1); o.Sc[4] = dot3(1, 2); o.Sc[5] = dot3(2, 2);
  // Affine projection Jacobian at p with the tangent clamp.
  const double fx = cam.fx, fy = cam.fy;
  const double limx = (double)kTanClamp * 0.5 * (double)cam.width / fx;
  const double limy = (double)kTanClamp * 0.5 * (double)cam.height / fy;
  const double zinv = 1.0 / z;
  double tx = o.p[0] * zinv, ty = o.p[1] * zinv;
  o.clampx = tx > limx ? 1 : (tx < -limx ? -1 : 0);
  o.clampy = ty > limy ? 1 : (ty < -limy ? -1 : 0);
  if (o.clampx) tx = o.clampx * limx;
  if (o.clampy) ty = o.clampy * limy;
  o.tx = tx; o.ty = ty;
  o.J00 = fx * zinv;
  o.J02 = -fx * tx * zinv;
  o.J11 = fy * zinv;
  o.J12 = -fy * ty * zinv;
  const double* S = o.Sc;
  o.cov[0] = o.J00 * o.J00 * S[0] + 2.0 * o.J00 * o.J02 * S[2] + o.J02 * o.J02 * S[5] + (double)kDilation;
  o.cov[1] = o.J00 * o.J11 * S[1] + o.J00 * o.J12 * S[2] + o.J02 * o.J11 * S[4] + o.J02 * o.J12 * S[5];
  o.cov[2] = o.J11 * o.J11 * S[3] + 2.0 * o.J11 * o.J12 * S[4] + o.J12 * o.J12 * S[5] + (double)kDilation;
  const double det = o.cov[0] * o.cov[2] - o.cov[1] * o.cov[1];
  if (!(det > 0.0)) return false;
  const double dinv = 1.0 / det;
  o.conic[0] = o.cov[2] * dinv;
  o.conic[1] = -o.cov[1] * dinv;
  o.conic[2] = o.cov[0] * dinv;
  return true;
}

// A wave's (Gaussian, tile) pairs, spread evenly over its 64 lanes.  Each
// lane owns ntiles tiles of its Gaussian's rectangle (tx0, ty0, width w); a
// single large Gaussian would otherwise keep one lane busy for hundreds of
// tiles while the rest of the chip waits for that wave.  The lanes' exclusive
// prefix offsets go to LDS; pair k of the wave belongs to the last lane whose
// offset is <= k (lanes without tiles share the next lane's offset, so they
// are never chosen).  Every lane of the wave must call this.
struct WavePairs {
  uint32_t* off;    // [64] exclusive prefix of ntiles
  uint32_t* org;    // [64] tx0 | ty0 << 16
  uint32_t* wid;    // [64] rectangle width in tiles
  uint32_t total;
};

__device__ __forceinline__ WavePairs wave_pairs(uint32_t ntiles, uint32_t tx0, uint32_t ty0, uint32_t w,
                                                uint32_t* lds_off, uint32_t* lds_org, uint32_t* lds_wid) {
  const int lane = threadIdx.x & 63;
  uint32_t incl = ntiles;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d);
    if (lane >= d) incl += y;
  }
  lds_off[lane] = incl - ntiles;
  lds_org[lane] = tx0 | (ty0 << 16);
  lds_wid[lane] = w;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the LDS writes have landed
  return WavePairs{lds_off, lds_org, lds_wid, (uint32_t)__shfl(incl, 63)};
}

// Owner lane and tile (within the view, row-major) of pair k of the wave.
__device__ __forceinline__ uint32_t pair_tile(const WavePairs& wp, uint32_t k, int tiles_x, int* owner) {
  int j = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1)
    if (wp.off[j + step] <= k) j += step;
  const uint32_t local = k - wp.off[j], w = wp.wid[j], org = wp.org[j];
  *owner = j;
  return ((org >> 16) + local / w) * (uint32_t)tiles_x + (org & 0xFFFF) + local % w;
}

// View-dependent colour (Sec. 3.1): real spherical harmonics with the
// Condon-Shortley phase, k = l^2 + l + m, at the unit direction (x, y, z).
// Each constant is the normalisation sqrt((2l + 1) / (4 pi) (l - |m|)! /
// (l + |m|)!) (times sqrt 2 for m != 0) times the leading coefficient of the
// harmonic's polynomial.
constexpr float kSh00 = 0.28209479177387814f;   // sqrt(1 / (4 pi))
constexpr float kSh1 = 0.4886025119029199f;     // sqrt(3 / (4 pi))
constexpr float kSh2a = 1.0925484305920792f;    // sqrt(15 / (4 pi))
constexpr float kSh20 = 0.31539156525252005f;   // sqrt(5 / (16 pi))
constexpr float kSh22 = 0.5462742152960396f;    // sqrt(15 / (16 pi))
constexpr float kSh33 = 0.5900435899266435f;    // sqrt(35 / (32 pi))
constexpr float kSh32 = 2.890611442640554f;     // sqrt(105 / (4 pi))
constexpr float kSh31 = 0.4570457994644658f;    // sqrt(21 / (32 pi))
constexpr float kSh30 = 0.3731763325901154f;    // sqrt(7 / (16 pi))
constexpr float kSh32b = 1.445305721320277f;    // sqrt(105 / (16 pi))

__device__ __forceinline__ void sh_basis(int degree, float x, float y, float z, float (&Y)[16]) {
  Y[0] = kSh00;
  if (degree < 1) return;
  Y[1] = -kSh1 * y;
  Y[2] = kSh1 * z;
  Y[3] = -kSh1 * x;
  if (degree < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kSh2a * x * y;
  Y[5] = -kSh2a * y * z;
  Y[6] = kSh20 * (3.f * zz - 1.f);
  Y[7] = -kSh2a * x * z;
  Y[8] = kSh22 * (xx - yy);
  if (degree < 3) return;
  Y[9] = -kSh33 * y * (3.f * xx - yy);
  Y[10] = kSh32 * x * y * z;
  Y[11] = -kSh31 * y * (5.f * zz - 1.f);
  Y[12] = kSh30 * z * (5.f * zz - 3.f);
  Y[13] = -kSh31 * x * (5.f * zz - 1.f);
  Y[14] = kSh32b * z * (xx - yy);
  Y[15] = -kSh33 * x * (xx - 3.f * yy);
}

// sum_k w_k grad Y_k at (x, y, z), k < (degree + 1)^2.
__device__ __forceinline__ float3 sh_grad(int degree, float x, float y, float z, const float (&w)[16]) {
  float gx = 0.f, gy = 0.f, gz = 0.f;
  if (degree >= 1) {
    gy -= kSh1 * w[1];
    gz += kSh1 * w[2];
    gx -= kSh1 * w[3];
  }
  if (degree >= 2) {
    gx += kSh2a * y * w[4];
    gy += kSh2a * x * w[4];
    gy -= kSh2a * z * w[5];
    gz -= kSh2a * y * w[5];
    gz += 6.f * kSh20 * z * w[6];
    gx -= kSh2a * z * w[7];
    gz -= kSh2a * x * w[7];
    gx += 2.f * kSh22 * x * w[8];
    gy -= 2.f * kSh22 * y * w[8];
  }
  if (degree >= 3) {
    const float xx = x * x, yy = y * y, zz = z * z;
    gx -= kSh33 * 6.f * x * y * w[9];
    gy -= kSh33 * 3.f * (xx - yy) * w[9];
    gx += kSh32 * y * z * w[10];
    gy += kSh32 * x * z * w[10];
    gz += kSh32 * x * y * w[10];
    gy -= kSh31 * (5.f * zz - 1.f) * w[11];
    gz -= kSh31 * 10.f * y * z * w[11];
    gz += kSh30 * (15.f * zz - 3.f) * w[12];
    gx -= kSh31 * (5.f * zz - 1.f) * w[13];
    gz -= kSh31 * 10.f * x * z * w[13];
    gx += kSh32b * 2.f * x * z * w[14];
    gy -= kSh32b * 2.f * y * z * w[14];
    gz += kSh32b * (xx - yy) * w[14];
    gx -= kSh33 * 3.f * (xx - yy) * w[15];
    gy += kSh33 * 6.f * x * y * w[15];
  }
  return make_float3(gx, gy, gz);
}

// Viewing direction of Gaussian i from the camera centre C = -R^T t of pose
// P, its inverse distance, the harmonics there and the colour
// max(0, sum_k sh_k Y_k + 1/2) per channel (clamped[c]: below zero).
struct ShColour {
  float d[3], inv_len;
  float Y[16];
  float c[48];   // the Gaussian's coefficients, [k][channel], k < (degree + 1)^2
  float col[3];
  bool clamped[3];
};

// Whether a Gaussian's 3 K coefficients can move as 16-byte words: a whole
// number of them and a 16-byte aligned array (then every Gaussian's block is).
__device__ __forceinline__ bool sh_vector(const float* base, int K) {
  return (3 * K) % 4 == 0 && (reinterpret_cast<uintptr_t>(base) & 15u) == 0;
}

// Loads the 3 K coefficients at c into cf (the rest zero): 16-byte loads
// where sh_vector allows, one lane reading its Gaussian's contiguous block.
__device__ __forceinline__ void load_sh(const float* base, int64_t i, int K, float (&cf)[48]) {
  const float* c = base + (int64_t)3 * K * i;
  if (sh_vector(base, K)) {
    const float4* c4 = reinterpret_cast<const float4*>(c);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const float4 v = 4 * q < 3 * K ? c4[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      cf[4 * q] = v.x;
      cf[4 * q + 1] = v.y;
      cf[4 * q + 2] = v.z;
      cf[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 48; ++e) cf[e] = e < 3 * K ? c[e] : 0.f;
  }
}

__device__ __forceinline__ void sh_colour(const GaussianPtrs& g, int64_t i, const float* P, ShColour& o) {
  const float* X = g.means + 3 * i;
  float v[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = X[k] + (P[k] * P[9] + P[3 + k] * P[10] + P[6 + k] * P[11]);
  const float len2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  o.inv_len = len2 > 0.f ? 1.0f / sqrtf(len2) : 0.f;
  o.d[0] = v[0] * o.inv_len;
  o.d[1] = v[1] * o.inv_len;
  o.d[2] = len2 > 0.f ? v[2] * o.inv_len : 1.f;
  sh_basis(g.sh_degree, o.d[0], o.d[1], o.d[2], o.Y);
  const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
  load_sh(g.sh, i, K, o.c);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float sum = 0.5f;
    // a constant trip count keeps Y in registers (a bound of K would index
    // it at run time, which puts the array in scratch memory)
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < K) sum = __builtin_fmaf(o.c[3 * k + ch], o.Y[k], sum);
    o.clamped[ch] = sum < 0.f;
    o.col[ch] = o.clamped[ch] ? 0.f : sum;
  }
}

__global__ __launch_bounds__(kThreads) void project_kernel(GaussianPtrs g, const float* __restrict__ poses,
                                                           ViewTable vt, ProjectBufs b) {
  __shared__ uint32_t s_off[kThreads], s_org[kThreads], s_wid[kThreads];
  __shared__ uint64_t s_key[kThreads];
  __shared__ float4 s_r0[kThreads], s_r1[kThreads];   // record fields the pair test reads
  check_table(vt, b.counters);
  const int v = blockIdx.y;
  const int64_t N = g.n;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const ViewInfo cam = vt.io[v].info;
  uint32_t ntiles = 0, tx0 = 0, ty0 = 0, width = 1;
  uint64_t key = 0;
  if (i < N) {
    const float* P = poses + 12 * v;
    const int64_t m = (int64_t)v * N + i;
    // every parameter the record needs, colour included, in one round trip
    const GaussianIn in = load_gaussian(g, i);
    float rgb[3] = {0.f, 0.f, 0.f};
    if (!g.sh) {
#pragma unroll
      for (int k = 0; k < 3; ++k) rgb[k] = g.rgb[3 * i + k];
    }
    Proj o;
    if (project_core(in, P, cam, o)) {
      const double mux = (double)cam.fx * (o.p[0] / o.p[2]) + (double)cam.cx;
      const double muy = (double)cam.fy * (o.p[1] / o.p[2]) + (double)cam.cy;
      // Bounding box of the alpha >= 1/255 ellipse, widened by the margins.
      const double r2 = 2.0 * (double)logf((float)(255.0 * o.opacity)) * (double)kBinR2Rel + (double)kBinR2Abs;
      const double ex = sqrt(r2 * o.cov[0]), ey = sqrt(r2 * o.cov[2]);
      const double u0 = fmax(0.0, ceil(mux - ex)), u1 = fmin((double)(cam.width - 1), floor(mux + ex));
      const double v0 = fmax(0.0, ceil(muy - ey)), v1 = fmin((double)(cam.height - 1), floor(muy + ey));
      if (u0 <= u1 && v0 <= v1) {
        tx0 = (uint32_t)u0 / kTile;
        ty0 = (uint32_t)v0 / kTile;
        const uint32_t tx1 = (uint32_t)u1 / kTile, ty1 = (uint32_t)v1 / kTile;
        width = tx1 - tx0 + 1;
        ntiles = width * (ty1 - ty0 + 1);
        float c[3];
        if (g.sh) {
          ShColour sc;
          sh_colour(g, i, P, sc);
          c[0] = sc.col[0];
          c[1] = sc.col[1];
          c[2] = sc.col[2];
        } else {
          c[0] = rgb[0];
          c[1] = rgb[1];
          c[2] = rgb[2];
        }
        float4* rec = b.rec + kRecF4 * m;
        // The mean is kept as a float pair hi + lo; the blend kernels take it
        // relative to their tile's origin, where hi - origin is exact.
        const float hx = (float)mux, hy = (float)muy;
        // completed-square conic: a, k = b / a, c' = c - b^2 / a = 1 / Sigma2d_yy
        rec[0] = make_float4(hx, hy, (float)o.conic[0], (float)(o.conic[1] / o.conic[0]));
        rec[1] = make_float4((float)(1.0 / o.cov[2]), (float)o.opacity, (float)o.p[2], c[0]);
        rec[2] = make_float4(c[1], c[2], (float)(mux - (double)hx), (float)(muy - (double)hy));
        s_r0[threadIdx.x] = make_float4(hx, hy, (float)o.conic[0], (float)(o.conic[1] / o.conic[0]));
        s_r1[threadIdx.x] = make_float4((float)(1.0 / o.cov[2]), (float)o.opacity, (float)(mux - (double)hx),
                                        (float)(muy - (double)hy));
        const uint32_t cx0 = (uint32_t)u0 / 8u, cx1 = (uint32_t)u1 / 8u, cy0 = (uint32_t)v0 / 8u,
                       cy1 = (uint32_t)v1 / 8u;
        b.rect[m] = make_uint2(cx0 | (cx1 << 16), cy0 | (cy1 << 16));
        // key = float bits of the camera depth (positive, so the bits order
        // like the values) << 32 | record id
        key = ((uint64_t)float_key((float)o.p[2]) << 32) | (uint64_t)m;
      }
    }
    b.tiles[m] = ntiles;
  }
  // Emission: the wave's pairs spread over its lanes, each taking a slot in
  // its tile's bucket with a returning atomic -- up to kBatchPairs before
  // using any, so a lane waits once per batch -- and writing its key there.
  // A pair whose Gaussian cannot reach alpha >= 1/255 on any pixel of the
  // tile (box_reached on the tile's 16x16 square, with the record fields the
  // blends stage) is not emitted: the blends would skip it at every pixel.
  const int wv = threadIdx.x >> 6;
  const uint32_t lane = threadIdx.x & 63;
  s_key[threadIdx.x] = key;
  const WavePairs wp = wave_pairs(ntiles, tx0, ty0, width, s_off + 64 * wv, s_org + 64 * wv, s_wid + 64 * wv);
  constexpr uint32_t kBatchPairs = 8;
  constexpr uint32_t kSkip = 0xFFFFFFFFu;
  uint32_t lost = 0;   // one past the fullest slot of a pair that found its bucket full
  for (uint32_t k0 = lane; k0 < wp.total; k0 += 64 * kBatchPairs) {
    uint32_t tile[kBatchPairs], slot[kBatchPairs];
    uint64_t kk[kBatchPairs];
#pragma unroll
    for (uint32_t j = 0; j < kBatchPairs; ++j) {
      const uint32_t k = k0 + 64 * j;
      slot[j] = kSkip;
      if (k < wp.total) {
        int owner;
        const uint32_t local = pair_tile(wp, k, cam.tiles_x, &owner);
        const float4 r0 = s_r0[64 * wv + owner], r1 = s_r1[64 * wv + owner];
        const float ox = (float)((local % (uint32_t)cam.tiles_x) * kTile),
                    oy = (float)((local / (uint32_t)cam.tiles_x) * kTile);
        const float4 A = make_float4((r0.x - ox) + r1.z, (r0.y - oy) + r1.w, (-0.5f * kLog2e) * r0.z, r0.w);
        const float4 B = make_float4((-0.5f * kLog2e) * r1.x, r1.y, 0.f, 0.f);
        tile[j] = cam.tile_base + local;
        kk[j] = s_key[64 * wv + owner];
        if (box_reached(A, B, 0.f, 0.f, (float)(kTile - 1)))
          slot[j] = atomicAdd(&b.tile_count[(size_t)tile[j] * kTileCounterStride], 1u);
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < kBatchPairs; ++j) {
      if (k0 + 64 * j >= wp.total) break;
      if (slot[j] == kSkip) continue;
      if (slot[j] < b.tile_cap) b.keys[(uint64_t)tile[j] * b.tile_cap + slot[j]] = kk[j];
      else lost = max(lost, slot[j] + 1u);
    }
  }
  // Only a pair that found its bucket full reports, so the counters see no
  // atomics in a render that fits: the largest such slot is the count the
  // fullest bucket needs, for this render and (above flag_cap) sticky until
  // the next check, with the overflow flag.
  if (lost) {
    atomicMax(&b.counters[kCntRenderPeak], lost);
    if (lost > b.flag_cap) {
      atomicMax(&b.counters[kCntPeak], lost);
      b.counters[kCntOverflow] = 1u;
    }
  }
}

// Backward of project_kernel for one record.  rec_grad holds what the blend
// backward accumulated over the record's pixels: the sums u1, u2, sxx, sxy,
// syy of dL/dpower times (t, dy, dx^2, dx dy, dy^2), dL/dopacity, dL/ddepth
// and dL/dcolour; it is read and cleared here so the next backward starts
// from zero.
__global__ __launch_bounds__(kThreads) void project_backward_kernel(GaussianPtrs g, const float* __restrict__ poses,
                                                                    ViewTable vt, float* rec_grad,
                                                                    const uint32_t* __restrict__ tiles,
                                                                    GradPtrs dg, int param_grads, int atomic_params,
                                                                    int view_loop, double* pose_acc, float* dens_grad,
                                                                    uint32_t* dens_count, uint32_t* counters) {
  __shared__ float s_pose[2][4][6];
  check_table(vt, counters);
  const int64_t N = g.n;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  // view_loop: a lane walks its Gaussian's records of every view, so it owns
  // the Gaussian's parameter gradients and adds to them without atomics;
  // otherwise blockIdx.y is the view.
  const int v_begin = view_loop ? 0 : (int)blockIdx.y;
  const int v_end = view_loop ? vt.n : v_begin + 1;
  for (int v = v_begin; v < v_end; ++v) {
    const int64_t m = (int64_t)v * N + i;
    float gp[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < N && tiles[m] != 0u) {
      float4* gr = reinterpret_cast<float4*>(rec_grad + (int64_t)kGradStride * m);
      const float4 g0 = gr[0], g1 = gr[1], g2 = gr[2];
      const GaussianIn in = load_gaussian(g, i);   // with the sums, one round trip
      gr[0] = make_float4(0.f, 0.f, 0.f, 0.f);
      gr[1] = make_float4(0.f, 0.f, 0.f, 0.f);
      gr[2] = make_float4(0.f, 0.f, 0.f, 0.f);
      const float dop = g1.y, dd = g1.z;
      const ViewInfo cam = vt.io[v].info;
      const float* P = poses + 12 * v;
      Proj o;
      // the record was visible in the forward at this pose, so this holds
      if (project_core(in, P, cam, o)) {
        // power = -(a t^2 + c' dy^2) / 2 with t = dx + k dy, k = b / a and
        // c' = c - b^2 / a = 1 / Sigma2d_yy (dx, dy = mu - pixel), so
        // dpower/dmu = -(a t, a k t + c' dy) and dpower/d(a, b, c) =
        // -(dx^2 / 2, dx dy, dy^2 / 2).
        const double qa = o.conic[0], qk = o.conic[1] / o.conic[0], qc = 1.0 / o.cov[2];
        const float dmux = (float)(-qa * (double)g0.x);
        const float dmuy = (float)(-(qa * qk * (double)g0.x + qc * (double)g0.y));
        const float da = -0.5f * g0.z, db = -g0.w, dc = -0.5f * g1.x;
        if (dens_grad) {
          atomicAdd(dens_grad + i, sqrtf(dmux * dmux + dmuy * dmuy));
          atomicAdd(dens_count + i, 1u);
        }
        const float x = (float)o.p[0], y = (float)o.p[1], z = (float)o.p[2];
        const float zinv = 1.0f / z, zinv2 = zinv * zinv;
        // dL/dSigma2d = -Q dQ Q with the off-diagonal conic entry counted twice.
        const float a = (float)o.conic[0], b = (float)o.conic[1], c = (float)o.conic[2];
        const float hb = 0.5f * db;
        const float QG00 = a * da + b * hb, QG01 = a * hb + b * dc;
        const float QG10 = b * da + c * hb, QG11 = b * hb + c * dc;
        const float A00 = -(QG00 * a + QG01 * b);
        const float A01 = -(QG00 * b + QG01 * c);
        const float A11 = -(QG10 * b + QG11 * c);
        // Sigma2d = J Sc J^T: dSc = J^T A J, dJ = 2 A J Sc.
        const float J00 = (float)o.J00, J02 = (float)o.J02, J11 = (float)o.J11, J12 = (float)o.J12;
        float dS[6];
        dS[0] = J00 * J00 * A00;
        dS[1] = J00 * A01 * J11;
        dS[2] = J00 * (A00 * J02 + A01 * J12);
        dS[3] = J11 * J11 * A11;
        dS[4] = J11 * (A01 * J02 + A11 * J12);
        dS[5] = J02 * J02 * A00 + 2.f * J02 * J12 * A01 + J12 * J12 * A11;
        float S[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) S[k] = (float)o.Sc[k];
        // (J Sc) rows
        const float JS00 = J00 * S[0] + J02 * S[2], JS02 = J00 * S[2] + J02 * S[5];
        const float JS11 = J11 * S[3] + J12 * S[4], JS12 = J11 * S[4] + J12 * S[5];
        const float JS01 = J00 * S[1] + J02 * S[4], JS10 = J11 * S[1] + J12 * S[2];
        const float dJ00 = 2.f * (A00 * JS00 + A01 * JS10);
        const float dJ02 = 2.f * (A00 * JS02 + A01 * JS12);
        const float dJ11 = 2.f * (A01 * JS01 + A11 * JS11);
        const float dJ12 = 2.f * (A01 * JS02 + A11 * JS12);
        // Camera-space mean.
        float dp0 = dmux * cam.fx * zinv;
        float dp1 = dmuy * cam.fy * zinv;
        float dp2 = -(dmux * cam.fx * x + dmuy * cam.fy * y) * zinv2 + dd;
        dp2 -= (dJ00 * cam.fx + dJ11 * cam.fy) * zinv2;
        if (o.clampx == 0) {
          dp0 -= dJ02 * cam.fx * zinv2;
          dp2 += dJ02 * 2.f * cam.fx * x * zinv2 * zinv;
        } else {
          dp2 += dJ02 * cam.fx * o.tx * zinv2;
        }
        if (o.clampy == 0) {
          dp1 -= dJ12 * cam.fy * zinv2;
          dp2 += dJ12 * 2.f * cam.fy * y * zinv2 * zinv;
        } else {
          dp2 += dJ12 * cam.fy * o.ty * zinv2;
        }
        // View-dependent colour: colour_c = max(0, sum_k sh_kc Y_k(d) + 1/2),
        // d = v / |v|, v = X - C, C = -R^T t.  dL/dv = (I - d d^T) dL/dd / |v|
        // reaches the mean (+dL/dv) and the camera centre (-dL/dv); C moves to
        // C - R^T rho under exp(xi^) T, so dL/drho gains R dL/dv.
        float dv[3] = {0.f, 0.f, 0.f};
        if (g.sh) {
          ShColour sc;
          sh_colour(g, i, P, sc);
          const float gcol[3] = {g1.w, g2.x, g2.y};
          float dc[3];
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) dc[ch] = sc.clamped[ch] ? 0.f : gcol[ch];
          const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
          float w[16];
#pragma unroll
          for (int k = 0; k < 16; ++k)
            w[k] = k < K ? dc[0] * sc.c[3 * k] + dc[1] * sc.c[3 * k + 1] + dc[2] * sc.c[3 * k + 2] : 0.f;
          const float3 gd = sh_grad(g.sh_degree, sc.d[0], sc.d[1], sc.d[2], w);
          const float dot = gd.x * sc.d[0] + gd.y * sc.d[1] + gd.z * sc.d[2];
          dv[0] = (gd.x - sc.d[0] * dot) * sc.inv_len;
          dv[1] = (gd.y - sc.d[1] * dot) * sc.inv_len;
          dv[2] = (gd.z - sc.d[2] * dot) * sc.inv_len;
          if (param_grads && dg.sh) {
            float* out = dg.sh + (int64_t)3 * K * i;
            if (!atomic_params && sh_vector(dg.sh, K)) {
              // 16-byte read-modify-writes of the Gaussian's block (48 scalar
              // ones took 49 of the 114 us of a 500k-Gaussian degree-3 view)
              float4* o4 = reinterpret_cast<float4*>(out);
#pragma unroll
              for (int q = 0; q < 12; ++q) {
                if (4 * q < 3 * K) {
                  float4 v = o4[q];
                  v.x += dc[(4 * q) % 3] * sc.Y[(4 * q) / 3];
                  v.y += dc[(4 * q + 1) % 3] * sc.Y[(4 * q + 1) / 3];
                  v.z += dc[(4 * q + 2) % 3] * sc.Y[(4 * q + 2) / 3];
                  v.w += dc[(4 * q + 3) % 3] * sc.Y[(4 * q + 3) / 3];
                  o4[q] = v;
                }
              }
            } else {
#pragma unroll
              for (int k = 0; k < 16; ++k) {
                if (k < K) {
#pragma unroll
                  for (int ch = 0; ch < 3; ++ch) {
                    const float val = dc[ch] * sc.Y[k];
                    if (atomic_params) unsafeAtomicAdd(out + 3 * k + ch, val);
                    else out[3 * k + ch] += val;
                  }
                }
              }
            }
          }
        }
        if (param_grads) {
          // Means: p = W X + t.
          float dX[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) dX[k] = P[k] * dp0 + P[3 + k] * dp1 + P[6 + k] * dp2;
          // dSigma = W^T dSc W (symmetric, full 3x3 for the products below).
          const float dSf[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
          float T1[9], dSig[9];
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              T1[3 * r + cc] = P[r] * dSf[cc] + P[3 + r] * dSf[3 + cc] + P[6 + r] * dSf[6 + cc];
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              dSig[3 * r + cc] = T1[3 * r] * P[cc] + T1[3 * r + 1] * P[3 + cc] + T1[3 * r + 2] * P[6 + cc];
          // Sigma = sum_k s_k^2 r_k r_k^T.
          float dls[3], dR[9];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            float quad = 0.f;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
              for (int cc = 0; cc < 3; ++cc) quad += o.R[3 * r + k] * dSig[3 * r + cc] * o.R[3 * cc + k];
            dls[k] = 2.f * o.s[k] * o.s[k] * quad;
          }
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              dR[3 * r + cc] =
                  2.f * (dSig[3 * r] * o.R[cc] + dSig[3 * r + 1] * o.R[3 + cc] + dSig[3 * r + 2] * o.R[6 + cc]) *
                  o.s[cc] * o.s[cc];
          const float w = o.qn[0], qx = o.qn[1], qy = o.qn[2], qz = o.qn[3];
          float dq[4];
          dq[0] = 2.f * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
          dq[1] = 2.f * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.f * qx * dR[4] - w * dR[5] + qz * dR[6] + w * dR[7] -
                         2.f * qx * dR[8]);
          dq[2] = 2.f * (-2.f * qy * dR[0] + qx * dR[1] + w * dR[2] + qx * dR[3] + qz * dR[5] - w * dR[6] + qz * dR[7] -
                         2.f * qy * dR[8]);
          dq[3] = 2.f * (-2.f * qz * dR[0] - w * dR[1] + qx * dR[2] + w * dR[3] - 2.f * qz * dR[4] + qy * dR[5] +
                         qx * dR[6] + qy * dR[7]);
          const float dotq = o.qn[0] * dq[0] + o.qn[1] * dq[1] + o.qn[2] * dq[2] + o.qn[3] * dq[3];
          const float dlogit = dop * o.opacity * (1.f - o.opacity);
          float* outs[5] = {dg.means, dg.log_scales, dg.quats, dg.opacity_logits, dg.rgb};
          float vals_mean[3] = {dX[0], dX[1], dX[2]};
          auto put = [&](float* base, int64_t idx, float val) {
            if (!base) return;
            if (atomic_params) unsafeAtomicAdd(base + idx, val);
            else base[idx] += val;
          };
          for (int k = 0; k < 3; ++k) vals_mean[k] += dv[k];
          for (int k = 0; k < 3; ++k) put(outs[0], 3 * i + k, vals_mean[k]);
          for (int k = 0; k < 3; ++k) put(outs[1], 3 * i + k, dls[k]);
          for (int k = 0; k < 4; ++k) put(outs[2], 4 * i + k, (dq[k] - o.qn[k] * dotq) * o.qinv);
          put(outs[3], i, dlogit);
          if (!g.sh) {
            put(outs[4], 3 * i + 0, g1.w);
            put(outs[4], 3 * i + 1, g2.x);
            put(outs[4], 3 * i + 2, g2.y);
          }
        }
        // Pose, left perturbation: drho = dp; dphi = p x dp + 2 vee(skew(Sc dSc)).
        const float Sf[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
        const float dSf[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
        auto Mrc = [&](int r, int cc) {
          return Sf[3 * r] * dSf[cc] + Sf[3 * r + 1] * dSf[3 + cc] + Sf[3 * r + 2] * dSf[6 + cc];
        };
        gp[0] = dp0 + P[0] * dv[0] + P[1] * dv[1] + P[2] * dv[2];
        gp[1] = dp1 + P[3] * dv[0] + P[4] * dv[1] + P[5] * dv[2];
        gp[2] = dp2 + P[6] * dv[0] + P[7] * dv[1] + P[8] * dv[2];
        gp[3] = y * dp2 - z * dp1 + 2.f * (Mrc(1, 2) - Mrc(2, 1));
        gp[4] = z * dp0 - x * dp2 + 2.f * (Mrc(2, 0) - Mrc(0, 2));
        gp[5] = x * dp1 - y * dp0 + 2.f * (Mrc(0, 1) - Mrc(1, 0));
      }
    }
    if (pose_acc) {
      // Workgroup reduction of the six pose terms, then one double atomic each;
      // pose_finalize_kernel hands the sums to the caller.  Views alternate
      // between two LDS slots, so the next view's writes cannot meet this
      // view's reads.
      float (*sp)[6] = s_pose[v & 1];
      const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
      const float t6 = wave_sum_many<8>(gp);
      const int idx = reduced_value_index<8>(lane);
      if ((lane & 7) == 0 && idx < 6) sp[w][idx] = t6;
      __syncthreads();
      if (threadIdx.x < 6) {
        const float t = sp[0][threadIdx.x] + sp[1][threadIdx.x] + sp[2][threadIdx.x] + sp[3][threadIdx.x];
        if (t != 0.f) atomicAdd(pose_acc + 6 * v + threadIdx.x, (double)t);
      }
    }
  }
}

// One wave per view, lane k on component k: hands the summed pose gradient
// to the caller (dposes +=) and/or to an Adam step with retraction, and
// clears the accumulator.
__global__ __launch_bounds__(64) void pose_finalize_kernel(double* pose_acc, float* dposes, float* poses, float* adam,
                                                           AdamParams ap) {
  const int v = blockIdx.x, k = threadIdx.x;
  float g = 0.f;
  if (k < 6) {
    g = (float)pose_acc[6 * v + k];
    pose_acc[6 * v + k] = 0.0;
    if (dposes) dposes[6 * v + k] += g;
  }
  if (adam) adam_retract_wave(poses + 12 * v, adam + 16 * v, g, ap);
}

}  // namespace

void launch_project(const GaussianPtrs& g, const float* poses, const ViewTable& vt, const ProjectBufs& b,
                    hipStream_t s) {
  const dim3 grid((unsigned)std::max<int64_t>(1, (g.n + kThreads - 1) / kThreads), (unsigned)vt.n);
  hipLaunchKernelGGL(project_kernel, grid, dim3(kThreads), 0, s, g, poses, vt, b);
}

void launch_project_backward(const GaussianPtrs& g, const float* poses, const ViewTable& vt, float* rec_grad,
                             const uint32_t* tiles, const GradPtrs& dg, bool param_grads, double* pose_acc,
                             float* dposes, const PoseStep* step, float* dens_grad, uint32_t* dens_count,
                             uint32_t* counters, hipStream_t s) {
  // Several views: one lane per Gaussian over all views (no atomics on the
  // parameter gradients, one workgroup per Gaussian block instead of one per
  // (view, block)); one view: one grid row.
  const bool view_loop = vt.n > 1;
  const dim3 grid((unsigned)std::max<int64_t>(1, (g.n + kThreads - 1) / kThreads), view_loop ? 1u : (unsigned)vt.n);
  const bool pose = dposes || step;
  hipLaunchKernelGGL(project_backward_kernel, grid, dim3(kThreads), 0, s, g, poses, vt, rec_grad, tiles, dg,
                     param_grads ? 1 : 0, (vt.n > 1 && !view_loop) ? 1 : 0, view_loop ? 1 : 0,
                     pose ? pose_acc : nullptr, dens_grad, dens_count, counters);
  if (pose)
    hipLaunchKernelGGL(pose_finalize_kernel, dim3((unsigned)vt.n), dim3(64), 0, s, pose_acc, dposes,
                       step ? step->poses : nullptr, step ? step->adam : nullptr,
                       step ? step->params : AdamParams{0.f, 0.f, 0.f, 0.f, 1.f});
}

}  // namespace cgsr
