// Tile blending, forward (Sec. 3.1 Eq. 3-9, Sec. 3.2 Eq. 10) and backward.
//
// One workgroup per 16x16 tile.  A lane owns kPPL pixels (1, 2 or 4), so a
// tile takes 256 / kPPL lanes; pixel q of the tile lies in the 8x8 quadrant
// q / 64, and lane t owns pixels t, t + L, t + 2L, ... (L lanes), so a wave's
// pixels are whole quadrants and leave together.  The tile's depth-ordered
// records are staged through LDS kBatch at a time (see stage_record); every lane
// then reads the same LDS address, a broadcast free of bank conflicts, and
// uses it for all of its pixels.
//
// Each wave stages its own copy of the batch holding only the records whose
// binning rectangle reaches one of its 8x8 quadrants (the projection keeps
// the rectangle in 8-pixel cells) and whose alpha >= 1/255 region does by the
// closed-form test box_reached, so a wave walks a list shorter than 8x8
// binning's while the sort and the tile buckets stay at 16x16.  A record left
// out of a wave's copy has alpha below 1/255 at every one of its pixels, so
// the results are exactly those of walking the whole tile list.
//
// kNu (mapping renders) also keeps, per pixel, the blended Gaussian of
// largest weight alpha T -- the pixel is "dominated" by it (Sec. 3.2,
// Eq. 13) -- and at the end adds w (D - d)^2 and 1 to that Gaussian's
// uncertainty sum and count when the pixel has a sensor depth D > 0.
//
// Tracking mode (kTrack) forms the gradient images of the tracking loss
// (Eq. 19: L1 colour, Eq. 14, and L1 depth, Eq. 16) at the end of the
// forward, straight from the blended values in registers.  The loss is per
// pixel, so a tile's backward needs nothing from other tiles:
// raster_track_kernel runs the forward and the pose backward of a tile in one
// workgroup, the per-pixel state never leaves registers, and the records
// staged for the forward are reused by the backward when the tile's list fits
// one batch; when every bucket holds at most one key per thread it also sorts
// its own bucket first (no separate sort launch).  The separate kernels serve
// rendering and the mapping backward.
#include "kernels.hpp"

namespace cgsr {
namespace {

constexpr int kBatch = 128;   // tile-list entries staged at a time
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

// Wave priority from the work ahead (s_setprio).  The workgroups of a frame
// are all resident from the start (1200 tiles of 640x480 fit the chip at
// once), so a launch lasts as long as its longest tiles, whose waves share
// their SIMDs with shorter ones.  Letting the waves with the longest lists
// issue first, while shorter ones fill the gaps, brings the long tiles' end
// forward: the fused tracking blend went from 34.3 to 31.0 us and the
// single-view mapping blends from 0.320 to 0.310 ms.  The levels are list
// lengths of the workloads measured (tracking: 46 entries per 16x16 tile
// and 29 per 8x8 quadrant on average; mapping: about 200 per tile).
// n must be wave-uniform.
__device__ __forceinline__ void prioritise(uint32_t n, uint32_t t1, uint32_t t2, uint32_t t3) {
  if (n >= t3) __builtin_amdgcn_s_setprio(3);
  else if (n >= t2) __builtin_amdgcn_s_setprio(2);
  else if (n >= t1) __builtin_amdgcn_s_setprio(1);
}
// tracking: tile list, quadrant list; mapping: tile list
constexpr uint32_t kTrackTilePrio[3] = {45, 60, 80};
constexpr uint32_t kTrackWavePrio[3] = {28, 36, 44};
constexpr uint32_t kMapTilePrio[3] = {180, 240, 320};

// The LDS batch of staged records (see stage_record) and their record ids,
// one compacted copy per wave (W waves per tile), and each copy's length.
// B.w of a staged record holds one past its position in the tile's list and
// C.w its record id (as int bits), so a walk compares the position with its
// pixel's bounds without arithmetic and reads the id with the record.
template <int W>
struct Stage {
  float4 A[W][kBatch], B[W][kBatch], C[W][kBatch];
  uint32_t cnt[W];
  uint32_t scan[4];
};

// Whether wave w of W takes a staged record: one of its quadrants (q / 64 of
// pixel q, see pixel_of: w, w + W, ..., kPPL = 4 / W of them) lies in the
// record's binning rectangle (8-pixel cells) and box_reached passes for it.
template <int W>
__device__ __forceinline__ bool wave_takes(int w, uint32_t cx0, uint32_t cx1, uint32_t cy0, uint32_t cy1,
                                           uint32_t tcx, uint32_t tcy, const float4& A, const float4& B) {
  bool any = false;
#pragma unroll
  for (int k = 0; k < 4 / W; ++k) {
    const int qd = w + k * W;
    const uint32_t cx = tcx + (qd & 1), cy = tcy + (qd >> 1);
    if (cx0 <= cx && cx <= cx1 && cy0 <= cy && cy <= cy1)
      any = any || box_reached(A, B, (float)(8 * (qd & 1)), (float)(8 * (qd >> 1)), 7.f);
  }
  return any;
}

// Stages n <= kBatch entries of the tile's list, record ids ids[0, n), into
// each wave's copy; every thread calls it.  pos0: the position of ids[0] in
// the tile's list.  (tcx, tcy): the tile's first 8-pixel cell.  With one wave
// per tile every record reaches it.  kPerWave: each wave stages its copy on
// its own (tracking), else the block shares the loads and tests (mapping).
template <int L, int W, bool kPerWave>
__device__ __forceinline__ void stage_batch(const RasterBufs& b, Stage<W>& s, const uint32_t* ids, uint32_t pos0,
                                            int n, float2 org, uint32_t tcx, uint32_t tcy, int rot = 0) {
  __syncthreads();
  if constexpr (W == 1) {
    for (int i = threadIdx.x; i < n; i += L) {
      const uint32_t m = ids[i];
      float4 B, C;
      stage_record(b.rec + (int64_t)kRecF4 * m, org.x, org.y, s.A[0][i], B, C);
      B.w = __int_as_float((int)(pos0 + i + 1));
      C.w = __uint_as_float(m);
      s.B[0][i] = B;
      s.C[0][i] = C;
    }
    if (threadIdx.x == 0) s.cnt[0] = (uint32_t)n;
  } else if constexpr (kPerWave) {
    // Each wave builds its own copy: lane l takes entries l, l + 64 of the
    // batch, tests them against the wave's own quadrants, and the entries it
    // keeps go to consecutive slots in list order (ballot rank).  Every wave
    // loads and tests the whole batch, but none waits on a block scan or on
    // one thread testing all quadrants: the shorter path for latency-bound
    // tracking tiles.
    static_assert(kBatch <= 2 * kWave, "two entries per lane");
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    uint32_t cnt = 0;
#pragma unroll
    for (int r0 = 0; r0 < kBatch; r0 += kWave) {
      if (r0 >= n) break;
      const int i = r0 + lane;
      bool take = false;
      float4 A, B, C;
      if (i < n) {
        const uint32_t m = ids[i];
        stage_record(b.rec + (int64_t)kRecF4 * m, org.x, org.y, A, B, C);
        B.w = __int_as_float((int)(pos0 + i + 1));
        C.w = __uint_as_float(m);
        const uint2 r = b.rect[m];
        take = wave_takes<W>(W == 4 ? ((wv + rot) & 3) : wv, r.x & 0xFFFFu, r.x >> 16, r.y & 0xFFFFu, r.y >> 16, tcx,
                             tcy, A, B);
      }
      const uint64_t bal = __ballot(take);
      if (take) {
        const uint32_t d =
            cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        s.A[wv][d] = A;
        s.B[wv][d] = B;
        s.C[wv][d] = C;
      }
      cnt += (uint32_t)__popcll(bal);
    }
    if (lane == 0) s.cnt[wv] = cnt;
  } else {
    // L >= kBatch: one record per thread, tested against every wave's
    // quadrants.  A byte per wave counts the records it takes; their
    // exclusive prefix over the threads is the record's slot in that wave's
    // copy (no byte exceeds kBatch < 256).
    static_assert(L >= kBatch && W <= 4, "one record per thread");
    const int i = threadIdx.x;
    uint32_t take = 0, m = 0;
    float4 A, B, C;
    if (i < n) {
      m = ids[i];
      stage_record(b.rec + (int64_t)kRecF4 * m, org.x, org.y, A, B, C);
      B.w = __int_as_float((int)(pos0 + i + 1));
      C.w = __uint_as_float(m);
      const uint2 r = b.rect[m];
      const uint32_t cx0 = r.x & 0xFFFFu, cx1 = r.x >> 16, cy0 = r.y & 0xFFFFu, cy1 = r.y >> 16;
#pragma unroll
      for (int w = 0; w < W; ++w) take |= wave_takes<W>(w, cx0, cx1, cy0, cy1, tcx, tcy, A, B) ? 1u << (8 * w) : 0u;
    }
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    uint32_t inc = take;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d);
      if (lane >= d) inc += y;
    }
    if (lane == kWave - 1) s.scan[wv] = inc;
    __syncthreads();
    uint32_t pre = inc - take, total = 0;
#pragma unroll
    for (int q = 0; q < L / kWave; ++q) {
      pre += q < wv ? s.scan[q] : 0u;
      total += s.scan[q];
    }
#pragma unroll
    for (int w = 0; w < W; ++w)
      if ((take >> (8 * w)) & 1u) {
        const uint32_t d = (pre >> (8 * w)) & 0xFFu;
        s.A[w][d] = A;
        s.B[w][d] = B;
        s.C[w][d] = C;
      }
    if (threadIdx.x < W) s.cnt[threadIdx.x] = (total >> (8 * threadIdx.x)) & 0xFFu;
  }
  __syncthreads();
}

// Per-lane state of the forward walk.
template <int kPPL>
struct FwdPix {
  float fx[kPPL], fy[kPPL], dobs[kPPL], T[kPPL], C0[kPPL], C1[kPPL], C2[kPPL], D[kPPL], U[kPPL],
      Dmed[kPPL];
  int64_t pix[kPPL];
  uint32_t med1[kPPL];            // one past the median's position in the tile's list, 0 if none
  uint32_t last[kPPL], evaluated[kPPL], blended[kPPL], wlast[kPPL];
  uint32_t wave_len;   // entries of the wave's list the walk went through
  float wdom[kPPL], ddom[kPPL];   // kNu: largest weight so far and its depth
  uint32_t dom[kPPL];             // kNu: its record id, kNone if none
  bool inside[kPPL], done[kPPL];
};

// Front-to-back walk of the tile's list (Eq. 3-9, Eq. 10 with kTrack off).
// On return the stage holds the last batch walked; that is the whole list when
// it fits one batch.  evaluated, wlast and blended count entries of the
// wave's own (8x8) list; last and med1 are one past positions in the tile's
// list.  With kFull off (a tracking step that keeps no statistics) the walk
// keeps only what the tracking loss and the pose backward read: colour,
// depth, transmittance and the last blended entry; kStats off (no work
// counts) drops evaluated, wlast and blended alone.
// ids: the tile's record ids in list order.
template <int kPPL, bool kTrack, bool kNu, bool kFull = true, bool kStats = kFull>
__device__ __forceinline__ void forward_tile(const RasterBufs& b, Stage<kTilePixels / kPPL / kWave>& s, int gtile,
                                             const ViewIO& io, float2 org, uint2 range, const uint32_t* ids,
                                             FwdPix<kPPL>& f, int rot = 0) {
  constexpr int L = kTilePixels / kPPL;
  constexpr int W = L / kWave;
  const int wv = threadIdx.x / kWave;
  const uint32_t tcx = (uint32_t)org.x / 8u, tcy = (uint32_t)org.y / 8u;
  uint32_t loc = 0;   // entries of the wave's list before this batch
  const ViewInfo& cam = io.info;
  bool lane_done = true;
#pragma unroll
  for (int k = 0; k < kPPL; ++k) {
    const int q = k * L + threadIdx.x;   // quadrant q / 64, turned by rot
    const PixelCoord pc = pixel_of(cam, gtile, ((((q >> 6) + rot) & 3) << 6) | (q & 63));
    f.fx[k] = (float)(pc.px - pc.ox);
    f.fy[k] = (float)(pc.py - pc.oy);
    f.inside[k] = pc.inside;
    f.pix[k] = (int64_t)pc.py * cam.width + pc.px;
    f.dobs[k] = (!kTrack && io.depth_obs && pc.inside) ? io.depth_obs[f.pix[k]] : 0.f;
    f.T[k] = 1.f;
    f.C0[k] = f.C1[k] = f.C2[k] = f.D[k] = f.U[k] = f.Dmed[k] = 0.f;
    f.med1[k] = 0;
    f.last[k] = 0;
    f.blended[k] = 0;
    f.wdom[k] = f.ddom[k] = 0.f;
    f.dom[k] = kNone;
    f.evaluated[k] = 0;
    f.wlast[k] = 0;
    f.done[k] = !pc.inside;
    lane_done = lane_done && f.done[k];
  }
  for (uint32_t base = range.x; base < range.y; base += kBatch) {
    const int n = (int)min((uint32_t)kBatch, range.y - base);
    stage_batch<L, W, kTrack>(b, s, ids + (base - range.x), base - range.x, n, org, tcx, tcy, rot);
    // the copy's length is the same for the whole wave
    const int nw = (int)__builtin_amdgcn_readfirstlane(s.cnt[wv]);
    if (kTrack && base == range.x) prioritise((uint32_t)nw, kTrackWavePrio[0], kTrackWavePrio[1], kTrackWavePrio[2]);
    // The wave walks the whole batch while any of its lanes still blends;
    // lanes that are done ride along predicated off.  (A vote every few
    // records to leave early cost more issue slots than it saved: at tracking
    // sizes most pixels never reach the stop threshold.)
    if (__ballot(!lane_done) != 0ull) {
      for (int j = 0; j < nw; ++j) {
        const float4 A = s.A[wv][j];
        const float4 B = s.B[wv][j];
        const float4 Cc = s.C[wv][j];
        const uint32_t pos1 = (uint32_t)__float_as_int(B.w);   // one past its position in the tile's list
        // Straight-line, predicated per lane: a lane that skips (alpha below
        // 1/255, or already done) adds exact zeros, so the results are those
        // of the branching form, without exec-mask bookkeeping per record.
#pragma unroll
        for (int k = 0; k < kPPL; ++k) {
          float dx, dy, tq;
          const float e = pair_exponent(A, B, f.fx[k], f.fy[k], dx, dy, tq);
          const float raw = B.y * __builtin_amdgcn_exp2f(e);
          const bool hit = !f.done[k] && raw >= kAlphaMin;
          const float alpha = fminf(kAlphaMax, raw);
          const float wa = alpha * f.T[k];
          const float Tn = f.T[k] - wa;
          // Blend or stop splits the hits.  The issue-bound mapping walks take
          // it from one compare; the tracking walk, bound by latency, ran
          // slower that way.
          bool stop, blend;
          if constexpr (kTrack) {
            stop = hit && Tn < kTStop;
            blend = hit && !stop;
          } else {
            blend = hit && Tn >= kTStop;   // Tn is finite
            stop = hit != blend;
          }
          f.done[k] = f.done[k] || stop;
          if (kStats) f.evaluated[k] = stop ? loc + j + 1 : f.evaluated[k];
          const float wgt = blend ? wa : 0.f;
          f.C0[k] = __builtin_fmaf(wgt, Cc.x, f.C0[k]);
          f.C1[k] = __builtin_fmaf(wgt, Cc.y, f.C1[k]);
          f.C2[k] = __builtin_fmaf(wgt, Cc.z, f.C2[k]);
          f.D[k] = __builtin_fmaf(wgt, B.z, f.D[k]);
          if (!kTrack) {
            const float dz = B.z - f.dobs[k];
            f.U[k] = __builtin_fmaf(wgt * dz, dz, f.U[k]);
          }
          if (kFull) {
            const bool first_med = blend && f.med1[k] == 0u && Tn < kTMedian;
            f.med1[k] = first_med ? pos1 : f.med1[k];
            f.Dmed[k] = first_med ? B.z : f.Dmed[k];
          }
          if (kNu) {
            const bool more = blend && wgt > f.wdom[k];   // strict: the first of equal maxima
            f.wdom[k] = more ? wgt : f.wdom[k];
            f.ddom[k] = more ? B.z : f.ddom[k];
            f.dom[k] = more ? __float_as_uint(Cc.w) : f.dom[k];
          }
          f.T[k] = blend ? Tn : f.T[k];
          f.last[k] = blend ? pos1 : f.last[k];
          if (kStats) {
            f.wlast[k] = blend ? loc + j + 1 : f.wlast[k];
            f.blended[k] += blend ? 1u : 0u;
          }
        }
      }
      bool all = true;
#pragma unroll
      for (int k = 0; k < kPPL; ++k) all = all && f.done[k];
      lane_done = all;
    }
    loc += (uint32_t)nw;
    if (__syncthreads_count(lane_done) == L) break;
  }
  // a pixel that never stopped evaluated every entry of its wave's list
#pragma unroll
  for (int k = 0; k < kPPL; ++k) f.evaluated[k] = f.evaluated[k] ? f.evaluated[k] : loc;
  f.wave_len = loc;
}

// Everything the forward leaves behind: maps, saved per-pixel state, the
// tracking-loss gradients (returned in g; stored for a separate backward when
// store_grad) and the Eq. 13 accumulation.
// Without kFull only the colour and depth maps are written (the tracking
// step requests none) and no per-pixel state is saved; without kStats the
// saved state holds no work counts.
template <int kPPL, bool kTrack, bool kNu, bool kFull = true, bool kStats = kFull>
__device__ __forceinline__ void forward_outputs(const RasterBufs& b, int v, const ViewIO& io,
                                                const FwdPix<kPPL>& f, float (&g)[kPPL][4], bool store_grad) {
  const ViewInfo& cam = io.info;
  const int64_t hw = (int64_t)cam.width * cam.height;
  if (kTrack) {
    // dL/dcolour and dL/ddepth of L = lc mean_n |I^ - I|_1 + ld mean_n |D^ - D|.
    float l = 0.f;
    const float inv = 1.0f / (float)hw;
    const float lc = b.lambda_color * inv, ld = b.lambda_depth * inv;
#pragma unroll
    for (int k = 0; k < kPPL; ++k) {
      g[k][0] = g[k][1] = g[k][2] = g[k][3] = 0.f;
      if (!f.inside[k]) continue;
      const int64_t p = f.pix[k];
      const float e0 = f.C0[k] - io.t_color[p], e1 = f.C1[k] - io.t_color[hw + p],
                  e2 = f.C2[k] - io.t_color[2 * hw + p];
      const float ed = f.D[k] - io.t_depth[p];
      g[k][0] = lc * sgn(e0);
      g[k][1] = lc * sgn(e1);
      g[k][2] = lc * sgn(e2);
      g[k][3] = ld * sgn(ed);
      if (store_grad) b.pixel_grad[cam.pixel_base + p] = make_float4(g[k][0], g[k][1], g[k][2], g[k][3]);
      l += lc * (fabsf(e0) + fabsf(e1) + fabsf(e2)) + ld * fabsf(ed);
    }
    if (b.loss) {
      const float t = wave_sum(l);
      if ((threadIdx.x & 63) == 0 && t != 0.f) atomicAdd(b.loss + v, t);
    }
  }
#pragma unroll
  for (int k = 0; k < kPPL; ++k) {
    if (!f.inside[k]) continue;
    const int64_t p = f.pix[k];
    if (io.color) {
      io.color[p] = f.C0[k];
      io.color[hw + p] = f.C1[k];
      io.color[2 * hw + p] = f.C2[k];
    }
    if (io.depth) io.depth[p] = f.D[k];
    if (!kFull) continue;
    // Eq. 9's sum of the blend weights: each weight is the drop in
    // transmittance it causes, so the sum is 1 - T (up to rounding)
    if (io.opacity) io.opacity[p] = 1.f - f.T[k];
    if (io.depth_median) io.depth_median[p] = f.Dmed[k];
    if (io.uncertainty) io.uncertainty[p] = f.U[k];
    // the median's position, or ~0u if it has none
    b.pixel_state[cam.pixel_base + p] =
        make_uint4(__float_as_uint(f.T[k]), f.last[k], f.med1[k] - 1u, kStats ? f.evaluated[k] : 0u);
    if (kStats) b.pixel_count[cam.pixel_base + p] = make_uint2(f.blended[k], f.wlast[k]);
    if (kNu) {
      // record id m = view * N + Gaussian index
      const int gi = f.dom[k] == kNone ? -1 : (int)(f.dom[k] - (uint32_t)v * (uint32_t)b.views.n_gauss);
      if (io.dominant) io.dominant[p] = gi;
      if (gi >= 0 && f.dobs[k] > 0.f && b.nu_sum) {
        const float e = f.dobs[k] - f.ddom[k];
        unsafeAtomicAdd(b.nu_sum + gi, f.wdom[k] * e * e);
        atomicAdd(b.nu_count + gi, 1u);
      }
    }
  }
}

// Per-lane state of the backward walk.
template <int kPPL>
struct BwdPix {
  float fx[kPPL], fy[kPPL], T[kPPL], gc0[kPPL], gc1[kPPL], gc2[kPPL], gd[kPPL], go[kPPL], gm[kPPL], gu[kPPL],
      dobs[kPPL];
  float gu2[kPPL];   // 2 gu
  float Bg[kPPL];   // sum_x g_x Bx, the behind sums weighted by the pixel's upstream gradients
  int walked[kPPL], med1[kPPL];   // one past the last blended entry's / the median's position (0: none)
};

// Largest walked length over the workgroup.
__device__ __forceinline__ int block_max(uint32_t lane_max, uint32_t* s_max) {
  __syncthreads();
  if (threadIdx.x == 0) *s_max = 0u;
  __syncthreads();
  if (lane_max) atomicMax(s_max, lane_max);
  __syncthreads();
  return (int)*s_max;
}

// Back-to-front over each pixel's blended run.  With the normalised "behind"
// sums Bx = sum_{k>j} w_k x_k / T_{j+1}, dL/dalpha_j = T_j sum_x g_x (x_j - Bx)
// = T_j (G_j - Bg) with G_j = sum_x g_x x_j and Bg = sum_x g_x Bx; since every
// Bx moves one Gaussian forward as Bx <- alpha_j x_j + (1 - alpha_j) Bx and
// the g_x are fixed per pixel, so does Bg <- Bg + alpha_j (G_j - Bg) (one
// multiply-add on the G_j - Bg that dL/dalpha_j needs anyway), one running
// sum for all the quantities x (colour, depth, opacity, uncertainty).
// T_j = T_{j+1} / (1 - alpha_j) recovers the transmittance from the final
// one.
// A lane first sums its pixels' contributions to a Gaussian, then the wave
// reduces all of the Gaussian's gradient terms together (wave_sum_many) and
// issues one atomic instruction.  kParams adds the opacity and colour
// gradients (mapping); kColor alone adds the colour gradients (the pose
// gradient needs them when the colour depends on the viewpoint); kTrack has
// colour and depth upstream gradients only.
// staged_n > 0: the stage already holds list entries [0, staged_n).
template <int kPPL, bool kParams, bool kTrack, bool kColor = false>
__device__ __forceinline__ void backward_tile(const RasterBufs& b, Stage<kTilePixels / kPPL / kWave>& s, uint2 range,
                                              float2 org, int nmax, int staged_n, BwdPix<kPPL>& p, int rot = 0) {
  constexpr int L = kTilePixels / kPPL;
  constexpr int W = L / kWave;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x / kWave;
  const uint32_t tcx = (uint32_t)org.x / 8u, tcy = (uint32_t)org.y / 8u;
  for (int end = nmax; end > 0; end -= kBatch) {
    const int start = max(0, end - kBatch);
    const int n = end - start;
    if (!(start == 0 && end <= staged_n))
      stage_batch<L, W, kTrack>(b, s, b.vals + range.x + start, start, n, org, tcx, tcy, rot);
    for (int j = (int)__builtin_amdgcn_readfirstlane(s.cnt[wv]) - 1; j >= 0; --j) {
      const float4 A = s.A[wv][j];
      const float4 B = s.B[wv][j];
      float u1 = 0.f, u2 = 0.f, sxx = 0.f, sxy = 0.f, syy = 0.f, gop = 0.f, gdd = 0.f;
      float gr = 0.f, gg = 0.f, gbl = 0.f;
      bool any = false;
      const float4 Cc = s.C[wv][j];
      const int pos1 = __float_as_int(B.w);   // one past its position in the tile's list
      const uint32_t m = __float_as_uint(Cc.w);
      // Straight-line, predicated per lane: a lane that did not blend this
      // record (past its last blended one, or alpha below 1/255) takes
      // alpha = 0, which leaves T and the behind sums exactly unchanged and
      // adds exact zeros to every gradient term.
#pragma unroll
      for (int k = 0; k < kPPL; ++k) {
        float dx, dy, tq;
        const float e = pair_exponent(A, B, p.fx[k], p.fy[k], dx, dy, tq);
        const float g = __builtin_amdgcn_exp2f(e);
        const float raw = B.y * g;
        const bool hit = pos1 <= p.walked[k] && raw >= kAlphaMin;
        any = any || hit;
        const float alpha = hit ? fminf(kAlphaMax, raw) : 0.f;
        const float oma = 1.f - alpha;
        const float Tj = p.T[k] * __builtin_amdgcn_rcpf(oma);
        const float wgt = alpha * Tj;
        float G = __builtin_fmaf(p.gc0[k], Cc.x,
                                 __builtin_fmaf(p.gc1[k], Cc.y, __builtin_fmaf(p.gc2[k], Cc.z, p.gd[k] * B.z)));
        float dz = 0.f;
        if (!kTrack) {
          dz = B.z - p.dobs[k];
          G = __builtin_fmaf(p.gu[k], dz * dz, G + p.go[k]);
        }
        const float dsum = G - p.Bg[k];
        p.Bg[k] = __builtin_fmaf(alpha, dsum, p.Bg[k]);
        const float dalpha = Tj * dsum;
        p.T[k] = Tj;
        const bool live = hit && !(raw > kAlphaMax);   // a capped alpha has no gradient
        const float dlive = live ? dalpha : 0.f;
        const float dpower = dlive * raw;   // alpha = opacity * exp(power)
        // power = -(a dx^2 + 2 b dx dy + c dy^2) / 2 = ln2 (qa t^2 + qc dy^2)
        // with t = dx + k dy, so d power/d mu = 2 ln2 (qa t, qa k t + qc dy)
        // and d power/d(a, b, c) = -(dx^2 / 2, dx dy, dy^2 / 2).  These are
        // linear in the sums u1 = sum dpower t, u2 = sum dpower dy and the
        // second moments, so lanes, waves and tiles only add those up; the
        // factors that belong to the record (qa, k, qc, the constants) are
        // applied once per record by the projection backward.
        const float pdx = dpower * dx, pdy = dpower * dy;
        // the first pixel's terms start the sums, so nothing adds a zero
        auto acc = [&](float& sum, float x) { sum = k == 0 ? x : sum + x; };
        auto acc_fma = [&](float& sum, float x, float y) { sum = k == 0 ? x * y : __builtin_fmaf(x, y, sum); };
        acc_fma(u1, dpower, tq);
        acc(u2, pdy);
        acc_fma(sxx, pdx, dx);
        acc_fma(sxy, pdx, dy);
        acc_fma(syy, pdy, dy);
        if (kTrack) {
          acc_fma(gdd, wgt, p.gd[k]);
        } else {
          acc_fma(gdd, wgt, __builtin_fmaf(dz, p.gu2[k], p.gd[k]));
          gdd += pos1 == p.med1[k] ? p.gm[k] : 0.f;   // the median entry was blended
        }
        if (kParams) acc(gop, dlive * g);
        if (kParams || kColor) {
          acc_fma(gr, wgt, p.gc0[k]);
          acc_fma(gg, wgt, p.gc1[k]);
          acc_fma(gbl, wgt, p.gc2[k]);
        }
      }
      if (__ballot(any)) {
        float* dst = b.rec_grad + (int64_t)kGradStride * m;
        // slots 0-4: the sums u1, u2, sxx, sxy, syy; 5 opacity, 6 depth, 7-9 colour
        if (kParams) {
          const float vals[10] = {u1, u2, sxx, sxy, syy, gop, gdd, gr, gg, gbl};
          const float t = wave_sum_many<16>(vals);
          const int idx = reduced_value_index<16>(lane);
          if ((lane & 3) == 0 && idx < 10) unsafeAtomicAdd(dst + idx, t);
        } else if (kColor) {
          const float vals[9] = {u1, u2, sxx, sxy, syy, gdd, gr, gg, gbl};
          const float t = wave_sum_many<16>(vals);
          const int idx = reduced_value_index<16>(lane);
          if ((lane & 3) == 0 && idx < 9) unsafeAtomicAdd(dst + (idx < 5 ? idx : idx + 1), t);
        } else {
          const float vals[6] = {u1, u2, sxx, sxy, syy, gdd};
          const float t = wave_sum_many<8>(vals);
          const int idx = reduced_value_index<8>(lane);
          if ((lane & 7) == 0 && idx < 6) unsafeAtomicAdd(dst + (idx == 5 ? 6 : idx), t);
        }
      }
    }
  }
}

// kStats: keep the work counts of the statistics.
template <int kPPL, bool kTrack, bool kNu, bool kStats = true>
__global__ __launch_bounds__(kTilePixels / kPPL) void raster_forward_kernel(RasterBufs b) {
  __shared__ Stage<kTilePixels / kPPL / kWave> s;
  const int gtile = b.order ? (int)(b.order[blockIdx.x] & kOrderTileMask) : (int)blockIdx.x;
  const int v = view_of_tile(b.views, gtile);
  const ViewIO io = b.views.io[v];
  FwdPix<kPPL> f;
  const uint2 range = b.ranges[gtile];
  prioritise(range.y - range.x, kMapTilePrio[0], kMapTilePrio[1], kMapTilePrio[2]);
  forward_tile<kPPL, kTrack, kNu, true, kStats>(b, s, gtile, io, tile_origin(io.info, gtile), range, b.vals + range.x,
                                                f);
  float g[kPPL][4];
  forward_outputs<kPPL, kTrack, kNu, true, kStats>(b, v, io, f, g, true);
}

template <int kPPL, bool kParams, bool kTrack, bool kColor>
__global__ __launch_bounds__(kTilePixels / kPPL) void raster_backward_kernel(RasterBufs b) {
  constexpr int L = kTilePixels / kPPL;
  __shared__ Stage<kTilePixels / kPPL / kWave> s;
  __shared__ uint32_t s_max;
  const int gtile = b.order ? (int)(b.order[blockIdx.x] & kOrderTileMask) : (int)blockIdx.x;
  const int v = view_of_tile(b.views, gtile);
  const ViewIO io = b.views.io[v];
  const ViewInfo& cam = io.info;
  const int64_t hw = (int64_t)cam.width * cam.height;
  {
    const uint2 rg = b.ranges[gtile];
    prioritise(rg.y - rg.x, kMapTilePrio[0], kMapTilePrio[1], kMapTilePrio[2]);
  }
  BwdPix<kPPL> p;
  uint32_t lane_max = 0;
#pragma unroll
  for (int k = 0; k < kPPL; ++k) {
    const PixelCoord pc = pixel_of(cam, gtile, k * L + threadIdx.x);
    const int64_t pix = (int64_t)pc.py * cam.width + pc.px;
    p.fx[k] = (float)(pc.px - pc.ox);
    p.fy[k] = (float)(pc.py - pc.oy);
    p.T[k] = 1.f;
    p.walked[k] = 0;
    p.med1[k] = 0;
    p.gc0[k] = p.gc1[k] = p.gc2[k] = p.gd[k] = p.go[k] = p.gm[k] = p.gu[k] = p.dobs[k] = p.gu2[k] = 0.f;
    p.Bg[k] = 0.f;
    if (pc.inside) {
      const uint4 ps = b.pixel_state[cam.pixel_base + pix];
      p.T[k] = __uint_as_float(ps.x);
      p.walked[k] = (int)ps.y;
      p.med1[k] = (int)(ps.z + 1u);
      if (kTrack) {
        const float4 g4 = b.pixel_grad[cam.pixel_base + pix];
        p.gc0[k] = g4.x;
        p.gc1[k] = g4.y;
        p.gc2[k] = g4.z;
        p.gd[k] = g4.w;
      } else {
        if (io.g_color) {
          p.gc0[k] = io.g_color[pix];
          p.gc1[k] = io.g_color[hw + pix];
          p.gc2[k] = io.g_color[2 * hw + pix];
        }
        if (io.g_depth) p.gd[k] = io.g_depth[pix];
        if (io.g_opacity) p.go[k] = io.g_opacity[pix];
        if (io.g_median) p.gm[k] = io.g_median[pix];
        if (io.g_uncertainty) p.gu[k] = io.g_uncertainty[pix];
        p.gu2[k] = 2.f * p.gu[k];
        if (io.depth_obs) p.dobs[k] = io.depth_obs[pix];
      }
      lane_max = max(lane_max, (uint32_t)p.walked[k]);
    }
  }
  const int nmax = block_max(lane_max, &s_max);
  backward_tile<kPPL, kParams, kTrack, kColor>(b, s, b.ranges[gtile], tile_origin(cam, gtile), nmax, 0, p);
}

// The tile's bucket, at most L keys, sorted by the workgroup itself: a
// key's rank is the number of keys below it (keys are unique), so the ids
// come out in (depth, id) order as the segmented sort leaves them.  The
// bucket is read whole while its count is still in flight, so the ranking
// waits for one memory round trip, not two.  Leaves the ids in ids (LDS) and
// in the sorted list, writes the tile's range and resets its counter, as the
// segmented sort does.
template <int L>
__device__ __forceinline__ uint2 sort_own_bucket(const RasterBufs& b, int gtile, uint64_t* s_key, uint32_t* ids,
                                                 uint32_t* s_n) {
  const uint64_t base = (uint64_t)gtile * b.tile_cap;
  uint32_t* counter = b.tile_count + (size_t)gtile * kTileCounterStride;
  const uint64_t key = threadIdx.x < b.tile_cap ? b.bucket_keys[base + threadIdx.x] : 0ull;
  if (threadIdx.x == 0) {
    const uint32_t n = min(*counter, b.tile_cap);   // beyond the bucket only after an overflow, which is reported
    if (!b.keep_counts) *counter = 0u;
    *s_n = n;
    b.ranges[gtile] = make_uint2((uint32_t)base, (uint32_t)(base + n));
    if (gtile == 0) b.counters[kCntRenderPeak] = 0u;
  }
  s_key[threadIdx.x] = key;
  __syncthreads();
  const uint32_t n = *s_n;
  if (threadIdx.x < n) {
    uint32_t rank = 0;
    for (uint32_t i = 0; i < n; ++i) rank += s_key[i] < key ? 1u : 0u;
    ids[rank] = (uint32_t)key;
    b.vals[base + rank] = (uint32_t)key;
  }
  __syncthreads();
  return make_uint2((uint32_t)base, (uint32_t)(base + n));
}

// Tracking iteration of one tile: forward, tracking-loss gradients in
// registers, pose backward (kColor: with the colour gradients that the pose
// gradient of a view-dependent colour needs; kFull: also the per-pixel state
// and work counts that the statistics read).
template <int kPPL, bool kColor, bool kFull>
__global__ __launch_bounds__(kTilePixels / kPPL) void raster_track_kernel(RasterBufs b) {
  constexpr int L = kTilePixels / kPPL;
  __shared__ Stage<kTilePixels / kPPL / kWave> s;
  __shared__ uint32_t s_max;
  __shared__ uint32_t s_ids[L];
  // The bucket's keys are ranked before the first batch is staged, so they
  // share the stage's storage (keeping the workgroup's LDS at 25.6 KB, six
  // workgroups per CU at one pixel per lane).
  static_assert(sizeof(s.A) >= sizeof(uint64_t) * L, "sort keys fit the stage");
  uint64_t* s_key = reinterpret_cast<uint64_t*>(&s.A[0][0]);
  const uint32_t ord = b.order ? b.order[blockIdx.x] : (uint32_t)blockIdx.x;
  const int gtile = (int)(ord & kOrderTileMask);
  // one pixel per lane: wave w takes quadrant (w + rot) & 3, a rotation the
  // order chose per workgroup so that the SIMDs of a CU get even work
  const int rot = kPPL == 1 ? (int)(ord >> 30) : 0;
  const int v = view_of_tile(b.views, gtile);
  const ViewIO io = b.views.io[v];
  const float2 org = tile_origin(io.info, gtile);
  const uint2 range = b.sort_here ? sort_own_bucket<L>(b, gtile, s_key, s_ids, &s_max) : b.ranges[gtile];
  prioritise(range.y - range.x, kTrackTilePrio[0], kTrackTilePrio[1], kTrackTilePrio[2]);
  BwdPix<kPPL> p;
  uint32_t lane_max = 0;
  {
    FwdPix<kPPL> f;
    forward_tile<kPPL, true, false, kFull>(b, s, gtile, io, org, range, b.sort_here ? s_ids : b.vals + range.x, f,
                                           rot);
    float g[kPPL][4];
    forward_outputs<kPPL, true, false, kFull>(b, v, io, f, g, false);
    // each quadrant's work for the next step's order (word 1 + quadrant of
    // the tile's counter line)
    if constexpr (kPPL == 1) {
      if ((threadIdx.x & (kWave - 1)) == 0)
        b.tile_count[(size_t)gtile * kTileCounterStride + 1 + ((threadIdx.x / kWave + rot) & 3)] = f.wave_len;
    } else {
      constexpr int W = kTilePixels / kPPL / kWave;
      if ((threadIdx.x & (kWave - 1)) == 0)
        b.tile_count[(size_t)gtile * kTileCounterStride + 1 + threadIdx.x / kWave] = f.wave_len;
      if (threadIdx.x < 4 - W) b.tile_count[(size_t)gtile * kTileCounterStride + 1 + W + threadIdx.x] = 0u;
    }
#pragma unroll
    for (int k = 0; k < kPPL; ++k) {
      p.fx[k] = f.fx[k];
      p.fy[k] = f.fy[k];
      p.T[k] = f.T[k];
      p.walked[k] = f.inside[k] ? (int)f.last[k] : 0;
      p.med1[k] = 0;
      p.gc0[k] = g[k][0];
      p.gc1[k] = g[k][1];
      p.gc2[k] = g[k][2];
      p.gd[k] = g[k][3];
      p.go[k] = p.gm[k] = p.gu[k] = p.dobs[k] = p.gu2[k] = 0.f;
      p.Bg[k] = 0.f;
      lane_max = max(lane_max, (uint32_t)p.walked[k]);
    }
  }
  const int nmax = block_max(lane_max, &s_max);
  const int len = (int)(range.y - range.x);
  backward_tile<kPPL, false, true, kColor>(b, s, range, org, nmax, len <= kBatch ? len : 0, p, rot);
}

template <int kPPL>
void launch_fwd(const RasterBufs& b, bool track, hipStream_t s) {
  const dim3 grid(b.total_tiles), block(kTilePixels / kPPL);
  if (track) hipLaunchKernelGGL((raster_forward_kernel<kPPL, true, false>), grid, block, 0, s, b);
  else if (b.nu) hipLaunchKernelGGL((raster_forward_kernel<kPPL, false, true>), grid, block, 0, s, b);
  else if (b.count_work) hipLaunchKernelGGL((raster_forward_kernel<kPPL, false, false>), grid, block, 0, s, b);
  else hipLaunchKernelGGL((raster_forward_kernel<kPPL, false, false, false>), grid, block, 0, s, b);
}

template <int kPPL>
void launch_bwd(const RasterBufs& b, bool params, bool track, hipStream_t s) {
  const dim3 grid(b.total_tiles), block(kTilePixels / kPPL);
  if (track && b.color_grads)
    hipLaunchKernelGGL((raster_backward_kernel<kPPL, false, true, true>), grid, block, 0, s, b);
  else if (track) hipLaunchKernelGGL((raster_backward_kernel<kPPL, false, true, false>), grid, block, 0, s, b);
  else if (params || b.color_grads)
    hipLaunchKernelGGL((raster_backward_kernel<kPPL, true, false, false>), grid, block, 0, s, b);
  else hipLaunchKernelGGL((raster_backward_kernel<kPPL, false, false, false>), grid, block, 0, s, b);
}

template <int kPPL>
void launch_track(const RasterBufs& b, hipStream_t s) {
  const dim3 grid(b.total_tiles), block(kTilePixels / kPPL);
  if (b.color_grads && b.count_work) hipLaunchKernelGGL((raster_track_kernel<kPPL, true, true>), grid, block, 0, s, b);
  else if (b.color_grads) hipLaunchKernelGGL((raster_track_kernel<kPPL, true, false>), grid, block, 0, s, b);
  else if (b.count_work) hipLaunchKernelGGL((raster_track_kernel<kPPL, false, true>), grid, block, 0, s, b);
  else hipLaunchKernelGGL((raster_track_kernel<kPPL, false, false>), grid, block, 0, s, b);
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

void launch_raster_track(const RasterBufs& b, int ppl, hipStream_t s) {
  if (b.total_tiles <= 0) return;
  if (ppl == 4) launch_track<4>(b, s);
  else if (ppl == 2) launch_track<2>(b, s);
  else launch_track<1>(b, s);
}

}  // namespace cgsr
