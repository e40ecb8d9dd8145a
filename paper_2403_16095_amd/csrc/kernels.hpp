// Host-side launchers of the cgsr kernels (one translation unit per stage).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace cgsr {

// Counters kept in device memory, one block of them per state.
enum Counter : int {
  kCntOverflow = 1,     // 1 if a render since the last check had a tile over its bucket
  kCntPeak = 2,         // most pairs an overflowing tile needed since the last check
  kCntStaleTable = 3,   // 1 if a launch since the last check read a view table other than its own
  kCntRenderPeak = 4,   // most pairs an overflowing tile needs in the render in flight (reset by the sort)
};
constexpr int kCounterWords = 8;
// An entry of a tile order: the tile in the low 30 bits; the top two bits
// turn the quadrants of a fused tracking workgroup at one pixel per lane.
constexpr uint32_t kOrderTileMask = 0x3FFFFFFFu;

// A launch replayed from a captured graph reads whatever view table the state
// holds when it runs; one workgroup compares the table's hash with the one
// the launch was set up with and raises kCntStaleTable if they differ.
__device__ __forceinline__ void check_table(const ViewTable& vt, uint32_t* counters) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && counters &&
      reinterpret_cast<const uint32_t*>(vt.io + vt.n)[0] != vt.hash)
    atomicOr(counters + kCntStaleTable, 1u);
}

// Every workgroup takes the per-tile counters by atomics; each counter sits on
// a 128-byte line of its own so that atomics on neighbouring tiles do not queue
// behind one another.
constexpr int kTileCounterStride = 32;

struct ProjectBufs {
  float4* rec;              // [M][3]
  uint32_t* tiles;          // [M] tiles touched (0 = culled)
  uint2* rect;              // [M] binning rect in 8-pixel cells: x = cx0 | cx1 << 16, y = cy0 | cy1 << 16
  uint32_t* tile_count;     // [T * kTileCounterStride] pairs per tile (zero on entry; reset by the segment sort)
  uint32_t* counters;       // Counter enum above
  int32_t total_tiles;
  uint64_t* keys;           // [T][tile_cap] each tile's bucket of pair keys: depth bits << 32 | record id
  uint32_t tile_cap;        // pairs a bucket holds (later ones are dropped)
  uint32_t flag_cap;        // a tile needing more raises the overflow flag
};

struct GaussianPtrs {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* rgb;
  int64_t n;
  const float* sh;     // null, or [n][(sh_degree + 1)^2][3]: view-dependent colour
  int32_t sh_degree;
};

struct GradPtrs {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* rgb;
  float* sh;
};

// Projection (one lane per (view, Gaussian)) with the emission of every
// (tile, Gaussian) pair into its tile's bucket.
void launch_project(const GaussianPtrs& g, const float* poses, const ViewTable& vt, const ProjectBufs& b,
                    hipStream_t s);
// Chain rule from the per-record projected gradients to the parameters and
// the poses.  pose_acc: device double[views][6] scratch, zero on entry and
// left zero on exit; dposes (+=) may be null.
// Optional Adam step applied to the summed pose gradient right away.
struct PoseStep {
  float* poses;   // [views][12], updated in place
  float* adam;    // [views][16]
  AdamParams params;
};
// dens_grad / dens_count (may be null): per Gaussian, += |dL/dmu| of every
// record that reaches the image and += 1 (the densification statistic).
void launch_project_backward(const GaussianPtrs& g, const float* poses, const ViewTable& vt, float* rec_grad,
                             const uint32_t* tiles, const GradPtrs& dg, bool param_grads, double* pose_acc,
                             float* dposes, const PoseStep* step, float* dens_grad, uint32_t* dens_count,
                             uint32_t* counters, hipStream_t s);

// Gaussian management (management.hip).  Writable parameter arrays of a set
// (colour in rgb, or sh with K coefficients per channel).
struct GaussArrays {
  float *means, *log_scales, *quats, *opacity_logits, *rgb, *sh;
};
constexpr int kMaxExtraArrays = 12;
// Additional per-Gaussian float arrays compacted along with a set.
struct ExtraArrays {
  int n;
  const float* src[kMaxExtraArrays];
  float* dst[kMaxExtraArrays];
  int width[kMaxExtraArrays];
};
constexpr int kRankKinds = 3;
// Each runs a ranked selection and synchronises the stream to return the
// totals: spawned pixels; kept Gaussians; (not split, cloned, split).
hipError_t run_spawn(const GaussArrays& dst, int64_t n, int64_t capacity, const ViewInfo& cam, const float* pose,
                     const float* color, const float* depth, const float* opacity, float psi, int stride,
                     float init_logit, int K, uint32_t* total, hipStream_t s);
hipError_t run_compact(int64_t n, const uint8_t* keep, const GaussArrays& src, const GaussArrays& dst, int colour_w,
                       const ExtraArrays& extra, uint32_t* total, hipStream_t s);
// The same without device allocation: its counters live in a fixed
// per-GPU array of the library; n <= kNoAllocMaxN.  Overlapping calls on one
// GPU share that array.
constexpr int64_t kNoAllocMaxN = CGSR_COMPACT_NOALLOC_MAX_N;
hipError_t run_compact_noalloc(int64_t n, const uint8_t* keep, const GaussArrays& src, const GaussArrays& dst,
                               int colour_w, const ExtraArrays& extra, uint32_t* total, hipStream_t s);
hipError_t run_densify(int64_t n, const float* grad_accum, const uint32_t* count, float threshold, float dense_scale,
                       const float* normals, const GaussArrays& src, const GaussArrays& dst, int colour_w,
                       int64_t capacity, uint32_t* totals, hipStream_t s);

// Segmented sort: one workgroup per tile orders its bucket of keys and
// writes the record ids in depth order plus the tile's range.
struct SegSortBufs {
  uint64_t* keys[2];        // [T][cap] the buckets, and scratch for long segments
  uint32_t* sorted_vals;    // [T][cap] record ids in (depth, id) order
  uint32_t* tile_count;     // [T * kTileCounterStride] read, then reset to zero here
  uint2* ranges;            // [T]
  uint32_t* counters;       // resets kCntRenderPeak
  uint32_t cap;
};
void launch_segment_sort(const SegSortBufs& b, int32_t total_tiles, hipStream_t s);
// Fill n uint32 with zero (a kernel, so it can sit in a captured graph).
void launch_clear_u32(uint32_t* p, int64_t n, hipStream_t s);
// Tiles by descending list length, in order[tiles]: lengths from the ranges
// after the sort, or with ranges null from the pair counters (stride
// kTileCounterStride) before a blend that sorts its own buckets.
void launch_tile_order(const uint2* ranges, const uint32_t* counts, int32_t tiles, uint32_t* order, hipStream_t s);
// The order a fused tracking launch whose tiles are all resident at once
// keeps across steps (1 .. kKeptOrderMaxTiles tiles): lengths are the sums of
// quads[0..3] of each tile's line (stride kTileCounterStride: the four
// quadrants' work the previous step measured), every other run of 256
// positions is reversed, the last, short run is placed by the work the full
// runs gave each position, and each entry gets a quadrant rotation in bits
// 30..31 (kOrderTileMask keeps the tile).
constexpr int32_t kKeptOrderMaxTiles = 2048;
void launch_tile_order_kept(const uint32_t* quads, int32_t tiles, uint32_t* order, hipStream_t s);
// Pair counter of each tile = the length of its range (undoes the reset of
// a tracking kernel that sorted its own buckets).
void launch_restore_counts(uint32_t* tile_count, const uint2* ranges, int32_t tiles, hipStream_t s);

struct RasterBufs {
  const float4* rec;
  uint32_t* vals;           // sorted record ids
  uint2* ranges;
  uint4* pixel_state;       // [total pixels]: final T bits, entries up to the last blended one,
                            // median position or -1, alpha evaluations
  uint2* pixel_count;       // [total pixels]: Gaussians blended, entries of the wave's list up to the
                            // last blended one
  const uint2* rect;        // [M] binning rect in 8-pixel cells (see ProjectBufs)
  float4* pixel_grad;       // [total pixels]: tracking-loss gradient (colour, depth)
  float* rec_grad;          // [M][kGradStride]
  ViewTable views;          // device table of the pass (forward or backward pointers)
  int32_t total_tiles;
  float lambda_color, lambda_depth;  // tracking loss weights (Eq. 19)
  float* loss;              // [views] tracking loss (+=) or null
  // Eq. 13 accumulation (mapping renders): per Gaussian, sum of w (D - d)^2
  // over its dominated pixels and their number (+=); nu selects the kernel
  // variant that tracks each pixel's largest-weight Gaussian.
  float* nu_sum;
  uint32_t* nu_count;
  bool nu;
  // The backward also reduces the colour gradients when the pose gradient
  // needs them (view-dependent colour) even without parameter gradients.
  bool color_grads;
  // The fused tracking kernel keeps the per-pixel state and work counts; the
  // forward blend of a render (no tracking, no nu) keeps the work counts.
  bool count_work;
  // The fused tracking kernel sorts its tile's bucket itself (no separate
  // segmented sort): every bucket holds at most one key per thread.  It then
  // reads the buckets and pair counters and writes vals and ranges as that
  // sort would.
  bool sort_here;
  const uint64_t* bucket_keys;   // [T][tile_cap]
  uint32_t* tile_count;          // [T * kTileCounterStride], reset to zero here; the fused
                                 // tracking kernel leaves each quadrant's work in words 1..4
  uint32_t* counters;            // kCntRenderPeak reset here
  uint32_t tile_cap;
  // Timing re-runs of a tracking step's kernel leave the pair counters as
  // they are, so every re-run sorts and walks the same buckets.
  bool keep_counts;
  // Tile of each workgroup, longest list first (launch_tile_order), or null
  // for workgroup b on tile b; entries are masked with kOrderTileMask, and
  // the fused tracking kernel at one pixel per lane turns its quadrants by
  // the top two bits.
  const uint32_t* order;
};
// ppl: pixels per lane, 1, 2 or 4 (256 / ppl lanes per 16x16 tile).
void launch_raster_forward(const RasterBufs& b, bool track, int ppl, hipStream_t s);
// One view of the mapping objective (Eq. 18).  Inputs: rendered maps and
// targets; outputs (null = not wanted): gradient images, overwritten, and the
// view's loss (+=).  median != null enables the alignment term (it then
// needs depth), dcolor the colour L1 and SSIM terms, ddepth the depth L1.
struct ObjectiveView {
  int width, height;
  const float *color, *depth, *median, *unc, *tcolor, *tdepth;
  float *dcolor, *ddepth, *dmedian, *dunc, *loss;
};
struct ObjectiveWeights {
  float color, ssim, geo, align, iso, var;
};
// ssim_part: scratch of 9 floats per pixel of the view.
void launch_objective_view(const ObjectiveView& o, const ObjectiveWeights& w, float* ssim_part, hipStream_t s);
// Eq. 17 over each view's visible Gaussians (tiles[v * n + i] > 0): counts
// (scratch, n_views words), dlog_scales (+=, may be null), loss[v] (+=).
void launch_iso(int64_t n, int n_views, const uint32_t* tiles, uint32_t* counts, const float* log_scales, float w_iso,
                float eps, float* dlog_scales, float* loss, hipStream_t s);
// Adam over the Gaussian parameter groups (element-wise; moments
// [2][(11 + colour_width) n] in group order), bias-corrected with the device
// step counter, which a second one-lane launch then increments.  Gradients
// are zeroed after use.  The colour group is rgb (width 3) or the SH
// coefficients (width 3 K), whose degree >= 1 entries take lr_sh_rest.
struct GaussianAdam {
  float* param[5];       // means, log_scales, quats, opacity_logits, colour
  float* grad[5];
  float lr[5];
  float beta1, beta2, eps;
  int32_t colour_width;  // 3 (rgb) or 3 (sh_degree + 1)^2
  float lr_sh_rest;
};
void launch_gaussian_adam(int64_t n, const GaussianAdam& a, float* moments, uint32_t* step, hipStream_t s);
// nu_i = nu_sum_i / nu_count_i (0 without dominated pixels); Gaussians with
// nu_i > tau get opacity_logit = min(opacity_logit, low_logit).
void launch_nu_prune(int64_t n, const float* nu_sum, const uint32_t* nu_count, float tau, float low_logit,
                     float* opacity_logits, float* nu, uint32_t* n_pruned, hipStream_t s);
void launch_raster_backward(const RasterBufs& b, bool param_grads, bool track, int ppl, hipStream_t s);
// Forward, tracking-loss gradients and pose-only blend backward of each tile
// in one launch (rec_grad +=); writes pixel_state / pixel_count for the stats.
void launch_raster_track(const RasterBufs& b, int ppl, hipStream_t s);

void launch_tracking_loss(int w, int h, const float* color, const float* depth, const float* tcolor,
                          const float* tdepth, float lc, float ld, float* dcolor, float* ddepth, float* loss,
                          hipStream_t s);
void launch_mapping_loss(int w, int h, const float* color, const float* depth, const float* unc,
                         const float* tcolor, const float* tdepth, float* dcolor, float* ddepth, float* dunc,
                         float* loss, hipStream_t s);
void launch_pose_adam(int n_views, float* poses, float* dposes, float* adam, const AdamParams& ap, hipStream_t s);

// Statistics: visible records, alpha evaluations, blended pairs, walked
// entries, (tile, record) pairs and the fullest tile's pairs, added into out6.
void launch_stats(const uint32_t* tiles, int64_t m, const uint4* pixel_state, const uint2* pixel_count,
                  int64_t pixels, const uint2* ranges, int64_t n_tiles, unsigned long long* out6, hipStream_t s);

}  // namespace cgsr
