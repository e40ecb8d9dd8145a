// Host runtime behind the C ABI of include/cgsr.h: workspace ownership,
// argument checks, and the launch sequence of a render and its backward.
//
// Render: project (counts pairs per tile) -> emit (keys into tile segments)
// -> segment sort (depth order per tile, tile ranges) -> blend.
// Backward: blend backward -> projection backward (parameters, pose).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "kernels.hpp"

using namespace cgsr;

namespace {

thread_local std::string g_last_error;

cgsr_status fail(cgsr_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(CGSR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

template <typename T>
cgsr_status dev_alloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)count);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(CGSR_ERR_OOM, "hipMalloc of %lld bytes failed: %s", (long long)(sizeof(T) * count),
                hipGetErrorString(e));
  }
  return CGSR_OK;
}

template <typename T>
void dev_free(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

}  // namespace

// Fewest tiles for which a fused tracking step orders its tiles longest
// first from its own pair counters, in a launch of its own: about the
// workgroups the chip holds at once (256 CUs x 6); below it the step keeps
// an order taken from the previous step's lengths (render_impl).  No launch
// orders more than kOrderMaxTiles: the one-workgroup order kernel then costs
// about what it saves (32 frames of mixed resolution, 54k tiles: 0.5 %
// slower with the order; eight 1200x680 views, 25.8k tiles: 1.5 % faster).
constexpr int32_t kOrderMinTiles = 1536;
static_assert(kOrderMinTiles <= kKeptOrderMaxTiles, "every step below kOrderMinTiles tiles can keep its order");
constexpr int kTunePasses = 2;   // timing passes over an autotuner's candidates
constexpr int32_t kOrderMaxTiles = 32768;

struct cgsr_state {
  int device = 0;
  cgsr_settings settings{};
  // capacities
  int64_t cap_records = 0, cap_pixels = 0, cap_tiles = 0;
  int64_t cap_tile_pairs = 0;   // pairs one tile's bucket holds
  int64_t bucket_tiles = 0;     // tiles the bucket buffers are sized for
  // per (view, Gaussian) record
  float4* rec = nullptr;
  uint32_t* tiles = nullptr;
  uint2* rect = nullptr;
  float* rec_grad = nullptr;
  // per tile
  uint32_t* tile_count = nullptr;
  uint2* ranges = nullptr;
  uint32_t* tile_order = nullptr;   // tiles by descending list length, for the blends
  bool order_ok = false;            // tile_order holds the last render's order
  // tile_order holds the order a fused tracking step of track_order_tiles
  // tiles took from the previous step's lengths, and nothing has overwritten it
  bool track_order_ok = false;
  int32_t track_order_tiles = 0;
  unsigned long long order_capture = 0;   // the graph capture that last computed it
  bool tiles_dirty = false;   // a render stopped between projection and sort
  // per-tile buckets of pairs, [bucket_tiles][cap_tile_pairs]
  uint64_t* keys[2] = {nullptr, nullptr};
  uint32_t* sorted_vals = nullptr;
  // per pixel
  uint4* pixel_state = nullptr;
  uint2* pixel_count = nullptr;
  float4* pixel_grad = nullptr;
  // small buffers
  float* tune_dposes = nullptr;   // [64][6] scratch pose gradients of the autotuner
  float* obj_part = nullptr;      // SSIM moment derivatives, 9 floats per pixel of one view
  int64_t cap_obj_pixels = 0;
  uint32_t* obj_counts = nullptr; // visible Gaussians per view (isotropy term)
  uint32_t* counters = nullptr;
  float* dens_grad = nullptr;      // densification statistic (cgsr_set_densify_stats)
  uint32_t* dens_count = nullptr;
  double* pose_acc = nullptr;
  unsigned long long* stats_dev = nullptr;
  uint32_t* counters_pinned = nullptr;
  // Per-view tables of the forward (slot 0) and the backward (slot 1), each
  // re-uploaded only when its contents change, so a steady loop of render +
  // backward uploads nothing.
  struct IoTable {
    ViewIO* dev = nullptr;
    ViewIO* pinned = nullptr;
    hipEvent_t event = nullptr;
    bool event_pending = false;
    ViewIO cached[CGSR_MAX_VIEWS];
    int cached_n = -1;
    uint32_t hash = 0;   // of the table last uploaded, which dev[n] holds in its first word
  } io[2];
  // stage timing: ev_fwd[k] starts forward stage k, ev_fwd[k + 1] ends it
  hipEvent_t ev_fwd[CGSR_STAGE_BLEND_FWD + 2] = {};
  hipEvent_t ev_bwd[3] = {};
  bool fwd_timed = false, bwd_timed = false;
  // last render
  bool have_forward = false;
  bool tracked = false;   // the last forward was a tracking step
  bool counted = false;   // the last forward kept the per-pixel work counts
  int32_t n_views = 0;
  GaussianPtrs g{};
  const float* poses = nullptr;
  int64_t total_pixels = 0;
  int32_t total_tiles = 0;
  int64_t records = 0;
  ViewIO io_fwd[CGSR_MAX_VIEWS];
  // autotuner picks per workload shape (see tune_key)
  struct TunePick {
    uint64_t key;
    int32_t fwd, bwd;
  } tune_cache[16];
  int tune_n = 0;
  // the fused blend launch of the last tracking step, for timing re-runs;
  // valid while no other call has changed the state's buffers or tables
  RasterBufs track_rb{};
  int track_ppl = 1;
  bool track_rb_ok = false;
};

namespace {

cgsr_status set_device(cgsr_state* st) {
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != st->device) HIP_TRY(hipSetDevice(st->device));
  return CGSR_OK;
}

// Buckets for cap_tiles tiles of at least tile_pairs pairs each.  Sizes are
// kept in 32 bits on the device (tile ranges), so tiles x pairs < 2^32.
cgsr_status grow_buckets(cgsr_state* st, int64_t tile_pairs) {
  st->track_rb_ok = false;
  const int64_t cap = std::max<int64_t>(std::max<int64_t>(tile_pairs, st->cap_tile_pairs), 64);
  if (cap == st->cap_tile_pairs && st->bucket_tiles >= st->cap_tiles) return CGSR_OK;
  const int64_t tiles = std::max<int64_t>(st->cap_tiles, 1);
  if (tiles * cap >= (1ll << 32))
    return fail(CGSR_ERR_CAPACITY, "%lld tiles of %lld pairs exceed 2^32 bucket slots", (long long)tiles,
                (long long)cap);
  HIP_TRY(hipDeviceSynchronize());
  dev_free(st->keys[0]);
  dev_free(st->keys[1]);
  dev_free(st->sorted_vals);
  st->cap_tile_pairs = 0;
  st->bucket_tiles = 0;
  cgsr_status s;
  if ((s = dev_alloc(&st->keys[0], tiles * cap))) return s;
  if ((s = dev_alloc(&st->keys[1], tiles * cap))) return s;
  if ((s = dev_alloc(&st->sorted_vals, tiles * cap))) return s;
  st->cap_tile_pairs = cap;
  st->bucket_tiles = tiles;
  return CGSR_OK;
}

cgsr_status reserve(cgsr_state* st, int64_t records, int64_t pixels, int64_t tiles, int64_t tile_pairs) {
  st->track_rb_ok = false;
  if (records > st->cap_records || pixels > st->cap_pixels || tiles > st->cap_tiles)
    HIP_TRY(hipDeviceSynchronize());
  cgsr_status s;
  if (records > st->cap_records) {
    dev_free(st->rec);
    dev_free(st->tiles);
    dev_free(st->rect);
    dev_free(st->rec_grad);
    st->cap_records = 0;
    if ((s = dev_alloc(&st->rec, kRecF4 * records))) return s;
    if ((s = dev_alloc(&st->tiles, records))) return s;
    if ((s = dev_alloc(&st->rect, records))) return s;
    if ((s = dev_alloc(&st->rec_grad, kGradStride * records))) return s;
    HIP_TRY(hipMemset(st->rec_grad, 0, sizeof(float) * kGradStride * (size_t)records));
    st->cap_records = records;
  }
  if (pixels > st->cap_pixels) {
    dev_free(st->pixel_state);
    dev_free(st->pixel_count);
    dev_free(st->pixel_grad);
    st->cap_pixels = 0;
    if ((s = dev_alloc(&st->pixel_state, pixels))) return s;
    if ((s = dev_alloc(&st->pixel_count, pixels))) return s;
    if ((s = dev_alloc(&st->pixel_grad, pixels))) return s;
    st->cap_pixels = pixels;
  }
  if (tiles > st->cap_tiles) {
    dev_free(st->ranges);
    dev_free(st->tile_count);
    dev_free(st->tile_order);
    st->cap_tiles = 0;
    st->order_ok = false;
    st->track_order_ok = false;
    if ((s = dev_alloc(&st->ranges, tiles))) return s;
    if ((s = dev_alloc(&st->tile_order, tiles))) return s;
    if ((s = dev_alloc(&st->tile_count, tiles * kTileCounterStride))) return s;
    HIP_TRY(hipMemset(st->ranges, 0, sizeof(uint2) * (size_t)tiles));
    HIP_TRY(hipMemset(st->tile_count, 0, sizeof(uint32_t) * kTileCounterStride * (size_t)tiles));
    st->tiles_dirty = false;
    st->cap_tiles = tiles;
  }
  return grow_buckets(st, tile_pairs);
}

bool bad_camera(const cgsr_camera& c) {
  // the binning rectangle is kept in 8-pixel cells of 16 bits
  return c.width < 1 || c.height < 1 || c.width > 65535 * 8 || c.height > 65535 * 8 || !(c.fx > 0.f) ||
         !(c.fy > 0.f) || !(c.cx == c.cx) || !(c.cy == c.cy);
}

// Uploads a per-view table if it differs from its last upload.  Under graph
// capture the tables must already be current: an upload there would be a
// captured host-to-device copy of staging memory the next call overwrites.
cgsr_status upload_io(cgsr_state* st, int slot, const ViewIO* io, int n, hipStream_t stream) {
  auto& t = st->io[slot];
  if (n == t.cached_n && std::memcmp(io, t.cached, sizeof(ViewIO) * n) == 0) return CGSR_OK;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &cap));
  if (cap != hipStreamCaptureStatusNone)
    return fail(CGSR_ERR_STATE,
                "cameras or image pointers changed during graph capture; run the same call once "
                "before capturing it");
  if (t.event_pending) {
    HIP_TRY(hipEventSynchronize(t.event));
    t.event_pending = false;
  }
  // FNV-1a of the table, stored after it: launches compare it with their own
  uint32_t h = 2166136261u;
  const unsigned char* bytes = reinterpret_cast<const unsigned char*>(io);
  for (size_t k = 0; k < sizeof(ViewIO) * (size_t)n; ++k) h = (h ^ bytes[k]) * 16777619u;
  std::memcpy(t.pinned, io, sizeof(ViewIO) * n);
  std::memset(&t.pinned[n], 0, sizeof(ViewIO));
  std::memcpy(&t.pinned[n], &h, sizeof(h));
  HIP_TRY(hipMemcpyAsync(t.dev, t.pinned, sizeof(ViewIO) * (n + 1), hipMemcpyHostToDevice, stream));
  t.hash = h;
  HIP_TRY(hipEventRecord(t.event, stream));
  t.event_pending = true;
  std::memcpy(t.cached, io, sizeof(ViewIO) * n);
  t.cached_n = n;
  return CGSR_OK;
}

ProjectBufs project_bufs(cgsr_state* st) {
  ProjectBufs b;
  b.rec = st->rec;
  b.tiles = st->tiles;
  b.rect = st->rect;
  b.tile_count = st->tile_count;
  b.counters = st->counters;
  b.total_tiles = st->total_tiles;
  b.keys = st->keys[0];
  b.tile_cap = (uint32_t)st->cap_tile_pairs;
  b.flag_cap = b.tile_cap;
  return b;
}

RasterBufs raster_bufs(cgsr_state* st, int slot) {
  RasterBufs rb;
  rb.rec = st->rec;
  rb.vals = st->sorted_vals;
  rb.ranges = st->ranges;
  rb.pixel_state = st->pixel_state;
  rb.pixel_count = st->pixel_count;
  rb.rect = st->rect;
  rb.pixel_grad = st->pixel_grad;
  rb.rec_grad = st->rec_grad;
  rb.lambda_color = rb.lambda_depth = 0.f;
  rb.loss = nullptr;
  rb.nu_sum = nullptr;
  rb.nu_count = nullptr;
  rb.nu = false;
  rb.color_grads = st->g.sh != nullptr;
  rb.count_work = st->settings.count_work != 0;
  rb.sort_here = false;
  rb.bucket_keys = st->keys[0];
  rb.tile_count = st->tile_count;
  rb.counters = st->counters;
  rb.tile_cap = (uint32_t)st->cap_tile_pairs;
  rb.keep_counts = false;
  rb.order = st->order_ok ? st->tile_order : nullptr;
  rb.views = ViewTable{st->io[slot].dev, st->n_views, (int32_t)st->g.n, st->io[slot].hash};
  rb.total_tiles = st->total_tiles;
  return rb;
}

}  // namespace

extern "C" {

void cgsr_default_settings(cgsr_settings* s) {
  if (!s) return;
  s->sync_capacity = 1;
  s->timing = 0;
  s->fwd_pixels_per_lane = 1;
  s->bwd_pixels_per_lane = 1;
  s->count_work = 1;
}

cgsr_status cgsr_state_create(const cgsr_settings* s, cgsr_state** out) {
  if (!out) return fail(CGSR_ERR_INVALID_ARG, "cgsr_state_create: out is NULL");
  *out = nullptr;
  cgsr_state* st = new (std::nothrow) cgsr_state();
  if (!st) return fail(CGSR_ERR_OOM, "cgsr_state_create: host allocation failed");
  if (s) st->settings = *s;
  else cgsr_default_settings(&st->settings);
  auto ppl_ok = [](int32_t p) { return p == 1 || p == 2 || p == 4; };
  if (st->settings.sync_capacity < 0 || st->settings.sync_capacity > 1 || st->settings.timing < 0 ||
      st->settings.timing > 1 || !ppl_ok(st->settings.fwd_pixels_per_lane) ||
      !ppl_ok(st->settings.bwd_pixels_per_lane) || st->settings.count_work < 0 || st->settings.count_work > 1) {
    delete st;
    return fail(CGSR_ERR_INVALID_ARG,
                "settings: sync_capacity, timing and count_work must be 0 or 1, pixels per lane 1, 2 or 4");
  }
  cgsr_status r = CGSR_OK;
  hipError_t e = hipGetDevice(&st->device);
  if (e != hipSuccess) r = fail(CGSR_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (!r) r = dev_alloc(&st->counters, kCounterWords);
  if (!r && hipMemset(st->counters, 0, sizeof(uint32_t) * kCounterWords) != hipSuccess)
    r = fail(CGSR_ERR_HIP, "hipMemset of counters failed");
  if (!r) r = dev_alloc(&st->pose_acc, 6 * CGSR_MAX_VIEWS);
  if (!r && hipMemset(st->pose_acc, 0, sizeof(double) * 6 * CGSR_MAX_VIEWS) != hipSuccess)
    r = fail(CGSR_ERR_HIP, "hipMemset of pose accumulators failed");
  for (int k = 0; k < 2 && !r; ++k) {
    r = dev_alloc(&st->io[k].dev, CGSR_MAX_VIEWS + 1);
    if (!r && hipMemset(st->io[k].dev, 0, sizeof(ViewIO) * (CGSR_MAX_VIEWS + 1)) != hipSuccess)
      r = fail(CGSR_ERR_HIP, "hipMemset of a view table failed");
    if (!r && hipHostMalloc((void**)&st->io[k].pinned, sizeof(ViewIO) * (CGSR_MAX_VIEWS + 1),
                            hipHostMallocDefault) != hipSuccess)
      r = fail(CGSR_ERR_OOM, "pinned allocation failed");
    if (!r && hipEventCreateWithFlags(&st->io[k].event, hipEventDisableTiming) != hipSuccess)
      r = fail(CGSR_ERR_HIP, "hipEventCreate failed");
  }
  if (!r) r = dev_alloc(&st->stats_dev, 6);
  if (!r) r = dev_alloc(&st->tune_dposes, 6 * CGSR_MAX_VIEWS);
  if (!r) r = dev_alloc(&st->obj_counts, CGSR_MAX_VIEWS);
  for (auto& ev : st->ev_fwd)
    if (!r && hipEventCreate(&ev) != hipSuccess) r = fail(CGSR_ERR_HIP, "hipEventCreate failed");
  for (auto& ev : st->ev_bwd)
    if (!r && hipEventCreate(&ev) != hipSuccess) r = fail(CGSR_ERR_HIP, "hipEventCreate failed");
  if (!r && hipHostMalloc((void**)&st->counters_pinned, sizeof(uint32_t) * kCounterWords,
                                 hipHostMallocDefault) != hipSuccess)
    r = fail(CGSR_ERR_OOM, "pinned allocation failed");
  if (r) {
    cgsr_state_destroy(st);
    return r;
  }
  *out = st;
  return CGSR_OK;
}

cgsr_status cgsr_state_destroy(cgsr_state* st) {
  if (!st) return CGSR_OK;
  int cur = -1;
  if (hipGetDevice(&cur) == hipSuccess && cur != st->device) (void)hipSetDevice(st->device);
  (void)hipDeviceSynchronize();
  dev_free(st->rec);
  dev_free(st->tiles);
  dev_free(st->rect);
  dev_free(st->rec_grad);
  dev_free(st->tile_count);
  dev_free(st->tile_order);
  dev_free(st->ranges);
  dev_free(st->keys[0]);
  dev_free(st->keys[1]);
  dev_free(st->sorted_vals);
  dev_free(st->pixel_state);
  dev_free(st->pixel_count);
  dev_free(st->pixel_grad);
  dev_free(st->counters);
  dev_free(st->pose_acc);
  dev_free(st->stats_dev);
  dev_free(st->tune_dposes);
  dev_free(st->obj_counts);
  dev_free(st->obj_part);
  for (int k = 0; k < 2; ++k) {
    dev_free(st->io[k].dev);
    if (st->io[k].pinned) (void)hipHostFree(st->io[k].pinned);
    if (st->io[k].event) (void)hipEventDestroy(st->io[k].event);
  }
  for (auto& ev : st->ev_fwd)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& ev : st->ev_bwd)
    if (ev) (void)hipEventDestroy(ev);
  if (st->counters_pinned) (void)hipHostFree(st->counters_pinned);
  if (cur >= 0 && cur != st->device) (void)hipSetDevice(cur);
  delete st;
  return CGSR_OK;
}

cgsr_status cgsr_state_reserve(cgsr_state* st, int64_t max_records, int64_t max_pixels, int64_t max_tiles,
                               int64_t max_tile_pairs) {
  if (!st) return fail(CGSR_ERR_INVALID_ARG, "state is NULL");
  if (max_records < 0 || max_pixels < 0 || max_tiles < 0 || max_tile_pairs < 0 || max_records >= (1ll << 32) ||
      max_tile_pairs >= (1ll << 32) || max_tiles >= INT32_MAX || max_pixels >= INT32_MAX)
    return fail(CGSR_ERR_INVALID_ARG, "reserve: sizes out of range");
  cgsr_status s = set_device(st);
  if (s) return s;
  return reserve(st, max_records, max_pixels, max_tiles, max_tile_pairs);
}

}  // extern "C"

namespace {

// Checks the Gaussians and cameras of a render and fills the per-view table
// (camera constants; the caller adds the image pointers).
cgsr_status check_views(const cgsr_gaussians* g, int32_t n_views, const float* poses, const cgsr_camera* cams,
                        ViewIO* io, int64_t* tiles_out, int64_t* pixels_out) {
  if (!g || !poses || !cams) return fail(CGSR_ERR_INVALID_ARG, "render: NULL argument");
  if (n_views < 1 || n_views > CGSR_MAX_VIEWS)
    return fail(CGSR_ERR_INVALID_ARG, "render: n_views must be in [1, %d]", CGSR_MAX_VIEWS);
  if (g->n < 0) return fail(CGSR_ERR_INVALID_ARG, "render: negative Gaussian count");
  if (g->n > INT32_MAX) return fail(CGSR_ERR_INVALID_ARG, "render: more than 2^31 Gaussians");
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !(g->rgb || g->sh)))
    return fail(CGSR_ERR_INVALID_ARG, "render: NULL Gaussian parameter pointer");
  if (g->sh && (g->sh_degree < 0 || g->sh_degree > CGSR_MAX_SH_DEGREE))
    return fail(CGSR_ERR_INVALID_ARG, "render: sh_degree must be in [0, %d]", CGSR_MAX_SH_DEGREE);
  if ((int64_t)g->n * n_views >= (1ll << 32))
    return fail(CGSR_ERR_INVALID_ARG, "render: more than 2^32 (view, Gaussian) records");
  if (g->n > 0 && ((uintptr_t)g->quats & 15))
    return fail(CGSR_ERR_INVALID_ARG, "render: quats must be 16-byte aligned");
  int64_t tiles = 0, pixels = 0;
  for (int v = 0; v < n_views; ++v) {
    const cgsr_camera& c = cams[v];
    if (bad_camera(c)) return fail(CGSR_ERR_INVALID_ARG, "render: invalid camera for view %d", v);
    std::memset(&io[v], 0, sizeof(ViewIO));
    ViewInfo& vi = io[v].info;
    vi.width = c.width;
    vi.height = c.height;
    vi.fx = c.fx;
    vi.fy = c.fy;
    vi.cx = c.cx;
    vi.cy = c.cy;
    vi.tiles_x = (c.width + kTile - 1) / kTile;
    vi.tiles_y = (c.height + kTile - 1) / kTile;
    vi.tile_base = (int32_t)tiles;
    vi.pixel_base = (int32_t)pixels;
    tiles += (int64_t)vi.tiles_x * vi.tiles_y;
    pixels += (int64_t)c.width * c.height;
    if (tiles >= INT32_MAX || pixels >= INT32_MAX)
      return fail(CGSR_ERR_INVALID_ARG, "render: too many tiles or pixels");
  }
  *tiles_out = tiles;
  *pixels_out = pixels;
  return CGSR_OK;
}

struct RenderArgs {
  const cgsr_gaussians* g;
  int32_t n_views;
  const float* poses;
  const ViewIO* io;
  int64_t tiles, pixels;
  bool track;
  float lambda_color, lambda_depth;
  float* loss;
  bool nu;             // track dominated pixels (Eq. 13)
  float* nu_sum;
  uint32_t* nu_count;
  bool fused = false;  // tracking: run the pose-only blend backward in the same launch
};

// Projection with emission into tile buckets -> segment sort -> blend.
cgsr_status render_impl(cgsr_state* st, const RenderArgs& a, hipStream_t stream) {
  cgsr_status s = set_device(st);
  if (s) return s;
  const int64_t records = a.g->n * (int64_t)a.n_views;
  hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &capturing));
  const bool in_capture = capturing != hipStreamCaptureStatusNone;
  if (in_capture && (records > st->cap_records || a.pixels > st->cap_pixels || a.tiles > st->cap_tiles))
    return fail(CGSR_ERR_STATE, "render: workspace too small for graph capture; reserve it first");
  s = reserve(st, records, a.pixels, a.tiles, 0);
  if (s) return s;
  st->have_forward = false;
  st->track_rb_ok = false;
  st->tracked = false;
  st->n_views = a.n_views;
  st->g = GaussianPtrs{a.g->means, a.g->log_scales, a.g->quats, a.g->opacity_logits, a.g->rgb, a.g->n,
                       a.g->sh, a.g->sh ? a.g->sh_degree : 0};
  st->poses = a.poses;
  st->total_pixels = a.pixels;
  st->total_tiles = (int32_t)a.tiles;
  st->records = records;
  std::memcpy(st->io_fwd, a.io, sizeof(ViewIO) * a.n_views);
  s = upload_io(st, 0, a.io, a.n_views, stream);
  if (s) return s;
  if (st->tiles_dirty) {
    // A previous render stopped before its sort reset the per-tile counters.
    launch_clear_u32(st->tile_count, st->cap_tiles * kTileCounterStride, stream);
    launch_clear_u32(st->counters + kCntRenderPeak, 1, stream);
  }

  const ViewTable vt{st->io[0].dev, a.n_views, (int32_t)a.g->n, st->io[0].hash};
  const bool timed = st->settings.timing && !in_capture;
  auto mark = [&](int k) -> cgsr_status {
    if (timed) HIP_TRY(hipEventRecord(st->ev_fwd[k], stream));
    return CGSR_OK;
  };
  st->fwd_timed = false;
  if ((s = mark(CGSR_STAGE_PROJECT))) return s;
  st->tiles_dirty = true;
  ProjectBufs pb = project_bufs(st);
  const bool grow = st->settings.sync_capacity && !in_capture;
  // A render that grows the buckets itself raises no overflow flag: it reads
  // the render's fullest tile back and, if that did not fit, grows the
  // buckets and projects again.
  if (grow) pb.flag_cap = UINT32_MAX;
  launch_project(st->g, a.poses, vt, pb, stream);
  HIP_TRY(hipGetLastError());
  if (grow) {
    HIP_TRY(hipMemcpyAsync(st->counters_pinned, st->counters, sizeof(uint32_t) * kCounterWords,
                           hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const int64_t need = st->counters_pinned[kCntRenderPeak];
    if (need > st->cap_tile_pairs) {
      s = grow_buckets(st, need + need / 4);
      if (s) return s;
      launch_clear_u32(st->tile_count, (int64_t)st->total_tiles * kTileCounterStride, stream);
      launch_clear_u32(st->counters + kCntRenderPeak, 1, stream);
      pb = project_bufs(st);
      pb.flag_cap = UINT32_MAX;
      launch_project(st->g, a.poses, vt, pb, stream);
      HIP_TRY(hipGetLastError());
    }
  }
  // the emission is part of the projection: its stage is empty
  if ((s = mark(CGSR_STAGE_EMIT))) return s;
  if ((s = mark(CGSR_STAGE_SORT))) return s;
  SegSortBufs sb;
  sb.keys[0] = st->keys[0];
  sb.keys[1] = st->keys[1];
  sb.sorted_vals = st->sorted_vals;
  sb.tile_count = st->tile_count;
  sb.ranges = st->ranges;
  sb.counters = st->counters;
  sb.cap = (uint32_t)st->cap_tile_pairs;
  // A fused tracking step whose buckets hold at most one key per thread of
  // its blend sorts each bucket inside the blend: one launch fewer.
  const bool sort_here = a.track && a.fused && st->cap_tile_pairs <= kTilePixels / st->settings.fwd_pixels_per_lane;
  // The blends take the tiles longest list first.  A fused tracking step with
  // more tiles than fit the chip at once orders them from this render's pair
  // counters, in a launch of its own.  One with fewer (all its tiles resident
  // from the start, where the order only spreads the long lists over the
  // CUs) takes them by the work the previous step measured per tile (each
  // quadrant's list length, kept in words 1..4 of the tile's counter line),
  // with a quadrant rotation per workgroup that evens out the SIMDs of each
  // CU: steps follow one another with a pose that moves little, so the
  // order is computed by every eager step but only by the first such step of
  // a graph capture, and a captured solve pays for it once per replay.
  // Whatever the values read, the order is a permutation of the step's
  // tiles, and any order gives every tile the same result.
  st->order_ok = false;
  const bool order = st->total_tiles < kOrderMaxTiles;
  if (!sort_here) {
    launch_segment_sort(sb, st->total_tiles, stream);
    if (order) launch_tile_order(st->ranges, nullptr, st->total_tiles, st->tile_order, stream);
    HIP_TRY(hipGetLastError());
    st->order_ok = order;
    st->track_order_ok = false;
  } else if (order && st->total_tiles >= kOrderMinTiles) {
    launch_tile_order(nullptr, st->tile_count, st->total_tiles, st->tile_order, stream);
    HIP_TRY(hipGetLastError());
    st->order_ok = true;
    st->track_order_ok = false;
  } else if (order) {
    bool fresh = true;
    if (in_capture) {
      unsigned long long id = 0;
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      HIP_TRY(hipStreamGetCaptureInfo(stream, &cs, &id));
      fresh = !st->track_order_ok || st->track_order_tiles != st->total_tiles || id != st->order_capture;
      st->order_capture = id;
    }
    if (fresh) launch_tile_order_kept(st->tile_count + 1, st->total_tiles, st->tile_order, stream);
    HIP_TRY(hipGetLastError());
    st->order_ok = true;
    st->track_order_ok = true;
    st->track_order_tiles = st->total_tiles;
  }
  if ((s = mark(CGSR_STAGE_BLEND_FWD))) return s;
  RasterBufs rb = raster_bufs(st, 0);
  rb.lambda_color = a.lambda_color;
  rb.lambda_depth = a.lambda_depth;
  rb.loss = a.loss;
  rb.nu = a.nu;
  rb.nu_sum = a.nu_sum;
  rb.nu_count = a.nu_count;
  rb.sort_here = sort_here;
  if (a.track && a.fused) {
    launch_raster_track(rb, st->settings.fwd_pixels_per_lane, stream);
    st->track_rb = rb;
    st->track_ppl = st->settings.fwd_pixels_per_lane;
  } else {
    launch_raster_forward(rb, a.track, st->settings.fwd_pixels_per_lane, stream);
  }
  HIP_TRY(hipGetLastError());
  st->tiles_dirty = false;
  if ((s = mark(CGSR_STAGE_BLEND_FWD + 1))) return s;
  st->fwd_timed = timed;
  st->tracked = a.track;
  // renders of nu and split tracking steps always count
  st->counted = st->settings.count_work || a.nu || (a.track && !a.fused);
  st->have_forward = true;
  return CGSR_OK;
}

// Blend backward -> projection backward (-> pose hand-off / Adam step).
cgsr_status backward_impl(cgsr_state* st, int slot, bool params, bool track, const GradPtrs& gp, float* dposes,
                          const PoseStep* step, hipStream_t stream, bool blend_done = false) {
  hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &capturing));
  const bool timed = st->settings.timing && capturing == hipStreamCaptureStatusNone;
  st->bwd_timed = false;
  st->track_rb_ok = false;
  if (timed) HIP_TRY(hipEventRecord(st->ev_bwd[0], stream));
  const RasterBufs rb = raster_bufs(st, slot);
  if (!blend_done) launch_raster_backward(rb, params, track, st->settings.bwd_pixels_per_lane, stream);
  if (timed) HIP_TRY(hipEventRecord(st->ev_bwd[1], stream));
  launch_project_backward(st->g, st->poses, rb.views, st->rec_grad, st->tiles, gp, params, st->pose_acc, dposes, step,
                          st->dens_grad, st->dens_count, st->counters, stream);
  HIP_TRY(hipGetLastError());
  if (timed) HIP_TRY(hipEventRecord(st->ev_bwd[2], stream));
  st->bwd_timed = timed;
  return CGSR_OK;
}

// FNV-1a over the workload's shape: what the tuned kernels' speed depends on.
uint64_t tune_key(int kind, const cgsr_gaussians* g, int32_t n_views, const cgsr_camera* cams, int32_t extra) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(kind);
  mix(g ? g->n : 0);
  mix(g && g->sh ? g->sh_degree + 1 : 0);
  mix(n_views);
  for (int v = 0; v < n_views; ++v) {
    mix(cams[v].width);
    mix(cams[v].height);
  }
  mix(extra);
  return h;
}

const cgsr_state::TunePick* tune_lookup(const cgsr_state* st, uint64_t key) {
  for (int i = 0; i < st->tune_n; ++i)
    if (st->tune_cache[i].key == key) return &st->tune_cache[i];
  return nullptr;
}

void tune_store(cgsr_state* st, uint64_t key, int32_t fwd, int32_t bwd) {
  const int cap = (int)(sizeof(st->tune_cache) / sizeof(st->tune_cache[0]));
  const int i = st->tune_n < cap ? st->tune_n++ : (int)(key % (uint64_t)cap);   // full: replace one
  st->tune_cache[i] = cgsr_state::TunePick{key, fwd, bwd};
}

bool bad_adam(const cgsr_adam_params* p) {
  return !p || !(p->beta1 >= 0.f && p->beta1 < 1.f) || !(p->beta2 >= 0.f && p->beta2 < 1.f) || !(p->eps > 0.f) ||
         !(p->lr_rho >= 0.f) || !(p->lr_phi >= 0.f);
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

cgsr_status render_entry(const char* name, cgsr_state* st, const cgsr_gaussians* g, int32_t n_views,
                         const float* poses, const cgsr_camera* cams, const float* const* depth_obs,
                         const cgsr_images* outs, bool nu, int32_t* const* dominant, float* nu_sum,
                         uint32_t* nu_count, void* stream) {
  if (!st || !outs) return fail(CGSR_ERR_INVALID_ARG, "%s: NULL argument", name);
  ViewIO io[CGSR_MAX_VIEWS];
  int64_t tiles = 0, pixels = 0;
  cgsr_status s = check_views(g, n_views, poses, cams, io, &tiles, &pixels);
  if (s) return s;
  for (int v = 0; v < n_views; ++v) {
    io[v].depth_obs = depth_obs ? depth_obs[v] : nullptr;
    io[v].color = outs[v].color;
    io[v].depth = outs[v].depth;
    io[v].opacity = outs[v].opacity;
    io[v].depth_median = outs[v].depth_median;
    io[v].uncertainty = outs[v].uncertainty;
    if (io[v].uncertainty && !io[v].depth_obs)
      return fail(CGSR_ERR_INVALID_ARG, "%s: view %d asks for uncertainty without sensor depth", name, v);
    if (nu) {
      if (!io[v].depth_obs) return fail(CGSR_ERR_INVALID_ARG, "%s: view %d has no sensor depth", name, v);
      io[v].dominant = dominant ? dominant[v] : nullptr;
    }
  }
  return render_impl(st, RenderArgs{g, n_views, poses, io, tiles, pixels, false, 0.f, 0.f, nullptr, nu, nu_sum,
                                    nu_count},
                     (hipStream_t)stream);
}

}  // namespace

extern "C" {

cgsr_status cgsr_render(cgsr_state* st, const cgsr_gaussians* g, int32_t n_views, const float* poses,
                        const cgsr_camera* cams, const float* const* depth_obs, const cgsr_images* outs,
                        void* stream) {
  return render_entry("cgsr_render", st, g, n_views, poses, cams, depth_obs, outs, false, nullptr, nullptr, nullptr,
                      stream);
}

cgsr_status cgsr_render_nu(cgsr_state* st, const cgsr_gaussians* g, int32_t n_views, const float* poses,
                           const cgsr_camera* cams, const float* const* depth_obs, const cgsr_images* outs,
                           int32_t* const* dominant, float* nu_sum, uint32_t* nu_count, void* stream) {
  if (!depth_obs) return fail(CGSR_ERR_INVALID_ARG, "cgsr_render_nu: sensor depth is required");
  if ((nu_sum == nullptr) != (nu_count == nullptr))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_render_nu: give both nu_sum and nu_count, or neither");
  return render_entry("cgsr_render_nu", st, g, n_views, poses, cams, depth_obs, outs, true, dominant, nu_sum,
                      nu_count, stream);
}

cgsr_status cgsr_nu_prune(int64_t n, const float* nu_sum, const uint32_t* nu_count, float tau, float low_opacity,
                          float* opacity_logits, float* nu, uint32_t* n_pruned, void* stream) {
  if (n < 0) return fail(CGSR_ERR_INVALID_ARG, "cgsr_nu_prune: negative count");
  if (n > 0 && (!nu_sum || !nu_count)) return fail(CGSR_ERR_INVALID_ARG, "cgsr_nu_prune: NULL accumulator");
  if (!(tau >= 0.f) || !(low_opacity > 0.f && low_opacity < 1.f))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_nu_prune: need tau >= 0 and 0 < low_opacity < 1");
  const float low_logit = (float)std::log((double)low_opacity / (1.0 - (double)low_opacity));
  launch_nu_prune(n, nu_sum, nu_count, tau, low_logit, opacity_logits, nu, n_pruned, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return CGSR_OK;
}

cgsr_status cgsr_backward(cgsr_state* st, const cgsr_image_grads* dimgs, const cgsr_gaussian_grads* dG,
                          float* dposes, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!st || !dimgs) return fail(CGSR_ERR_INVALID_ARG, "cgsr_backward: NULL argument");
  if (!st->have_forward) return fail(CGSR_ERR_STATE, "cgsr_backward: no forward pass on this state");
  if (st->tracked) return fail(CGSR_ERR_STATE, "cgsr_backward: the last forward was a tracking step");
  const int n_views = st->n_views;
  const bool params = dG && (dG->means || dG->log_scales || dG->quats || dG->opacity_logits || dG->rgb || dG->sh);
  if (!params && !dposes) return CGSR_OK;
  ViewIO io[CGSR_MAX_VIEWS];
  for (int v = 0; v < n_views; ++v) {
    io[v] = st->io_fwd[v];
    io[v].g_color = dimgs[v].color;
    io[v].g_depth = dimgs[v].depth;
    io[v].g_opacity = dimgs[v].opacity;
    io[v].g_median = dimgs[v].depth_median;
    io[v].g_uncertainty = dimgs[v].uncertainty;
    if (io[v].g_uncertainty && !io[v].depth_obs)
      return fail(CGSR_ERR_INVALID_ARG, "cgsr_backward: view %d has an uncertainty gradient but no sensor depth", v);
  }
  cgsr_status s = set_device(st);
  if (s) return s;
  s = upload_io(st, 1, io, n_views, stream);
  if (s) return s;
  GradPtrs gp{};
  if (params) gp = GradPtrs{dG->means, dG->log_scales, dG->quats, dG->opacity_logits, dG->rgb, dG->sh};
  return backward_impl(st, 1, params, false, gp, dposes, nullptr, stream);
}

cgsr_status cgsr_tracking_step(cgsr_state* st, const cgsr_gaussians* g, int32_t n_views, float* poses,
                               const cgsr_camera* cams, const float* const* target_color,
                               const float* const* target_depth, float lambda_color, float lambda_depth,
                               float* dposes, float* adam, const cgsr_adam_params* adam_params, float* loss,
                               void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!st || !target_color || !target_depth) return fail(CGSR_ERR_INVALID_ARG, "cgsr_tracking_step: NULL argument");
  if (adam && bad_adam(adam_params)) return fail(CGSR_ERR_INVALID_ARG, "cgsr_tracking_step: bad Adam parameters");
  if (!(lambda_color >= 0.f) || !(lambda_depth >= 0.f))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_tracking_step: loss weights must be non-negative");
  ViewIO io[CGSR_MAX_VIEWS];
  int64_t tiles = 0, pixels = 0;
  cgsr_status s = check_views(g, n_views, poses, cams, io, &tiles, &pixels);
  if (s) return s;
  for (int v = 0; v < n_views; ++v) {
    if (!target_color[v] || !target_depth[v])
      return fail(CGSR_ERR_INVALID_ARG, "cgsr_tracking_step: view %d has no target", v);
    io[v].t_color = target_color[v];
    io[v].t_depth = target_depth[v];
  }
  // With a pose update or gradient to produce, the blend forward and its
  // pose-only backward share one launch per tile.
  const bool fused = dposes || adam;
  RenderArgs ra{g, n_views, poses, io, tiles, pixels, true, lambda_color, lambda_depth, loss, false, nullptr, nullptr};
  ra.fused = fused;
  s = render_impl(st, ra, stream);
  if (s) return s;
  if (!fused) return CGSR_OK;
  PoseStep step{poses, adam, AdamParams{}};
  if (adam)
    step.params = AdamParams{adam_params->lr_rho, adam_params->lr_phi, adam_params->beta1, adam_params->beta2,
                             adam_params->eps};
  s = backward_impl(st, 0, false, true, GradPtrs{}, dposes, adam ? &step : nullptr, stream, true);
  if (!s) st->track_rb_ok = true;
  return s;
}

cgsr_status cgsr_time_tracking_blend(cgsr_state* st, int32_t reps, void* stream_, float* ms_out) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!st || !ms_out) return fail(CGSR_ERR_INVALID_ARG, "cgsr_time_tracking_blend: NULL argument");
  if (reps < 1 || reps > 100000)
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_time_tracking_blend: reps must be 1 .. 100000");
  if (!st->track_rb_ok)
    return fail(CGSR_ERR_STATE, "cgsr_time_tracking_blend: the last call on this state was not a tracking step "
                                "with a pose gradient or update");
  cgsr_status s = set_device(st);
  if (s) return s;
  hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &capturing));
  if (capturing != hipStreamCaptureStatusNone)
    return fail(CGSR_ERR_STATE, "cgsr_time_tracking_blend: not available under graph capture");
  RasterBufs rb = st->track_rb;
  rb.loss = nullptr;        // the step's loss sum is not added to again
  rb.keep_counts = true;
  hipEvent_t ev[2] = {nullptr, nullptr};
  HIP_TRY(hipEventCreate(&ev[0]));
  hipError_t e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(CGSR_ERR_HIP, "cgsr_time_tracking_blend: %s", hipGetErrorString(e));
  }
  // From here on the counters are restored and always reset again below.
  if (rb.sort_here) launch_restore_counts(st->tile_count, st->ranges, st->total_tiles, stream);
  float ms = 0.f;
  e = hipEventRecord(ev[0], stream);
  for (int r = 0; e == hipSuccess && r < reps; ++r) {
    launch_raster_track(rb, st->track_ppl, stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
  // leave the state as the step left it: counters reset, record sums cleared
  if (rb.sort_here) launch_clear_u32(st->tile_count, (int64_t)st->total_tiles * kTileCounterStride, stream);
  launch_clear_u32(reinterpret_cast<uint32_t*>(st->rec_grad), st->records * kGradStride, stream);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (e != hipSuccess) return fail(CGSR_ERR_HIP, "cgsr_time_tracking_blend: %s", hipGetErrorString(e));
  *ms_out = ms / (float)reps;
  st->track_rb_ok = true;
  return CGSR_OK;
}

cgsr_status cgsr_autotune_tracking(cgsr_state* st, const cgsr_gaussians* g, int32_t n_views, const float* poses,
                                   const cgsr_camera* cams, const float* const* target_color,
                                   const float* const* target_depth, int32_t repeats, cgsr_settings* out,
                                   void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!st) return fail(CGSR_ERR_INVALID_ARG, "cgsr_autotune_tracking: NULL state");
  if (repeats < 1 || repeats > 1000) return fail(CGSR_ERR_INVALID_ARG, "cgsr_autotune_tracking: repeats in [1, 1000]");
  hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &capturing));
  if (capturing != hipStreamCaptureStatusNone)
    return fail(CGSR_ERR_STATE, "cgsr_autotune_tracking: not under graph capture");
  if (!g || !cams || n_views < 1 || n_views > CGSR_MAX_VIEWS)
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_autotune_tracking: need the Gaussians and 1 .. %d cameras", CGSR_MAX_VIEWS);
  cgsr_status s = set_device(st);
  if (s) return s;
  // the pick depends on the bucket size too: whether the blend sorts its own
  const uint64_t key = tune_key(1, g, n_views, cams, (int32_t)std::min<int64_t>(st->cap_tile_pairs, 1 << 20) * 2 +
                                                         st->settings.count_work);
  if (const cgsr_state::TunePick* hit = tune_lookup(st, key)) {
    st->settings.fwd_pixels_per_lane = hit->fwd;
    st->settings.bwd_pixels_per_lane = hit->bwd;
    if (out) *out = st->settings;
    return CGSR_OK;
  }
  const cgsr_settings saved = st->settings;
  hipEvent_t ev[2] = {nullptr, nullptr};
  HIP_TRY(hipEventCreate(&ev[0]));
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(CGSR_ERR_HIP, "cgsr_autotune_tracking: hipEventCreate failed");
  }
  const int32_t cand[3] = {1, 2, 4};
  // Two passes over the candidates, each candidate's faster one kept: the
  // first pass also warms the GPU up, which would otherwise count against
  // whichever candidate runs first.
  float time[3] = {1e30f, 1e30f, 1e30f};
  for (int it = 0; it < kTunePasses * 3 && !s; ++it) {
    const int c = it % 3;
    // The whole step (projection, sort unless the blend sorts its own
    // buckets, fused blend, projection backward) between two events: a
    // candidate whose buckets no longer fit one key per lane pays for the
    // segmented sort it needs.  One step with the caller's settings first
    // (it may grow the buckets), then the timed steps without the capacity
    // read-back.
    st->settings = saved;
    st->settings.timing = 0;
    st->settings.fwd_pixels_per_lane = cand[c];
    st->settings.bwd_pixels_per_lane = cand[c];
    s = cgsr_tracking_step(st, g, n_views, const_cast<float*>(poses), cams, target_color, target_depth, 1.f, 1.f,
                           st->tune_dposes, nullptr, nullptr, nullptr, stream);
    st->settings.sync_capacity = 0;
    hipError_t e = hipSuccess;
    if (!s) e = hipEventRecord(ev[0], stream);
    for (int r = 0; r < repeats && !s && e == hipSuccess; ++r)
      s = cgsr_tracking_step(st, g, n_views, const_cast<float*>(poses), cams, target_color, target_depth, 1.f, 1.f,
                             st->tune_dposes, nullptr, nullptr, nullptr, stream);
    float ms = 0.f;
    if (!s && e == hipSuccess) e = hipEventRecord(ev[1], stream);
    if (!s && e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (!s && e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (!s && e != hipSuccess) s = fail(CGSR_ERR_HIP, "cgsr_autotune_tracking: %s", hipGetErrorString(e));
    if (!s) time[c] = std::min(time[c], ms);
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  st->settings = saved;
  if (s) return s;
  int32_t pick = cand[0];
  float best = time[0];
  for (int c = 1; c < 3; ++c)
    if (time[c] < best) {
      best = time[c];
      pick = cand[c];
    }
  // the tracking step's forward and pose backward are one fused launch, so
  // one setting serves both
  st->settings.fwd_pixels_per_lane = pick;
  st->settings.bwd_pixels_per_lane = pick;
  tune_store(st, key, pick, pick);
  if (out) *out = st->settings;
  return CGSR_OK;
}

cgsr_status cgsr_autotune_render(cgsr_state* st, const cgsr_gaussians* g, int32_t n_views, const float* poses,
                                 const cgsr_camera* cams, const float* const* depth_obs, const cgsr_images* outs,
                                 const cgsr_image_grads* dimgs, const cgsr_gaussian_grads* dG, float* dposes,
                                 int32_t repeats, cgsr_settings* out, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!st || !g || !cams || !outs || !dimgs)
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_autotune_render: NULL argument");
  if (n_views < 1 || n_views > CGSR_MAX_VIEWS)
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_autotune_render: n_views in [1, %d]", CGSR_MAX_VIEWS);
  if (repeats < 1 || repeats > 1000) return fail(CGSR_ERR_INVALID_ARG, "cgsr_autotune_render: repeats in [1, 1000]");
  hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &capturing));
  if (capturing != hipStreamCaptureStatusNone)
    return fail(CGSR_ERR_STATE, "cgsr_autotune_render: not under graph capture");
  cgsr_status s = set_device(st);
  if (s) return s;
  const bool params = dG && (dG->means || dG->log_scales || dG->quats || dG->opacity_logits || dG->rgb || dG->sh);
  int32_t what = (params ? 1 : 0) | (dposes ? 2 : 0);
  for (int v = 0; v < n_views; ++v)
    what |= (depth_obs && depth_obs[v] ? 4 : 0) | (outs[v].uncertainty ? 8 : 0) | (dimgs[v].opacity ? 16 : 0) |
            (dimgs[v].depth_median ? 32 : 0);
  const uint64_t key = tune_key(2, g, n_views, cams, what);
  if (const cgsr_state::TunePick* hit = tune_lookup(st, key)) {
    st->settings.fwd_pixels_per_lane = hit->fwd;
    st->settings.bwd_pixels_per_lane = hit->bwd;
    if (out) *out = st->settings;
    return CGSR_OK;
  }
  const cgsr_settings saved = st->settings;
  hipEvent_t ev[2] = {nullptr, nullptr};
  HIP_TRY(hipEventCreate(&ev[0]));
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(CGSR_ERR_HIP, "cgsr_autotune_render: hipEventCreate failed");
  }
  const int32_t cand[3] = {1, 2, 4};
  // two passes, each pair's faster one kept (see cgsr_autotune_tracking)
  float time[9];
  for (float& t : time) t = 1e30f;
  for (int it = 0; it < kTunePasses * 9 && !s; ++it) {
    const int c = it % 9;
    // One render + backward with the caller's settings (it may grow the
    // buckets), then the timed ones without the capacity read-back.
    st->settings = saved;
    st->settings.timing = 0;
    st->settings.fwd_pixels_per_lane = cand[c / 3];
    st->settings.bwd_pixels_per_lane = cand[c % 3];
    hipError_t e = hipSuccess;
    for (int r = 0; r <= repeats && !s && e == hipSuccess; ++r) {
      if (r == 1) {
        st->settings.sync_capacity = 0;
        e = hipEventRecord(ev[0], stream);
        if (e != hipSuccess) break;
      }
      s = cgsr_render(st, g, n_views, poses, cams, depth_obs, outs, stream);
      if (!s) s = cgsr_backward(st, dimgs, dG, dposes, stream);
    }
    float ms = 0.f;
    if (!s && e == hipSuccess) e = hipEventRecord(ev[1], stream);
    if (!s && e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (!s && e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (!s && e != hipSuccess) s = fail(CGSR_ERR_HIP, "cgsr_autotune_render: %s", hipGetErrorString(e));
    if (!s) time[c] = std::min(time[c], ms);
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  st->settings = saved;
  if (s) return s;
  int32_t pick_f = cand[0], pick_b = cand[0];
  float best = time[0];
  for (int c = 1; c < 9; ++c)
    if (time[c] < best) {
      best = time[c];
      pick_f = cand[c / 3];
      pick_b = cand[c % 3];
    }
  st->settings.fwd_pixels_per_lane = pick_f;
  st->settings.bwd_pixels_per_lane = pick_b;
  tune_store(st, key, pick_f, pick_b);
  if (out) *out = st->settings;
  return CGSR_OK;
}

cgsr_status cgsr_tracking_loss_grad(int32_t width, int32_t height, const float* color, const float* depth,
                                    const float* target_color, const float* target_depth, float lambda_color,
                                    float lambda_depth, float* dcolor, float* ddepth, float* loss, void* stream) {
  if (width < 1 || height < 1) return fail(CGSR_ERR_INVALID_ARG, "tracking loss: empty image");
  if (!color || !depth || !target_color || !target_depth || !dcolor || !ddepth)
    return fail(CGSR_ERR_INVALID_ARG, "tracking loss: NULL argument");
  launch_tracking_loss(width, height, color, depth, target_color, target_depth, lambda_color, lambda_depth, dcolor,
                       ddepth, loss, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return CGSR_OK;
}

cgsr_status cgsr_mapping_loss_grad(int32_t width, int32_t height, const float* color, const float* depth,
                                   const float* uncertainty, const float* target_color, const float* target_depth,
                                   float* dcolor, float* ddepth, float* duncertainty, float* loss, void* stream) {
  if (width < 1 || height < 1) return fail(CGSR_ERR_INVALID_ARG, "mapping loss: empty image");
  if (!color || !depth || !uncertainty || !target_color || !target_depth || !dcolor || !ddepth || !duncertainty)
    return fail(CGSR_ERR_INVALID_ARG, "mapping loss: NULL argument");
  launch_mapping_loss(width, height, color, depth, uncertainty, target_color, target_depth, dcolor, ddepth,
                      duncertainty, loss, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return CGSR_OK;
}

cgsr_status cgsr_pose_adam_step(int32_t n_views, float* poses, float* dposes, float* adam,
                                const cgsr_adam_params* p, void* stream) {
  if (n_views < 1 || n_views > CGSR_MAX_VIEWS) return fail(CGSR_ERR_INVALID_ARG, "pose adam: bad view count");
  if (!poses || !dposes || !adam) return fail(CGSR_ERR_INVALID_ARG, "pose adam: NULL argument");
  if (bad_adam(p)) return fail(CGSR_ERR_INVALID_ARG, "pose adam: bad hyper-parameters");
  launch_pose_adam(n_views, poses, dposes, adam, AdamParams{p->lr_rho, p->lr_phi, p->beta1, p->beta2, p->eps},
                   (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return CGSR_OK;
}

cgsr_status cgsr_mapping_objective(cgsr_state* st, const cgsr_mapping_weights* w, const cgsr_images* maps,
                                   const float* const* target_color, const float* const* target_depth,
                                   const cgsr_images* dimgs, float* dlog_scales, float* loss, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (!st || !w || !maps || !dimgs) return fail(CGSR_ERR_INVALID_ARG, "cgsr_mapping_objective: NULL argument");
  if (!st->have_forward) return fail(CGSR_ERR_STATE, "cgsr_mapping_objective: no forward pass on this state");
  if (st->tracked) return fail(CGSR_ERR_STATE, "cgsr_mapping_objective: the last forward was a tracking step");
  const float ws[7] = {w->color, w->ssim, w->geo, w->align, w->iso, w->var, w->iso_epsilon};
  for (float x : ws)
    if (!std::isfinite(x)) return fail(CGSR_ERR_INVALID_ARG, "cgsr_mapping_objective: non-finite weight");
  const int n_views = st->n_views;
  int64_t max_px = 0;
  for (int v = 0; v < n_views; ++v) {
    const cgsr_images& m = maps[v];
    const cgsr_images& d = dimgs[v];
    const float* tc = target_color ? target_color[v] : nullptr;
    const float* td = target_depth ? target_depth[v] : nullptr;
    const bool bad = ((w->color != 0.f || w->ssim != 0.f) && !d.color) || (d.color && (!m.color || !tc)) ||
                     ((w->geo != 0.f || w->align != 0.f) && !d.depth) || (d.depth && (!m.depth || !td)) ||
                     ((w->align != 0.f || d.depth_median) && (!m.depth_median || !m.depth)) ||
                     (w->var != 0.f && !d.uncertainty) || (d.uncertainty && !m.uncertainty);
    if (bad)
      return fail(CGSR_ERR_INVALID_ARG, "cgsr_mapping_objective: view %d lacks a map, target or gradient output "
                  "that its weighted terms need", v);
    max_px = std::max<int64_t>(max_px, (int64_t)st->io_fwd[v].info.width * st->io_fwd[v].info.height);
  }
  cgsr_status s = set_device(st);
  if (s) return s;
  if (w->ssim != 0.f && max_px > st->cap_obj_pixels) {
    hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &capturing));
    if (capturing != hipStreamCaptureStatusNone)
      return fail(CGSR_ERR_STATE, "cgsr_mapping_objective: SSIM scratch too small for graph capture; run once first");
    HIP_TRY(hipDeviceSynchronize());
    dev_free(st->obj_part);
    st->cap_obj_pixels = 0;
    if ((s = dev_alloc(&st->obj_part, 9 * max_px))) return s;
    st->cap_obj_pixels = max_px;
  }
  const ObjectiveWeights ow{w->color, w->ssim, w->geo, w->align, w->iso, w->var};
  for (int v = 0; v < n_views; ++v) {
    const cgsr_images& m = maps[v];
    const cgsr_images& d = dimgs[v];
    ObjectiveView o;
    o.width = st->io_fwd[v].info.width;
    o.height = st->io_fwd[v].info.height;
    o.color = m.color;
    o.depth = m.depth;
    o.median = (w->align != 0.f || d.depth_median) ? m.depth_median : nullptr;
    o.unc = m.uncertainty;
    o.tcolor = target_color ? target_color[v] : nullptr;
    o.tdepth = target_depth ? target_depth[v] : nullptr;
    o.dcolor = d.color;
    o.ddepth = d.depth;
    o.dmedian = d.depth_median;
    o.dunc = d.uncertainty;
    o.loss = loss ? loss + v : nullptr;
    launch_objective_view(o, ow, st->obj_part, stream);
    HIP_TRY(hipGetLastError());
  }
  if (w->iso != 0.f) {
    launch_iso(st->g.n, n_views, st->tiles, st->obj_counts, st->g.log_scales, w->iso, w->iso_epsilon, dlog_scales,
               loss, stream);
    HIP_TRY(hipGetLastError());
  }
  return CGSR_OK;
}

cgsr_status cgsr_gaussian_adam_step(int64_t n, const cgsr_gaussian_grads* params, const cgsr_gaussian_grads* grads,
                                    float* moments, uint32_t* step, const cgsr_gaussian_adam_params* hp,
                                    void* stream) {
  if (n < 0 || !params || !grads || !hp || !moments || !step)
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_gaussian_adam_step: NULL argument or negative count");
  if (!(hp->beta1 >= 0.f && hp->beta1 < 1.f) || !(hp->beta2 >= 0.f && hp->beta2 < 1.f) || !(hp->eps > 0.f))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_gaussian_adam_step: bad Adam parameters");
  const bool sh = params->sh || grads->sh;
  if (sh && !(params->sh && grads->sh))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_gaussian_adam_step: sh needs both the parameters and their gradients");
  if (sh && (hp->sh_degree < 0 || hp->sh_degree > CGSR_MAX_SH_DEGREE))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_gaussian_adam_step: sh_degree must be 0 .. %d", CGSR_MAX_SH_DEGREE);
  if (sh && !(hp->lr_sh_rest >= 0.f))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_gaussian_adam_step: negative learning rate");
  GaussianAdam a;
  float* const ps[5] = {params->means, params->log_scales, params->quats, params->opacity_logits,
                        sh ? params->sh : params->rgb};
  float* const gs[5] = {grads->means, grads->log_scales, grads->quats, grads->opacity_logits,
                        sh ? grads->sh : grads->rgb};
  const float lrs[5] = {hp->lr_means, hp->lr_log_scales, hp->lr_quats, hp->lr_opacity_logits, hp->lr_rgb};
  for (int k = 0; k < 5; ++k) {
    if (n > 0 && (!ps[k] || !gs[k]))
      return fail(CGSR_ERR_INVALID_ARG, "cgsr_gaussian_adam_step: every parameter and gradient array is required");
    if (!(lrs[k] >= 0.f)) return fail(CGSR_ERR_INVALID_ARG, "cgsr_gaussian_adam_step: negative learning rate");
    a.param[k] = ps[k];
    a.grad[k] = gs[k];
    a.lr[k] = lrs[k];
  }
  a.beta1 = hp->beta1;
  a.beta2 = hp->beta2;
  a.eps = hp->eps;
  a.colour_width = sh ? 3 * (hp->sh_degree + 1) * (hp->sh_degree + 1) : 3;
  a.lr_sh_rest = sh ? hp->lr_sh_rest : 0.f;
  launch_gaussian_adam(n, a, moments, step, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return CGSR_OK;
}

namespace {

// Checks a writable set; colour_w receives the colour floats per Gaussian.
// A set of no rows (empty) may have every array NULL; then *colour_w = 0.
static cgsr_status check_arrays(const cgsr_gaussian_arrays* a, const char* what, int* colour_w, bool empty = false) {
  if (!a) return fail(CGSR_ERR_INVALID_ARG, "%s: NULL arrays", what);
  if (empty && !a->means && !a->log_scales && !a->quats && !a->opacity_logits && !a->rgb && !a->sh) {
    *colour_w = 0;
    return CGSR_OK;
  }
  if (!a->means || !a->log_scales || !a->quats || !a->opacity_logits || !(a->sh || a->rgb))
    return fail(CGSR_ERR_INVALID_ARG, "%s: NULL parameter array", what);
  if (a->sh && (a->sh_degree < 0 || a->sh_degree > CGSR_MAX_SH_DEGREE))
    return fail(CGSR_ERR_INVALID_ARG, "%s: sh_degree must be in [0, %d]", what, CGSR_MAX_SH_DEGREE);
  *colour_w = a->sh ? 3 * (a->sh_degree + 1) * (a->sh_degree + 1) : 3;
  return CGSR_OK;
}

static GaussArrays gauss_arrays(const cgsr_gaussian_arrays* a) {
  return GaussArrays{a->means, a->log_scales, a->quats, a->opacity_logits, a->sh ? nullptr : a->rgb, a->sh};
}

// src and dst of an out-of-place pass: same colour layout, no shared array.
// src_empty / dst_empty: that side has no rows and may be all NULL.
static cgsr_status check_src_dst(const cgsr_gaussian_arrays* src, const cgsr_gaussian_arrays* dst, const char* what,
                                 int* colour_w, bool src_empty = false, bool dst_empty = false) {
  int wd = 0;
  cgsr_status s = check_arrays(src, what, colour_w, src_empty);
  if (!s) s = check_arrays(dst, what, &wd, dst_empty);
  if (s) return s;
  const bool both = src->means && dst->means;   // neither side empty
  if (both && ((src->sh != nullptr) != (dst->sh != nullptr) || wd != *colour_w))
    return fail(CGSR_ERR_INVALID_ARG, "%s: src and dst differ in their colour layout", what);
  if (*colour_w == 0) *colour_w = wd;   // an empty src takes dst's layout
  const void* sp[6] = {src->means, src->log_scales, src->quats, src->opacity_logits, src->rgb, src->sh};
  const void* dp[6] = {dst->means, dst->log_scales, dst->quats, dst->opacity_logits, dst->rgb, dst->sh};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j)
      if (sp[i] && sp[i] == dp[j]) return fail(CGSR_ERR_INVALID_ARG, "%s: dst shares an array with src", what);
  return CGSR_OK;
}

}  // namespace

cgsr_status cgsr_spawn_gaussians(const cgsr_gaussian_arrays* dst, int64_t n, int64_t capacity, const cgsr_camera* cam,
                                 const float* pose, const float* color, const float* depth, const float* opacity,
                                 float psi, int32_t stride, float init_logit, int64_t* n_out, void* stream) {
  int cw = 0;
  cgsr_status s = check_arrays(dst, "cgsr_spawn_gaussians", &cw, capacity == 0);
  if (s) return s;
  if (!cam || !pose || !color || !depth || !n_out)
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_spawn_gaussians: NULL argument");
  if (bad_camera(*cam)) return fail(CGSR_ERR_INVALID_ARG, "cgsr_spawn_gaussians: invalid camera");
  if (n < 0 || capacity < n || capacity > INT32_MAX)
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_spawn_gaussians: need 0 <= n <= capacity <= 2^31 - 1");
  if (stride < 1 || !(psi == psi) || !(init_logit == init_logit))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_spawn_gaussians: stride must be >= 1, psi and init_logit finite");
  ViewInfo vi{};
  vi.width = cam->width;
  vi.height = cam->height;
  vi.fx = cam->fx;
  vi.fy = cam->fy;
  vi.cx = cam->cx;
  vi.cy = cam->cy;
  uint32_t total = 0;
  HIP_TRY(run_spawn(gauss_arrays(dst), n, capacity, vi, pose, color, depth, opacity, psi, stride, init_logit,
                    dst->sh ? (dst->sh_degree + 1) * (dst->sh_degree + 1) : 0, &total, (hipStream_t)stream));
  *n_out = n + (int64_t)total;
  if (*n_out > capacity)
    return fail(CGSR_ERR_CAPACITY, "cgsr_spawn_gaussians: %lld Gaussians needed, capacity %lld",
                (long long)*n_out, (long long)capacity);
  return CGSR_OK;
}

namespace {

// Argument checks and the extra-array table shared by both compaction entry
// points.
static cgsr_status compact_args(const char* what, int64_t n, const uint8_t* keep, const cgsr_gaussian_arrays* src,
                                const cgsr_gaussian_arrays* dst, int32_t n_extra, const float* const* extra_src,
                                float* const* extra_dst, const int32_t* extra_width, int64_t* n_out, int* cw,
                                ExtraArrays* ex) {
  cgsr_status s = check_src_dst(src, dst, what, cw, n == 0, n == 0);
  if (s) return s;
  if (!n_out || (n > 0 && !keep)) return fail(CGSR_ERR_INVALID_ARG, "%s: NULL argument", what);
  if (n < 0 || n > INT32_MAX) return fail(CGSR_ERR_INVALID_ARG, "%s: need 0 <= n < 2^31", what);
  if (n_extra < 0 || n_extra > kMaxExtraArrays || (n_extra > 0 && (!extra_src || !extra_dst || !extra_width)))
    return fail(CGSR_ERR_INVALID_ARG, "%s: 0 .. %d extra arrays with their pointers and widths", what,
                kMaxExtraArrays);
  *ex = ExtraArrays{};
  ex->n = n_extra;
  for (int e = 0; e < n_extra; ++e) {
    if (!extra_src[e] || !extra_dst[e] || extra_width[e] < 1 || extra_src[e] == extra_dst[e])
      return fail(CGSR_ERR_INVALID_ARG, "%s: bad extra array %d", what, e);
    ex->src[e] = extra_src[e];
    ex->dst[e] = extra_dst[e];
    ex->width[e] = extra_width[e];
  }
  return CGSR_OK;
}

}  // namespace

cgsr_status cgsr_compact_gaussians(int64_t n, const uint8_t* keep, const cgsr_gaussian_arrays* src,
                                   const cgsr_gaussian_arrays* dst, int32_t n_extra, const float* const* extra_src,
                                   float* const* extra_dst, const int32_t* extra_width, int64_t* n_out,
                                   void* stream) {
  int cw = 0;
  ExtraArrays ex;
  cgsr_status s = compact_args("cgsr_compact_gaussians", n, keep, src, dst, n_extra, extra_src, extra_dst,
                               extra_width, n_out, &cw, &ex);
  if (s) return s;
  uint32_t total = 0;
  HIP_TRY(run_compact(n, keep, gauss_arrays(src), gauss_arrays(dst), cw, ex, &total, (hipStream_t)stream));
  *n_out = total;
  return CGSR_OK;
}

cgsr_status cgsr_compact_gaussians_noalloc(int64_t n, const uint8_t* keep, const cgsr_gaussian_arrays* src,
                                           const cgsr_gaussian_arrays* dst, int32_t n_extra,
                                           const float* const* extra_src, float* const* extra_dst,
                                           const int32_t* extra_width, int64_t* n_out, void* stream) {
  int cw = 0;
  ExtraArrays ex;
  cgsr_status s = compact_args("cgsr_compact_gaussians_noalloc", n, keep, src, dst, n_extra, extra_src, extra_dst,
                               extra_width, n_out, &cw, &ex);
  if (s) return s;
  if (n > CGSR_COMPACT_NOALLOC_MAX_N)
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_compact_gaussians_noalloc: n = %lld exceeds its fixed scratch (%d)",
                (long long)n, CGSR_COMPACT_NOALLOC_MAX_N);
  uint32_t total = 0;
  HIP_TRY(run_compact_noalloc(n, keep, gauss_arrays(src), gauss_arrays(dst), cw, ex, &total, (hipStream_t)stream));
  *n_out = total;
  return CGSR_OK;
}

cgsr_status cgsr_set_densify_stats(cgsr_state* st, float* grad_accum, uint32_t* count) {
  if (!st) return fail(CGSR_ERR_INVALID_ARG, "state is NULL");
  if ((grad_accum == nullptr) != (count == nullptr))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_set_densify_stats: both arrays or neither");
  st->dens_grad = grad_accum;
  st->dens_count = count;
  return CGSR_OK;
}

cgsr_status cgsr_densify_gaussians(int64_t n, const float* grad_accum, const uint32_t* count, float grad_threshold,
                                   float dense_scale, const float* normals, const cgsr_gaussian_arrays* src,
                                   const cgsr_gaussian_arrays* dst, int64_t capacity, int64_t* n_out,
                                   void* stream) {
  int cw = 0;
  cgsr_status s = check_src_dst(src, dst, "cgsr_densify_gaussians", &cw, n == 0, capacity == 0);
  if (s) return s;
  if (!n_out || (n > 0 && (!grad_accum || !count || !normals)))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_densify_gaussians: NULL argument");
  if (n < 0 || n > INT32_MAX / 3 || capacity < 0 || capacity > INT32_MAX)
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_densify_gaussians: need 0 <= n < 2^31 / 3 and 0 <= capacity < 2^31");
  if (!(grad_threshold == grad_threshold) || !(dense_scale == dense_scale))
    return fail(CGSR_ERR_INVALID_ARG, "cgsr_densify_gaussians: thresholds must not be NaN");
  uint32_t t[kRankKinds] = {0, 0, 0};
  HIP_TRY(run_densify(n, grad_accum, count, grad_threshold, dense_scale, normals, gauss_arrays(src), gauss_arrays(dst),
                      cw, capacity, t, (hipStream_t)stream));
  *n_out = (int64_t)t[0] + t[1] + 2 * (int64_t)t[2];
  if (*n_out > capacity)
    return fail(CGSR_ERR_CAPACITY, "cgsr_densify_gaussians: %lld Gaussians needed, capacity %lld",
                (long long)*n_out, (long long)capacity);
  return CGSR_OK;
}

cgsr_status cgsr_state_check(cgsr_state* st, void* stream) {
  if (!st) return fail(CGSR_ERR_INVALID_ARG, "state is NULL");
  cgsr_status s = set_device(st);
  if (s) return s;
  HIP_TRY(hipMemcpyAsync(st->counters_pinned, st->counters, sizeof(uint32_t) * 4, hipMemcpyDeviceToHost,
                         (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  const uint32_t overflow = st->counters_pinned[kCntOverflow], peak = st->counters_pinned[kCntPeak];
  const uint32_t stale = st->counters_pinned[kCntStaleTable];
  // start the next checking period (words kCntOverflow .. kCntStaleTable)
  launch_clear_u32(st->counters + kCntOverflow, 3, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  if (stale)
    return fail(CGSR_ERR_STATE,
                "a captured graph was replayed after another call on this state rewrote its table of cameras and "
                "image pointers; that replay's results are not the captured loop's");
  if (overflow)
    return fail(CGSR_ERR_CAPACITY, "a tile needed %u pairs, the buckets hold %lld", peak,
                (long long)st->cap_tile_pairs);
  return CGSR_OK;
}

cgsr_status cgsr_get_stats(cgsr_state* st, void* stream_, cgsr_stats* out) {
  if (!st || !out) return fail(CGSR_ERR_INVALID_ARG, "cgsr_get_stats: NULL argument");
  hipStream_t stream = (hipStream_t)stream_;
  cgsr_status s = set_device(st);
  if (s) return s;
  std::memset(out, 0, sizeof(*out));
  out->pair_capacity = st->cap_tile_pairs;
  out->n_views = st->n_views;
  if (!st->have_forward) return CGSR_OK;
  unsigned long long host[6];
  launch_clear_u32(reinterpret_cast<uint32_t*>(st->stats_dev), 12, stream);
  launch_stats(st->tiles, st->records, st->pixel_state, st->pixel_count, st->total_pixels, st->ranges,
               st->total_tiles, st->stats_dev, stream);
  HIP_TRY(hipMemcpyAsync(st->counters_pinned, st->counters, sizeof(uint32_t) * kCounterWords,
                         hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(host, st->stats_dev, sizeof(host), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  out->pairs = (int64_t)host[4];
  out->overflow = (int32_t)st->counters_pinned[kCntOverflow];
  // the last render's fullest tile, or the most any tile needed since the
  // last check if that overflowed
  out->peak_pairs = std::max<int64_t>((int64_t)host[5], st->counters_pinned[kCntPeak]);
  out->visible = (int64_t)host[0];
  out->processed = st->counted ? (int64_t)host[1] : -1;
  out->blended = st->counted ? (int64_t)host[2] : -1;
  out->walked = st->counted ? (int64_t)host[3] : -1;
  return CGSR_OK;
}

cgsr_status cgsr_get_timings(cgsr_state* st, float* ms_out) {
  if (!st || !ms_out) return fail(CGSR_ERR_INVALID_ARG, "cgsr_get_timings: NULL argument");
  if (!st->settings.timing) return fail(CGSR_ERR_STATE, "cgsr_get_timings: timing is off for this state");
  if (!st->fwd_timed || !st->bwd_timed)
    return fail(CGSR_ERR_STATE, "cgsr_get_timings: no timed render and backward since timing was enabled");
  cgsr_status s = set_device(st);
  if (s) return s;
  HIP_TRY(hipEventSynchronize(st->ev_fwd[CGSR_STAGE_BLEND_FWD + 1]));
  HIP_TRY(hipEventSynchronize(st->ev_bwd[2]));
  for (int k = 0; k <= CGSR_STAGE_BLEND_FWD; ++k)
    HIP_TRY(hipEventElapsedTime(&ms_out[k], st->ev_fwd[k], st->ev_fwd[k + 1]));
  HIP_TRY(hipEventElapsedTime(&ms_out[CGSR_STAGE_BLEND_BWD], st->ev_bwd[0], st->ev_bwd[1]));
  HIP_TRY(hipEventElapsedTime(&ms_out[CGSR_STAGE_PROJECT_BWD], st->ev_bwd[1], st->ev_bwd[2]));
  return CGSR_OK;
}

cgsr_status cgsr_debug_buffers(cgsr_state* st, const uint64_t** keys, const uint32_t** sorted_values,
                               const uint32_t** ranges, const float** records, const uint32_t** pixel_state) {
  if (!st) return fail(CGSR_ERR_INVALID_ARG, "state is NULL");
  if (!st->have_forward) return fail(CGSR_ERR_STATE, "no forward pass on this state");
  if (keys) *keys = st->keys[0];
  if (sorted_values) *sorted_values = st->sorted_vals;
  if (ranges) *ranges = reinterpret_cast<const uint32_t*>(st->ranges);
  if (records) *records = reinterpret_cast<const float*>(st->rec);
  if (pixel_state) *pixel_state = reinterpret_cast<const uint32_t*>(st->pixel_state);
  return CGSR_OK;
}

cgsr_status cgsr_debug_tile_order(cgsr_state* st, const uint32_t** order, int32_t* tiles, int32_t* kept) {
  if (!st) return fail(CGSR_ERR_INVALID_ARG, "state is NULL");
  if (!st->have_forward) return fail(CGSR_ERR_STATE, "no forward pass on this state");
  if (order) *order = st->order_ok ? st->tile_order : nullptr;
  if (tiles) *tiles = st->total_tiles;
  if (kept) *kept = st->order_ok && st->track_order_ok ? 1 : 0;
  return CGSR_OK;
}

const char* cgsr_last_error(void) { return g_last_error.c_str(); }

const char* cgsr_version(void) { return "cgsr 0.2 (gfx950)"; }

}  // extern "C"
