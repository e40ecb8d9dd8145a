/*
 * cgsr -- a differentiable 3-D Gaussian rasterizer for the tracking and
 * mapping of CG-SLAM (Hu et al., "CG-SLAM: Efficient Dense RGB-D SLAM in a
 * Consistent Uncertainty-aware 3D Gaussian Field"), written for AMD Instinct
 * MI355X (gfx950).
 *
 * C ABI.  Every pointer argument documented as "device" is HIP device memory
 * owned by the caller; the library reads or writes it only during the call's
 * stream-ordered work and never frees or retains it past the next call on the
 * same state.  Every "host" pointer is read during the call only.  Streams
 * are hipStream_t values passed as void* (NULL = the null stream).
 *
 * Errors: every call returns a cgsr_status and never aborts; cgsr_last_error()
 * returns a message for the calling thread's last failure.  Argument checks are
 * done on the host before any work is enqueued, so a failed call enqueues
 * nothing.  Device-side capacity overflow of the per-tile pair buckets is
 * reported by cgsr_state_check() (which synchronises the stream).
 *
 * Conventions shared by every entry point:
 *  - Gaussians are SoA float32: means[n][3], log_scales[n][3] (scale = exp),
 *    quats[n][4] as (w, x, y, z), normalised inside the forward pass,
 *    opacity_logits[n] (opacity = sigmoid), rgb[n][3]  (Sec. 3.1, Eq. 1), or,
 *    for view-dependent colour, sh[n][K][3] spherical-harmonic coefficients
 *    (K = (sh_degree + 1)^2, see cgsr_gaussians).
 *  - A pose is float32[12] in device memory: a row-major 3x3 rotation followed
 *    by a translation, mapping world points into the camera frame (x right,
 *    y down, z forward).
 *  - Pixel (u, v) has its centre at (u, v).
 *  - Images are planar float32: colour [3][H][W], every other map [H][W].
 *  - Pose gradients are the left se(3) perturbation T <- exp(xi^) T at xi = 0,
 *    xi = (rho, phi): translation part first, then rotation (Sec. 3.4 optimises
 *    the pose in its Lie algebra).
 *  - Gradients are accumulated (+=) into caller-zeroed buffers.
 */
#ifndef CGSR_H
#define CGSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CGSR_OK = 0,
    CGSR_ERR_INVALID_ARG = -1, /* bad pointer, size or combination of arguments */
    CGSR_ERR_OOM = -2,         /* device or host allocation failed             */
    CGSR_ERR_HIP = -3,         /* a HIP runtime call failed                    */
    CGSR_ERR_CAPACITY = -4,    /* more (tile, Gaussian) pairs than reserved    */
    CGSR_ERR_STATE = -5        /* backward without a matching forward, etc.    */
} cgsr_status;

/* Pinhole intrinsics of one view (host memory). */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
} cgsr_camera;

/* Gaussian parameters (device pointers, SoA float32, layouts above).
 * Colour (Sec. 3.1 gives each Gaussian spherical-harmonic coefficients for a
 * view-dependent radiance): with sh NULL the colour is rgb.  With sh
 * non-NULL, sh_degree in 0 .. 3, rgb is unused (may be NULL) and the colour
 * of Gaussian i in a view whose camera centre is C = -R^T t is, per channel c,
 *     max(0, sum_k sh[i][k][c] Y_k(d) + 1/2),   d = (X_i - C) / |X_i - C|,
 * Y_k the real spherical harmonics with the Condon-Shortley phase, ordered
 * k = l^2 + l + m (l = 0 .. sh_degree, m = -l .. l), d = (x, y, z) with z as
 * the polar axis -- the convention of the splatting rasterizer the paper
 * builds on, so its coefficients load unchanged.  The colour then depends on
 * the pose through C: pose gradients include that term. */
#define CGSR_MAX_SH_DEGREE 3
typedef struct {
    int64_t n;
    const float *means, *log_scales, *quats, *opacity_logits, *rgb;
    const float *sh;       /* NULL or [n][(sh_degree + 1)^2][3] */
    int32_t sh_degree;
} cgsr_gaussians;

/* Rendered maps of one view (device pointers; NULL = not written).
 *   color        [3][H][W]  alpha-blended colour,          Eq. 3
 *   depth        [H][W]     alpha-blended depth,           Eq. 6
 *   opacity      [H][W]     accumulated opacity,           Eq. 9
 *   depth_median [H][W]     depth of the median Gaussian,  Eq. 7-8 (0 if T never falls below 0.5)
 *   uncertainty  [H][W]     sum alpha T (d - D)^2,         Eq. 10 (needs the sensor depth D) */
typedef struct {
    float *color, *depth, *opacity, *depth_median, *uncertainty;
} cgsr_images;

/* Upstream gradients of one view, same layouts (device; NULL = zero). */
typedef struct {
    const float *color, *depth, *opacity, *depth_median, *uncertainty;
} cgsr_image_grads;

/* Gradient outputs for the Gaussian parameters (device, +=).  All NULL (or
 * the struct pointer NULL) selects the pose-only backward used by tracking.
 * sh receives the coefficient gradients (layout of cgsr_gaussians.sh) when
 * the rendered Gaussians carry sh; rgb is then not written. */
typedef struct {
    float *means, *log_scales, *quats, *opacity_logits, *rgb;
    float *sh;
} cgsr_gaussian_grads;

/* Library settings; cgsr_default_settings() fills the defaults. */
typedef struct {
    int32_t sync_capacity;   /* 1: render reads its fullest tile back and grows
                                the per-tile pair buckets as needed (one host
                                sync per render), except while its stream is
                                being captured into a graph.  0: never syncs; the
                                buckets must be large enough, see
                                cgsr_state_reserve().                            */
    int32_t timing;          /* 1: time every stage with HIP events on the call's
                                stream (not while it is being captured); read
                                the durations with cgsr_get_timings()            */
    int32_t fwd_pixels_per_lane; /* 1, 2 or 4 pixels per lane in the forward blend:
                                a 16x16 tile then takes 256 / that many lanes   */
    int32_t bwd_pixels_per_lane; /* same for the backward blend; each lane sums its
                                pixels before the per-Gaussian wave reduction   */
    int32_t count_work;      /* 1: tracking steps and renders keep the
                                per-pixel work counts that cgsr_get_stats
                                reports (processed, blended, walked).  0: they
                                skip that bookkeeping and cgsr_get_stats reports
                                -1 for them (renders with nu and tracking steps
                                without a pose update or gradient count anyway) */
} cgsr_settings;

typedef struct {
    int64_t visible;         /* (view, Gaussian) records that reach the image   */
    int64_t pairs;           /* (tile, Gaussian) pairs of the last render: the
                                tiles a Gaussian's binning rectangle overlaps,
                                less those where its alpha stays below 1/255
                                at every pixel (not emitted)                     */
    int64_t pair_capacity;   /* pairs one tile's bucket holds                    */
    int32_t overflow;        /* 1 if a render since the last cgsr_state_check
                                had a tile needing more than its bucket          */
    int32_t n_views;
    int64_t processed;       /* (pixel, list entry) alpha evaluations of the
                                forward blend, summed over pixels; a pixel's list
                                holds the Gaussians whose binning rectangle
                                reaches its 8x8 pixel cell and whose alpha can
                                reach 1/255 there                                */
    int64_t blended;         /* (pixel, Gaussian) pairs actually blended          */
    int64_t walked;          /* (pixel, list entry) pairs up to each pixel's last
                                blended Gaussian: what the backward revisits.
                                processed, blended and walked are -1 after a
                                render or tracking step with count_work 0     */
    int64_t peak_pairs;      /* pairs of the last render's fullest tile, or, if a
                                render since the last cgsr_state_check
                                overflowed, the most any tile needed there      */
} cgsr_stats;

/* Stages timed when cgsr_settings.timing is set. */
typedef enum {
    CGSR_STAGE_PROJECT = 0,     /* EWA projection and the (depth, record) keys
                                   into the tile buckets                      */
    CGSR_STAGE_EMIT = 1,        /* empty: the projection emits the keys       */
    CGSR_STAGE_SORT = 2,        /* per-tile depth sort and tile ranges        */
    CGSR_STAGE_BLEND_FWD = 3,   /* front-to-back blend                        */
    CGSR_STAGE_BLEND_BWD = 4,   /* back-to-front blend backward               */
    CGSR_STAGE_PROJECT_BWD = 5, /* projection backward and pose reduction     */
    CGSR_NUM_STAGES = 6
} cgsr_stage;

typedef struct cgsr_state cgsr_state;

/* Default settings. */
void cgsr_default_settings(cgsr_settings *s);

/* A state holds one forward pass's workspace and saved values: projected
 * records, sort buffers, tile ranges and per-pixel transmittance.  It is
 * bound to the device current at creation.  One state serves one stream at a
 * time; a backward consumes the state of the forward that preceded it. */
cgsr_status cgsr_state_create(const cgsr_settings *s /* NULL = defaults */, cgsr_state **out);
cgsr_status cgsr_state_destroy(cgsr_state *st);

/* Grow the workspace for up to max_records (views x Gaussians), max_pixels
 * (summed over views), max_tiles (summed over views) and max_tile_pairs
 * (the (tile, Gaussian) pairs of one tile: every tile gets a bucket of that
 * many, so max_tiles x max_tile_pairs must stay below 2^32); never
 * shrinks.  Allocation happens here, so a render whose sizes fit does not
 * allocate and can be captured into a HIP graph.  A captured graph reads the
 * table of cameras and image pointers the state holds when it replays; a call
 * on the same state with other cameras or images rewrites that table, so
 * replay after a call with the graph's own cameras and images, or keep one
 * state per captured loop (a replay with another table is reported by
 * cgsr_state_check).  Growing the workspace frees the buffers a graph
 * captured before then points to: such a graph must not be replayed. */
cgsr_status cgsr_state_reserve(cgsr_state *st, int64_t max_records, int64_t max_pixels,
                               int64_t max_tiles, int64_t max_tile_pairs);

/*
 * Forward render of n_views views of one Gaussian set (Sec. 3.1: EWA projection,
 * Eq. 2; depth pre-sort; front-to-back alpha blending, Eq. 3-9; uncertainty,
 * Eq. 10).  All views share one projection launch, one tile sort and one blend
 * launch.
 *   g          Gaussian parameters (device).
 *   n_views    1 .. CGSR_MAX_VIEWS.
 *   poses      device float[n_views][12].
 *   cams       host cgsr_camera[n_views].
 *   depth_obs  host array of n_views device pointers to [H][W] sensor depth,
 *              or NULL; entry v required iff outs[v].uncertainty != NULL.
 *   outs       host array of n_views cgsr_images.
 * The state records the argument pointers for the backward pass: the caller
 * keeps g, poses and depth_obs unchanged and alive until then.
 */
#define CGSR_MAX_VIEWS 64
cgsr_status cgsr_render(cgsr_state *st, const cgsr_gaussians *g, int32_t n_views, const float *poses,
                        const cgsr_camera *cams, const float *const *depth_obs,
                        const cgsr_images *outs, void *stream);

/*
 * cgsr_render plus the per-Gaussian depth uncertainty of Sec. 3.2, Eq. 13,
 * taken in the same blend pass.  A pixel is "dominated" by its blended
 * Gaussian of largest weight w = alpha T (the first of equal maxima in depth
 * order).  For every pixel with a blended Gaussian and a sensor depth D > 0
 * (D <= 0 marks a missing measurement), the dominating Gaussian i receives
 * w (D - d_i)^2 into nu_sum[i] and 1 into nu_count[i], d_i being its camera
 * depth in that view.  Rendering the k keyframes of a window, in one call or
 * several, accumulates the numerator and the denominator M_1 + ... + M_k of
 * Eq. 13; cgsr_nu_prune forms nu.
 *   depth_obs  required: a sensor depth map for every view.
 *   dominant   host array of n_views device int32[H][W] maps (each may be
 *              NULL) receiving the dominating Gaussian's index or -1; or NULL.
 *   nu_sum     device float[n] (+=), nu_count device uint32[n] (+=); both or
 *              neither.  The caller clears them at the start of a window.
 * Other arguments, the saved state and cgsr_backward as for cgsr_render.
 * The sums use float atomics, so their rounding depends on the order.
 */
cgsr_status cgsr_render_nu(cgsr_state *st, const cgsr_gaussians *g, int32_t n_views, const float *poses,
                           const cgsr_camera *cams, const float *const *depth_obs, const cgsr_images *outs,
                           int32_t *const *dominant, float *nu_sum, uint32_t *nu_count, void *stream);

/* Weights of the mapping objective, Eq. 18 (omega_1 .. omega_6), and the
 * anisotropy level epsilon of Eq. 17.  Sec. 4 uses {0.7, 0.1, 0.25, 0.25,
 * 0.1, 0.15} on Replica and {1.0, 0.1, 0.8, 0.5, 0.1, 0.5} on TUM and
 * ScanNet, epsilon = 1.0 (Sec. 3.3). */
typedef struct {
    float color, ssim, geo, align, iso, var;
    float iso_epsilon;
} cgsr_mapping_weights;

/*
 * Gradient images of the mapping objective, Eq. 18, for the views of the
 * last cgsr_render / cgsr_render_nu on this state, and the gradient of its
 * isotropy term with respect to the log-scales:
 *   color  L_color = mean over pixels of the L1 over RGB          (Eq. 14)
 *   ssim   L_ssim  = 1 - SSIM(I^, I): 11x11 Gaussian window of standard
 *          deviation 1.5, zero padding, C1 = 0.01^2, C2 = 0.03^2, mean over
 *          channels and pixels (the splatting conventions)         (Eq. 15)
 *   geo    L_geo   = mean |D^ - D|                                 (Eq. 16)
 *   align  L_align = mean |D^ - D^_median| over pixels that have a median
 *          Gaussian (median depth > 0), divided by H W            (Eq. 12)
 *   iso    L_iso   = mean over the view's visible Gaussians of
 *          max(max s / min s, epsilon) - epsilon                  (Eq. 17)
 *   var    L_var   = mean |U|                                      (Eq. 11)
 * The objective of a window is the sum over its views.
 *   maps          host array of n_views rendered maps (device; the render's
 *                 outputs): colour for colour/SSIM, depth for geo/align,
 *                 depth_median for align, uncertainty for var.
 *   target_color  host array of n_views device [3][H][W] (or NULL if unused);
 *   target_depth  host array of n_views device [H][W] (or NULL if unused).
 *   dimgs         host array of n_views gradient outputs (device, overwritten,
 *                 opacity unused): color, depth, depth_median, uncertainty.
 *                 Each term with a non-zero weight needs its outputs; each
 *                 given output needs the maps and targets of its terms.
 *                 They are the upstream gradients cgsr_backward then takes.
 *   dlog_scales   device float[n][3] (+=) gradient of the isotropy term, or
 *                 NULL.
 *   loss          device float[n_views] (+=) per-view objective, or NULL.
 * The Gaussians are the ones the state's last render read.  The first call
 * with SSIM allocates its scratch (9 floats per pixel of the largest view);
 * under graph capture that allocation is an error (CGSR_ERR_STATE).
 */
cgsr_status cgsr_mapping_objective(cgsr_state *st, const cgsr_mapping_weights *w, const cgsr_images *maps,
                                   const float *const *target_color, const float *const *target_depth,
                                   const cgsr_images *dimgs, float *dlog_scales, float *loss, void *stream);

/*
 * Per-Gaussian uncertainty and pruning (Sec. 3.2, Eq. 13): for i < n,
 * nu_i = nu_sum[i] / nu_count[i], or 0 when the Gaussian dominated no pixel
 * (no evidence).  Gaussians with nu_i > tau (the paper uses 0.025) have their
 * opacity lowered to low_opacity: opacity_logits[i] = min(opacity_logits[i],
 * logit(low_opacity)), never raised, so they can still recover or be removed
 * by later optimisation.  Optional outputs (device, may be NULL): nu [n]
 * (overwritten), n_pruned (a uint32 counter, += number of Gaussians over tau).
 * opacity_logits (device, in place) may be NULL to only evaluate nu.
 * Errors: n < 0, missing accumulators, tau < 0, low_opacity outside (0, 1).
 */
cgsr_status cgsr_nu_prune(int64_t n, const float *nu_sum, const uint32_t *nu_count, float tau,
                          float low_opacity, float *opacity_logits, float *nu, uint32_t *n_pruned,
                          void *stream);

/*
 * Backward of the last cgsr_render (or cgsr_render_nu) on this state: chain rule of Eq. 2-10 to
 * every Gaussian parameter (accumulated over views) and to each view's pose.
 *   dimgs   host array of n_views upstream gradients (device maps; NULL fields
 *           are zero).  An uncertainty gradient needs that view's sensor depth.
 *   dG      Gaussian gradients (device, +=), NULL or all-NULL for pose only.
 *   dposes  device float[n_views][6] (+=), or NULL to skip pose gradients.
 */
cgsr_status cgsr_backward(cgsr_state *st, const cgsr_image_grads *dimgs, const cgsr_gaussian_grads *dG,
                          float *dposes, void *stream);

/*
 * Gradient images of the tracking objective (Eq. 19):
 *   L = lambda_color * L_color (Eq. 14) + lambda_depth * L_geo (Eq. 16),
 * with L_color the mean over the H*W pixels of the L1 norm over RGB and L_geo
 * the mean absolute depth error.  Writes dL/dcolor [3][H][W] and dL/ddepth
 * [H][W] (device, overwritten) and adds L to *loss (device float, +=) if loss
 * is non-NULL.  The subgradient of |x| at 0 is 0.
 */
cgsr_status cgsr_tracking_loss_grad(int32_t width, int32_t height, const float *color,
                                    const float *depth, const float *target_color,
                                    const float *target_depth, float lambda_color,
                                    float lambda_depth, float *dcolor, float *ddepth, float *loss,
                                    void *stream);

/*
 * Gradient images of the mapping objective of the 1200x680 workload:
 *   L = L_color (Eq. 14) + mean_n U_n |D^_n - D_n|
 * (Eq. 16's depth error weighted per pixel by the rendered uncertainty U of
 * Eq. 10; the gradient flows through both factors).  Writes dL/dcolor
 * [3][H][W], dL/ddepth and dL/duncertainty [H][W] (device, overwritten) and
 * adds L to *loss (device float) if loss is non-NULL.
 */
cgsr_status cgsr_mapping_loss_grad(int32_t width, int32_t height, const float *color, const float *depth,
                                   const float *uncertainty, const float *target_color,
                                   const float *target_depth, float *dcolor, float *ddepth,
                                   float *duncertainty, float *loss, void *stream);

/* Adam hyper-parameters of the pose update; the paper uses learning rates
 * 0.0015 for the rotation (so(3)) part and 0.00215 for the translation part
 * (Sec. 4, Implementation Details).  beta1, beta2, eps as in Adam. */
typedef struct {
    float lr_rho, lr_phi, beta1, beta2, eps;
} cgsr_adam_params;

/*
 * One Adam step on each view's pose in its tangent space, then the left
 * retraction T <- exp(delta^) T (Sec. 3.4, Eq. 20; Adam with bias correction).
 *   poses      device float[n_views][12], updated in place.
 *   dposes     device float[n_views][6], read then zeroed.
 *   adam       device float[n_views][16]: m[6], v[6], step count,
 *              1 - beta1^step, 1 - beta2^step, 1 unused; zero-initialise
 *              before the first step.
 */
cgsr_status cgsr_pose_adam_step(int32_t n_views, float *poses, float *dposes, float *adam,
                                const cgsr_adam_params *params, void *stream);

/* Learning rates and Adam constants of cgsr_gaussian_adam_step.  The paper
 * defers the mapping learning rates to its supplementary material, so they
 * are the caller's choice. */
typedef struct {
    float lr_means, lr_log_scales, lr_quats, lr_opacity_logits, lr_rgb;
    float beta1, beta2, eps;
    float lr_sh_rest;      /* spherical-harmonic coefficients of degree >= 1 */
    int32_t sh_degree;     /* degree of params->sh / grads->sh when they are set */
} cgsr_gaussian_adam_params;

/*
 * One Adam step (with bias correction) on every Gaussian parameter: the
 * parameter half of the sliding-window bundle adjustment of Eq. 21, whose
 * pose half is cgsr_pose_adam_step.
 *   n        number of Gaussians.
 *   params   the parameter arrays (device, float, updated in place), in the
 *            layouts of cgsr_gaussians.  With params->sh set (and grads->sh),
 *            the colour group is sh, of hp->sh_degree, instead of rgb:
 *            lr_rgb then applies to its degree-0 coefficients and
 *            lr_sh_rest to the others.
 *   grads    their gradients (device; read, then zeroed for the next
 *            accumulation by cgsr_backward and cgsr_mapping_objective).
 *   moments  device float[2][(11 + W) n]: first then second moments, each the
 *            concatenation of the groups means (3n), log_scales (3n), quats
 *            (4n), opacity_logits (n) and colour (W n: W = 3 for rgb,
 *            3 (sh_degree + 1)^2 for sh); zero-initialise.
 *   step     device uint32 step counter (zero-initialise); the call reads it
 *            for the bias correction and then increments it, on the stream, so
 *            a captured loop keeps counting.
 * Errors: NULL arrays (n > 0), negative learning rates, betas outside [0, 1),
 * eps <= 0, sh on one side only, sh_degree outside 0 .. 3.
 */
cgsr_status cgsr_gaussian_adam_step(int64_t n, const cgsr_gaussian_grads *params, const cgsr_gaussian_grads *grads,
                                    float *moments, uint32_t *step, const cgsr_gaussian_adam_params *hp,
                                    void *stream);

/*
 * One sequential-tracking iteration (Sec. 3.4, Eq. 19-20) of n_views
 * independent frames in one launch sequence: render; the gradient images of
 *   L = lambda_color * L_color (Eq. 14) + lambda_depth * L_geo (Eq. 16)
 * formed inside the blend from the blended values (no maps are written);
 * pose-only backward; then, if adam is non-NULL, an Adam step with left
 * retraction of every pose.
 *   poses         device float[n_views][12]; updated in place when adam != NULL.
 *   target_color  host array of n_views device pointers to [3][H][W].
 *   target_depth  host array of n_views device pointers to [H][W].
 *   dposes        device float[n_views][6] (+= the pose gradient) or NULL.
 *   adam          device float[n_views][16] Adam state (as for
 *                 cgsr_pose_adam_step) or NULL; params required with it.
 *   loss          device float[n_views] (+= each frame's L) or NULL.
 * The state is left as after a render; cgsr_backward on it is an error.
 */
cgsr_status cgsr_tracking_step(cgsr_state *st, const cgsr_gaussians *g, int32_t n_views, float *poses,
                               const cgsr_camera *cams, const float *const *target_color,
                               const float *const *target_depth, float lambda_color, float lambda_depth,
                               float *dposes, float *adam, const cgsr_adam_params *adam_params,
                               float *loss, void *stream);

/*
 * Autotuner: picks the blend kernels' pixels per lane (1, 2 or 4; one value
 * for forward and backward, which the tracking step runs as one launch) for
 * a tracking workload on this state, as configured (work counts, bucket
 * capacity), by timing whole cgsr_tracking_step calls with each candidate:
 * one step with the state's settings (it may grow the buckets), then
 * `repeats` steps without the capacity read-back between two HIP events on
 * the stream (no Adam step, poses unchanged).  A candidate whose buckets
 * exceed one key per lane is timed with the segmented sort it then needs.
 * The candidates are timed in two passes and each keeps its faster one (the
 * first pass also warms the GPU up).  Stores the fastest in the state's
 * settings and returns them in *out (may be NULL).  Synchronises; not for use
 * under graph capture.
 */
cgsr_status cgsr_autotune_tracking(cgsr_state *st, const cgsr_gaussians *g, int32_t n_views, const float *poses,
                                   const cgsr_camera *cams, const float *const *target_color,
                                   const float *const *target_depth, int32_t repeats, cgsr_settings *out,
                                   void *stream);

/*
 * Autotuner of the mapping iteration's blends (Eq. 3-10 and their backward,
 * the batched window of Eq. 21): picks the forward and the backward blend's
 * pixels per lane (1, 2 or 4 each) for a render + backward workload on this
 * state by timing, for each of the nine pairs, one cgsr_render + cgsr_backward
 * with the state's settings (it may grow the buckets), then `repeats` more
 * between two HIP events on the stream without the capacity read-back, in
 * two passes over the pairs, each pair keeping its faster one.  The
 * arguments are those of cgsr_render and cgsr_backward.  The tuning runs
 * write the maps and add their gradients to dG and dposes 18 (repeats + 1)
 * times: the caller clears those after.
 *
 * Both autotuners keep their picks in the state, keyed by the workload's
 * shape (Gaussian count, SH degree, view count and sizes, and which outputs
 * and gradients are asked for; for tracking also the bucket size and work
 * counts): a later call with the same shape applies the kept pick without
 * timing.  The pick is stored in the state's settings and returned in *out
 * (may be NULL).  Synchronises; not for use under graph capture.
 */
cgsr_status cgsr_autotune_render(cgsr_state *st, const cgsr_gaussians *g, int32_t n_views, const float *poses,
                                 const cgsr_camera *cams, const float *const *depth_obs, const cgsr_images *outs,
                                 const cgsr_image_grads *dimgs, const cgsr_gaussian_grads *dG, float *dposes,
                                 int32_t repeats, cgsr_settings *out, void *stream);

/*
 * Gaussian management (Sec. 3.3).  The set is grown by spawning and
 * densification and shrunk by compaction; each call writes a new set (or
 * appends to one) in caller-owned arrays and returns the new count on the
 * host, so it synchronises the stream.  Orders are deterministic.
 *
 * Writable parameter arrays of a set (device float, layouts of
 * cgsr_gaussians): colour in rgb, or in sh (then rgb unused) with
 * sh_degree as in cgsr_gaussians.
 */
typedef struct {
    float *means, *log_scales, *quats, *opacity_logits, *rgb, *sh;
    int32_t sh_degree;
} cgsr_gaussian_arrays;

/* Rendered-opacity threshold below which a pixel is unobserved (Sec. 3.3). */
#define CGSR_SPAWN_PSI 0.5f

/*
 * Spawning (Sec. 3.3): new Gaussians from the pixels of one RGB-D view whose
 * rendered opacity (Eq. 9) is below psi and whose sensor depth D is
 * positive, appended at indices n, n + 1, ... in row-major pixel order.
 * With opacity NULL every pixel with a depth spawns (the dense
 * initialisation from the first frame).  stride >= 1 takes the pixels with
 * u and v multiples of stride only.  A new Gaussian (readings where the
 * paper is silent): mean = the back-projection of the pixel centre at depth
 * D through the pose, T^-1 (D K^-1 (u, v, 1)); isotropic scale
 * D / ((fx + fy) / 2) (one pixel at that depth); identity rotation;
 * opacity logit init_logit; colour = the pixel's colour (with sh: the
 * degree-0 coefficient (c - 1/2) sqrt(4 pi), the others zero).
 *   dst       the set's arrays, holding n Gaussians and room for capacity.
 *   cam       host camera of the view; pose device float[12] (world -> camera).
 *   color     device [3][H][W]; depth device [H][W]; opacity device [H][W] or NULL.
 *   n_out     host: n + the number spawned.  If that exceeds capacity, only
 *             the first capacity - n are written and CGSR_ERR_CAPACITY is
 *             returned with n_out still the full count.
 */
cgsr_status cgsr_spawn_gaussians(const cgsr_gaussian_arrays *dst, int64_t n, int64_t capacity,
                                 const cgsr_camera *cam, const float *pose, const float *color,
                                 const float *depth, const float *opacity, float psi, int32_t stride,
                                 float init_logit, int64_t *n_out, void *stream);

/*
 * Removal: writes the Gaussians i < n with keep[i] != 0 (device uint8[n]),
 * in order, to dst (which must not overlap src), and *n_out (host) = their
 * number.  n_extra (<= 12) further per-Gaussian float arrays extra_src[e]
 * of extra_width[e] floats per Gaussian (say Adam moments or uncertainty
 * sums; host arrays of device pointers and widths) are compacted the same
 * way into extra_dst[e].
 */
cgsr_status cgsr_compact_gaussians(int64_t n, const uint8_t *keep, const cgsr_gaussian_arrays *src,
                                   const cgsr_gaussian_arrays *dst, int32_t n_extra,
                                   const float *const *extra_src, float *const *extra_dst,
                                   const int32_t *extra_width, int64_t *n_out, void *stream);

/* Most Gaussians cgsr_compact_gaussians_noalloc takes (2^26). */
#define CGSR_COMPACT_NOALLOC_MAX_N 67108864

/*
 * cgsr_compact_gaussians for callers that cannot allocate device memory
 * (serving loops and harnesses that forbid hipMalloc): the same arguments,
 * result, ordering and errors, but the call allocates nothing.  Its
 * counters (one per 1024 Gaussians, 256 KB) live in a fixed array of the
 * library, one copy per GPU, held until the process ends; each call
 * rewrites the counters it reads before reading them.
 *   n   0 .. CGSR_COMPACT_NOALLOC_MAX_N; larger n is CGSR_ERR_INVALID_ARG
 *       (use cgsr_compact_gaussians).
 * Calls that overlap on one GPU (from several host threads, or on streams
 * not ordered with each other) share that array and race: serialise them.
 * Like cgsr_compact_gaussians it synchronises the stream to return *n_out.
 */
cgsr_status cgsr_compact_gaussians_noalloc(int64_t n, const uint8_t *keep, const cgsr_gaussian_arrays *src,
                                           const cgsr_gaussian_arrays *dst, int32_t n_extra,
                                           const float *const *extra_src, float *const *extra_dst,
                                           const int32_t *extra_width, int64_t *n_out, void *stream);

/*
 * Densification statistic (Sec. 3.3 keeps the densification of splatting):
 * from now on every cgsr_backward on this state adds, for each (view,
 * Gaussian) record that reaches the image, |dL/dmu| (the gradient of the
 * loss with respect to the Gaussian's projected mean, in pixels) to
 * grad_accum[i] and 1 to count[i] (device float[n] and uint32[n], caller
 * cleared).  NULL pointers stop the accumulation.
 */
cgsr_status cgsr_set_densify_stats(cgsr_state *st, float *grad_accum, uint32_t *count);

/*
 * Densification: with stat_i = grad_accum[i] / count[i] (0 if count is 0),
 * Gaussian i with stat_i >= grad_threshold is cloned when its largest scale
 * is at most dense_scale and split otherwise.  A clone is an exact copy; a
 * split replaces the Gaussian by two at mu + R diag(s) z_k (k = 0, 1; z the
 * caller's standard normal draws normals[i][k][3], device float[n][2][3])
 * with scales s / 1.6 and the other parameters copied.  dst (not
 * overlapping src) receives the Gaussians that were not split, in order,
 * then the clones in index order, then the split halves in index order (k
 * = 0 first); *n_out (host) = their number.  If it exceeds capacity only the
 * first capacity are written and CGSR_ERR_CAPACITY is returned.
 */
cgsr_status cgsr_densify_gaussians(int64_t n, const float *grad_accum, const uint32_t *count,
                                   float grad_threshold, float dense_scale, const float *normals,
                                   const cgsr_gaussian_arrays *src, const cgsr_gaussian_arrays *dst,
                                   int64_t capacity, int64_t *n_out, void *stream);

/* Synchronise the stream and report CGSR_ERR_CAPACITY if any render on this
 * state since the previous check (or since creation) overflowed its pair
 * buffer; the message names the most pairs a render needed.  CGSR_ERR_STATE
 * (reported first) if a launch since the previous check ran with a table of
 * cameras and image pointers other than the one it was set up with: a graph
 * captured on this state and replayed after a call with other cameras or
 * images (see cgsr_state_reserve); that replay's results are not the captured
 * loop's.  The check then starts a new period (clears both flags and the
 * peak). */
cgsr_status cgsr_state_check(cgsr_state *st, void *stream);

/* Synchronise the stream and read the counters of the last render. */
cgsr_status cgsr_get_stats(cgsr_state *st, void *stream, cgsr_stats *out);

/* Durations in milliseconds of the stages of the last timed render (stages
 * 0-3) and backward (stages 4-5) on this state; ms_out[CGSR_NUM_STAGES].
 * Synchronises on the recorded events.  CGSR_ERR_STATE if timing is off or a
 * stage has not run since timing was enabled. */
cgsr_status cgsr_get_timings(cgsr_state *st, float *ms_out);

/*
 * Measurement: re-runs the fused blend kernel of the last cgsr_tracking_step
 * on st (the one with dposes or adam) reps times back to back between two
 * HIP events on stream, and writes the average duration of one launch in
 * milliseconds to *ms_out.  Every re-run is the same kernel instantiation and
 * launch shape on the same tile buckets, pixels and targets as that step;
 * the step's loss sum (if any) is not added to again.  The state is left as
 * the step left it (pair counters reset, record gradient sums cleared), so
 * it may be called repeatedly and the next call on st proceeds as usual.
 *   reps   1 .. 100000.
 * CGSR_ERR_STATE if another call changed the state since that step, or under
 * graph capture.  Synchronises the stream.
 */
cgsr_status cgsr_time_tracking_blend(cgsr_state *st, int32_t reps, void *stream, float *ms_out);

/* Debug views of the last render (device buffers owned by the state; valid
 * until the next render on it).  keys: [tiles][pair_capacity] each tile's
 * bucket of emitted keys, depth bits << 32 | record id (overwritten by the
 * sort for buckets longer than 4096); sorted_values: [tiles][pair_capacity]
 * record ids of each tile in (depth, record id) order; ranges: [tiles][2]
 * start/end into sorted_values; records: [records][12] float32 projected
 * record (mu_x, mu_y, a, k, c', opacity, depth, r, g, b, mu_x lo, mu_y lo):
 * the mean is mu + lo, and the conic (a, b, c) of Eq. 5 is kept in the
 * completed-square form a (dx + k dy)^2 + c' dy^2 with k = b / a and
 * c' = c - b^2 / a;
 * pixel_state: [pixels][4] (final T as float bits, tile-list entries up to
 * the last blended one, median position in the tile list or -1, alpha
 * evaluations: entries of the pixel's 8x8-cell list walked). */
cgsr_status cgsr_debug_buffers(cgsr_state *st, const uint64_t **keys, const uint32_t **sorted_values,
                               const uint32_t **ranges, const float **records, const uint32_t **pixel_state);

/* Debug view of the order in which the last render's blends took their
 * (view, tile) work items (a device buffer owned by the state, valid until
 * the next call on it).  *order: [*tiles] entries, the workgroup at position p
 * taking tile order[p] & 0x3FFFFFFF, longest list first (Sec. 3.1 leaves the
 * order free: every order gives each tile the same result), or NULL when the
 * blends took the tiles in their own order.  *kept: 1 when it is the order a
 * fused tracking step keeps from the work the previous step measured, whose
 * entries also carry in bits 30-31 the quadrant rotation of that tile's
 * workgroup, else 0.  Any output pointer may be NULL.  CGSR_ERR_STATE before
 * the first render. */
cgsr_status cgsr_debug_tile_order(cgsr_state *st, const uint32_t **order, int32_t *tiles, int32_t *kept);

/* Message of the calling thread's last failure ("" if none). */
const char *cgsr_last_error(void);

/* Library version string. */
const char *cgsr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CGSR_H */
