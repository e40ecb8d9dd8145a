/*
 * FP64 CPU oracle of the CG-SLAM differentiable Gaussian rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP library: it is a plain, slow restatement of the paper's equations.
 *
 * What it computes (paper, Sec. 3.1 and 3.2):
 *   Eq. 1   covariance from scale and rotation, Sigma = R S S^T R^T
 *   Eq. 2   EWA projection, Sigma2d = J W Sigma W^T J^T
 *   Eq. 3-5 front-to-back alpha blending of colour
 *   Eq. 6   alpha-blended depth, Eq. 7-8 median depth, Eq. 9 opacity
 *   Eq. 10  uncertainty map  U = sum_i alpha_i T_i (d_i - D)^2
 *   Eq. 13  per-Gaussian depth uncertainty from its dominated pixels
 *   Sec. 3.1 view-dependent colour from spherical-harmonic coefficients
 * plus the analytic gradient of all of them with respect to every Gaussian
 * parameter and to the left se(3) perturbation of the world->camera pose
 * (Sec. 3.4 names these pose derivatives; their derivation is restated from
 * first principles here), and a frozen-decision finite-difference probe that
 * pins that gradient.
 *
 * Layouts: every array is plain row-major double.  Gaussian i owns
 * means[3i..3i+2], log_scales[3i..], quats[4i..] (w,x,y,z), opacity_logits[i],
 * rgb[3i..], and optionally sh[(K i + k) 3 + c] (K = (sh_degree + 1)^2
 * coefficients k per colour channel c).  Images are planar: colour [3][H][W],
 * the others [H][W].
 * pose = {R[9] row-major, t[3]} maps world to camera (OpenCV axes).
 * cam  = {fx, fy, cx, cy}; pixel (u, v) has its centre at (u, v).
 */
#ifndef CGSR_ORACLE_H
#define CGSR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Readings of constants the paper leaves to the 3D Gaussian splatting
 * rasterizer it builds on.  Kept identical, by value, on the HIP side. */
#define ORC_NEAR_Z      0.2           /* cull if camera z <= this            */
#define ORC_TAN_CLAMP   1.3           /* J uses x/z clamped to 1.3 x half-FOV */
#define ORC_DILATION    0.3           /* added to the 2-D covariance diagonal */
#define ORC_ALPHA_MAX   0.99          /* alpha is capped here                 */
#define ORC_ALPHA_MIN   (1.0 / 255.0) /* alpha below this is skipped          */
#define ORC_T_STOP      1.0e-4        /* stop before T would drop below this  */
#define ORC_T_MEDIAN    0.5           /* Eq. 8 threshold                      */
/* Binning rectangle: squared Mahalanobis radius of the alpha >= 1/255 support,
 * widened by a relative and an absolute margin so a float32 alpha test can
 * never accept a pixel outside the rectangle. */
#define ORC_BIN_R2_REL  (1.0 + 1.0 / 128.0)
#define ORC_BIN_R2_ABS  (1.0 / 256.0)

/* View-dependent colour (Sec. 3.1 gives each Gaussian spherical-harmonic
 * coefficients; the reading of their convention is that of the splatting
 * rasterizer the paper builds on): with sh non-NULL, the colour of Gaussian i
 * seen from camera centre C = -R^T t is, per channel c,
 *     colour_c = max(0, sum_k sh[i][k][c] Y_k(d) + 1/2),  d = (X_i - C) / |X_i - C|,
 * where Y_k are the real spherical harmonics of degree l <= sh_degree with
 * the Condon-Shortley phase, ordered k = l^2 + l + m, m = -l .. l, at the
 * unit direction d = (x, y, z) (z the polar axis, azimuth atan2(y, x)); rgb
 * is then unused.  With sh NULL the colour is rgb. */
#define ORC_SH_MAX_DEGREE 3
#define ORC_SH_MAX_COEFFS 16

typedef struct {
    int64_t n;
    const double *means, *log_scales, *quats, *opacity_logits, *rgb;
    const double *sh;      /* NULL or [n][(sh_degree + 1)^2][3] */
    int32_t sh_degree;     /* 0 .. ORC_SH_MAX_DEGREE */
} orc_gaussians;

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
} orc_camera;

typedef struct {
    double R[9];
    double t[3];
} orc_pose;

/* Per-Gaussian projection, all outputs [n] or [n][k]. */
typedef struct {
    int32_t *visible;   /* [n]   1 if it can reach the image                     */
    int32_t *clamp;     /* [n][2] -1/0/+1: tangent limit applied in J (x, y)       */
    double *p_cam;      /* [n][3] camera-space mean                              */
    double *mu;         /* [n][2] pixel-space mean                               */
    double *cov2d;      /* [n][3] Sigma2d xx, xy, yy (dilated)                    */
    double *conic;      /* [n][3] inverse of Sigma2d: a, b, c                     */
    double *depth;      /* [n]                                                   */
    double *opacity;    /* [n]   sigmoid(logit)                                  */
    int32_t *rect;      /* [n][4] pixel bounds u0, u1, v0, v1 (inclusive), -1 if none */
    double *rect_edges; /* [n][4] unrounded mu -/+ extent in x then y            */
} orc_projection;

/* Rendered maps; NULL members are not written. */
typedef struct {
    double *color;         /* [3][H][W] Eq. 3   */
    double *depth;         /* [H][W]    Eq. 6   */
    double *opacity;       /* [H][W]    Eq. 9   */
    double *depth_median;  /* [H][W]    Eq. 7-8 */
    double *uncertainty;   /* [H][W]    Eq. 10 (needs depth_obs) */
    int32_t *n_contrib;    /* [H][W]    number of Gaussians blended */
    double *t_final;       /* [H][W]    transmittance after the last blended one */
    int32_t *median_id;    /* [H][W]    Gaussian index of the median, -1 if none */
    double *decision_margin; /* [H][W] smallest relative distance of any alpha
                                skip/cap, stop or median decision to its threshold */
    double *order_margin;    /* [H][W] smallest relative depth gap between two
                                consecutively blended Gaussians (a swap keeps
                                the blended set, so the opacity)           */
    double *stop_order_margin; /* [H][W] smallest relative depth gap between
                                the Gaussian that stops the walk and its two
                                neighbours in the walk (the last blended one
                                and the next one past the skip test): a swap
                                there changes which Gaussians are blended  */
} orc_images;

/* Upstream gradient images (dL/d maps); NULL members are zero. */
typedef struct {
    const double *color, *depth, *opacity, *depth_median, *uncertainty;
} orc_image_grads;

/* Gradients, accumulated with +=; NULL members are skipped. */
typedef struct {
    double *means, *log_scales, *quats, *opacity_logits, *rgb;
    double *pose;          /* [6] (rho, phi): left perturbation exp(xi^) T_cw */
    double *sh;            /* [n][K][3] when the Gaussians carry sh */
    /* gradients with respect to the projected quantities, [n][k] */
    double *mu, *conic, *opacity, *depth;
} orc_grads;

/* Projection of every Gaussian (Eq. 1-2). */
int orc_project(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                orc_projection *out);

/* Forward render.  candidates: 0 = every visible Gaussian at every pixel
 * (brute force), 1 = only Gaussians whose binning rectangle holds the pixel
 * (the rectangle bounds the alpha support, so the result is the same).
 * pixels: optional list of n_pixels flat pixel indices v*W+u to render; then
 * every image is [n_pixels] (colour [3][n_pixels]).  NULL renders all.
 * depth_obs: [H][W] sensor depth or NULL (then no uncertainty). */
int orc_render(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
               const double *depth_obs, int candidates, const int64_t *pixels,
               int64_t n_pixels, orc_images *out);

/* Every admissible result of listed pixels whose discrete decisions sit within
 * rounding of their thresholds (Eq. 3-5 skip and stop, Eq. 7-8 median, and
 * the blend order of Gaussians whose depths nearly tie).  A float32
 * implementation evaluating alpha, T and the depth order may take either
 * outcome of such a decision, so each one is a branch point here:
 *   - alpha skip: |alpha_raw - 1/255| < decision_margin * (1/255);
 *   - stop:       |T (1 - alpha) - 1e-4| < decision_margin * 1e-4;
 *   - median:     |T (1 - alpha) - 0.5| < decision_margin * 0.5 while no
 *                 median has been found;
 *   - order:      two Gaussians adjacent in the pixel's walk whose depths
 *                 differ by less than order_margin * depth may come in either
 *                 order.
 * Each branch continues the walk of orc_render with its outcome, and every
 * walk's end is one alternative.  Per pixel k (flat index pixels[k]) the
 * alternatives go to alts[k][a][ORC_ALT_VALUES] as (colour r, g, b, depth,
 * opacity, median depth, uncertainty (0 without depth_obs), final T), and
 * n_alts[k] = their number, or max_alts + 1 if the pixel has more (only the
 * first max_alts are written).  A pixel with no decision inside the margins
 * has exactly one alternative, orc_render's result.  Duplicates are kept.
 * Candidate mode as in orc_render. */
#define ORC_ALT_VALUES 8
int orc_render_alternatives(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                            const double *depth_obs, int candidates, const int64_t *pixels,
                            int64_t n_pixels, double decision_margin, double order_margin,
                            int32_t max_alts, double *alts, int32_t *n_alts);

/* Analytic backward of orc_render over the whole image. */
int orc_backward(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                 const double *depth_obs, int candidates, const orc_image_grads *dimg,
                 orc_grads *out);

/* Frozen-decision central differences of the linear probe
 *     L = sum over maps and pixels of dimg * map
 * at n_coords coordinates.  Every discontinuous decision (culling, tangent
 * clamp, skip, stop, alpha cap, median choice, blend order, colour clamp at
 * zero) is recorded at the unperturbed point and replayed at the perturbed
 * ones, so the result is the derivative of one smooth branch.  kind: 0 means,
 * 1 log_scales, 2 quats, 3 opacity_logits, 4 rgb, 5 pose, 6 sh (comp =
 * 3 k + c); index = Gaussian index (ignored for pose); comp = component.  Step h = rel_step * max(1, |theta|) (pose: rel_step). */
int orc_fd_linear(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                  const double *depth_obs, const orc_image_grads *dimg,
                  int64_t n_coords, const int32_t *kind, const int64_t *index,
                  const int32_t *comp, double rel_step, double *out);

/* Per-Gaussian depth uncertainty of Eq. 13, the contribution of one keyframe.
 * A pixel is "dominated" by the blended Gaussian of largest weight
 * w = alpha T (the first of equal maxima in depth order).  For every pixel
 * with at least one blended Gaussian and a positive sensor depth D (a
 * non-positive depth is a missing measurement and does not count), the
 * dominating Gaussian i receives w (D - d_i)^2 into nu_sum[i] and 1 into
 * nu_count[i]; both are accumulated (+=), so calling this once per keyframe
 * of a window gives the numerator and the denominator M_1 + ... + M_k of
 * Eq. 13.  Optional per-pixel outputs: dominant[H][W] = the dominating
 * Gaussian's index or -1, dominant_margin[H][W] = (w1 - w2) / w1 against the
 * runner-up weight w2 (w2 = 0 if there is none; DBL_MAX if no Gaussian is
 * blended).  Candidate mode as in orc_render. */
int orc_gaussian_uncertainty(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                             const double *depth_obs, int candidates, double *nu_sum,
                             int64_t *nu_count, int32_t *dominant, double *dominant_margin);

/* The real spherical harmonics Y_k(d), k < (degree + 1)^2, of the colour
 * reading above at a unit direction d, and their gradients dY[k][3] with
 * respect to d (of the homogeneous polynomial form; only the part tangent to
 * the sphere is meaningful).  Returns the number of coefficients, -1 for a
 * degree outside 0 .. ORC_SH_MAX_DEGREE. */
int orc_sh_basis(int32_t degree, const double d[3], double *Y, double *dY);

/* SE(3) exponential of xi = (rho, phi): T = [exp(phi^), V(phi) rho]. */
void orc_se3_exp(const double xi[6], double R[9], double t[3]);

/* Number of OpenMP threads the oracle uses. */
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
