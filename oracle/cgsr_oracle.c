/*
 * FP64 CPU oracle of the CG-SLAM differentiable Gaussian rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Shares no code
 * with the HIP library.
 *
 * Every function follows the paper's equations in their order and notation;
 * comments name the equation.  There are no tiles, no sort keys and no
 * blocking: a pixel walks the visible Gaussians in ascending depth.
 */
#include "cgsr_oracle.h"

#include <float.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Per-Gaussian projection state                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int visible;
    int clamp[2];
    double s[3];       /* scales exp(log_scale)                  */
    double qn[4];      /* unit quaternion (w, x, y, z)           */
    double qnorm;
    double Rq[9];      /* rotation of the ellipsoid              */
    double Sigma[9];   /* world covariance, Eq. 1                */
    double p[3];       /* camera-space mean                      */
    double Sc[9];      /* W Sigma W^T                            */
    double J[6];       /* 2x3 affine projection Jacobian, Eq. 2  */
    double cov[3];     /* Sigma2d xx, xy, yy with dilation       */
    double conic[3];   /* inverse of Sigma2d: a, b, c            */
    double mu[2];      /* pixel-space mean                       */
    double depth;      /* camera z                               */
    double opacity;    /* sigmoid of the logit                   */
    double color[3];
    double dir[3];     /* unit viewing direction (SH colour)     */
    double vlen;       /* distance from the camera centre        */
    int col_clamped[3]; /* SH colour clamped at zero, per channel */
    int rect[4];       /* u0, u1, v0, v1 inclusive               */
    double edges[4];   /* mu_x - ext_x, mu_x + ext_x, mu_y - ext_y, mu_y + ext_y */
} gproj;

static void mat3_mul(const double *A, const double *B, double *C)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += A[3 * r + k] * B[3 * k + c];
            C[3 * r + c] = acc;
        }
}

static void mat3_transpose(const double *A, double *T)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) T[3 * c + r] = A[3 * r + c];
}

/* Rotation matrix of a unit quaternion (w, x, y, z). */
static void quat_to_rot(const double *q, double *R)
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
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

/* ------------------------------------------------------------------------ */
/* View-dependent colour (Sec. 3.1): real spherical harmonics               */
/* ------------------------------------------------------------------------ */

static double factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

/* Normalisation of the real harmonic (l, m):
 * sqrt((2l + 1) / (4 pi) (l - |m|)! / (l + |m|)!), times sqrt 2 for m != 0. */
static double sh_norm(int l, int m)
{
    const int a = m < 0 ? -m : m;
    const double pi = acos(-1.0);
    const double n = sqrt((2.0 * l + 1.0) / (4.0 * pi) * factorial(l - a) / factorial(l + a));
    return m == 0 ? n : sqrt(2.0) * n;
}

/*
 * Y_l^m = N_lm P_l^|m|(z) times cos(|m| phi) (m > 0) or sin(|m| phi) (m < 0),
 * with P_l^a the associated Legendre function including the Condon-Shortley
 * phase (-1)^a.  Writing P_l^a(z) = Q_la(z) sin^a(theta), the factor
 * sin^a cos(a phi) = Re (x + i y)^a and sin^a sin(a phi) = Im (x + i y)^a,
 * so each harmonic is the polynomial Q_la(z) T(x, y):
 *   P_1 = z:               Q_10 = z,               Q_11 = -1
 *   P_2 = (3z^2 - 1)/2:    Q_20 = (3z^2 - 1)/2,    Q_21 = -3z,  Q_22 = 3
 *   P_3 = (5z^3 - 3z)/2:   Q_30 = (5z^3 - 3z)/2,   Q_31 = -3/2 (5z^2 - 1),
 *                          Q_32 = 15z,             Q_33 = -15
 * (the a-th derivative of P_l times (-1)^a).
 */
static void sh_q(int l, int a, double z, double *q, double *dq)
{
    switch (10 * l + a) {
    case 0:  *q = 1.0;                          *dq = 0.0; break;
    case 10: *q = z;                            *dq = 1.0; break;
    case 11: *q = -1.0;                         *dq = 0.0; break;
    case 20: *q = 0.5 * (3.0 * z * z - 1.0);    *dq = 3.0 * z; break;
    case 21: *q = -3.0 * z;                     *dq = -3.0; break;
    case 22: *q = 3.0;                          *dq = 0.0; break;
    case 30: *q = 0.5 * (5.0 * z * z * z - 3.0 * z); *dq = 0.5 * (15.0 * z * z - 3.0); break;
    case 31: *q = -1.5 * (5.0 * z * z - 1.0);   *dq = -15.0 * z; break;
    case 32: *q = 15.0 * z;                     *dq = 15.0; break;
    default: *q = -15.0;                        *dq = 0.0; break;   /* l = 3, a = 3 */
    }
}

/* Re (m >= 0) or Im (m < 0) of (x + i y)^|m| and its gradient (x, y). */
static void sh_t(int m, double x, double y, double *t, double g[2])
{
    const int a = m < 0 ? -m : m;
    double re = 1.0, im = 0.0, dre[2] = {0.0, 0.0}, dim[2] = {0.0, 0.0};
    for (int k = 0; k < a; ++k) {   /* (re + i im)(x + i y), product rule */
        const double nre = re * x - im * y, nim = re * y + im * x;
        const double ndre[2] = {dre[0] * x + re - dim[0] * y, dre[1] * x - dim[1] * y - im};
        const double ndim[2] = {dre[0] * y + dim[0] * x + im, dre[1] * y + re + dim[1] * x};
        re = nre; im = nim;
        dre[0] = ndre[0]; dre[1] = ndre[1];
        dim[0] = ndim[0]; dim[1] = ndim[1];
    }
    if (m >= 0) { *t = re; g[0] = dre[0]; g[1] = dre[1]; }
    else        { *t = im; g[0] = dim[0]; g[1] = dim[1]; }
}

int orc_sh_basis(int32_t degree, const double d[3], double *Y, double *dY)
{
    if (degree < 0 || degree > ORC_SH_MAX_DEGREE) return -1;
    int k = 0;
    for (int l = 0; l <= degree; ++l)
        for (int m = -l; m <= l; ++m, ++k) {
            double q, dq, t, gt[2];
            sh_q(l, m < 0 ? -m : m, d[2], &q, &dq);
            sh_t(m, d[0], d[1], &t, gt);
            const double n = sh_norm(l, m);
            Y[k] = n * q * t;
            if (dY) {
                dY[3 * k + 0] = n * q * gt[0];
                dY[3 * k + 1] = n * q * gt[1];
                dY[3 * k + 2] = n * dq * t;
            }
        }
    return k;
}

static int sh_count(const orc_gaussians *g) { return (g->sh_degree + 1) * (g->sh_degree + 1); }

/*
 * Project Gaussian i (Eq. 1-2).  frozen, when given, replays the tangent-clamp
 * decisions (x, y) and the colour clamps (r, g, b) recorded at another
 * parameter point.
 */
static void project_one(const orc_gaussians *g, int64_t i, const orc_camera *cam,
                        const orc_pose *P, const int *frozen, gproj *o)
{
    memset(o, 0, sizeof(*o));
    o->rect[0] = o->rect[1] = o->rect[2] = o->rect[3] = -1;
    const double *X = g->means + 3 * i;
    const double *q = g->quats + 4 * i;

    /* Eq. 1: S = diag(exp(log_scale)), R from the normalised quaternion. */
    for (int k = 0; k < 3; ++k) o->s[k] = exp(g->log_scales[3 * i + k]);
    o->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(o->qnorm > 0.0)) return;
    for (int k = 0; k < 4; ++k) o->qn[k] = q[k] / o->qnorm;
    quat_to_rot(o->qn, o->Rq);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += o->Rq[3 * r + k] * o->s[k] * o->s[k] * o->Rq[3 * c + k];
            o->Sigma[3 * r + c] = acc;
        }
    o->opacity = 1.0 / (1.0 + exp(-g->opacity_logits[i]));
    if (g->sh) {
        /* Colour seen along d = (X - C) / |X - C| from the camera centre
         * C = -R^T t, from the SH coefficients (reading in the header). */
        double v[3];
        for (int k = 0; k < 3; ++k)
            v[k] = X[k] + (P->R[k] * P->t[0] + P->R[3 + k] * P->t[1] + P->R[6 + k] * P->t[2]);
        o->vlen = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int k = 0; k < 3; ++k) o->dir[k] = o->vlen > 0.0 ? v[k] / o->vlen : (k == 2 ? 1.0 : 0.0);
        double Y[ORC_SH_MAX_COEFFS];
        const int K = orc_sh_basis(g->sh_degree, o->dir, Y, NULL);
        for (int c = 0; c < 3; ++c) {
            double sum = 0.5;
            for (int k = 0; k < K; ++k) sum += g->sh[(K * i + k) * 3 + c] * Y[k];
            o->col_clamped[c] = frozen ? frozen[2 + c] : sum < 0.0;
            o->color[c] = o->col_clamped[c] ? 0.0 : sum;
        }
    } else {
        for (int k = 0; k < 3; ++k) o->color[k] = g->rgb[3 * i + k];
    }

    /* World to camera. */
    for (int r = 0; r < 3; ++r)
        o->p[r] = P->R[3 * r + 0] * X[0] + P->R[3 * r + 1] * X[1] + P->R[3 * r + 2] * X[2] + P->t[r];
    const double x = o->p[0], y = o->p[1], z = o->p[2];
    o->depth = z;
    if (!(z > ORC_NEAR_Z)) return;
    if (!(o->opacity >= ORC_ALPHA_MIN)) return;

    /* Eq. 2: Sigma2d = J W Sigma W^T J^T, J the affine approximation of the
     * pinhole projection at the camera-space mean (tangents clamped). */
    double WS[9], Wt[9];
    mat3_mul(P->R, o->Sigma, WS);
    mat3_transpose(P->R, Wt);
    mat3_mul(WS, Wt, o->Sc);
    const double limx = ORC_TAN_CLAMP * 0.5 * cam->width / cam->fx;
    const double limy = ORC_TAN_CLAMP * 0.5 * cam->height / cam->fy;
    double tx = x / z, ty = y / z;
    if (frozen) {
        o->clamp[0] = frozen[0];
        o->clamp[1] = frozen[1];
    } else {
        o->clamp[0] = tx > limx ? 1 : (tx < -limx ? -1 : 0);
        o->clamp[1] = ty > limy ? 1 : (ty < -limy ? -1 : 0);
    }
    if (o->clamp[0]) tx = o->clamp[0] * limx;
    if (o->clamp[1]) ty = o->clamp[1] * limy;
    double *J = o->J;
    J[0] = cam->fx / z; J[1] = 0.0;         J[2] = -cam->fx * tx / z;
    J[3] = 0.0;         J[4] = cam->fy / z; J[5] = -cam->fy * ty / z;
    double JS[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += J[3 * r + k] * o->Sc[3 * k + c];
            JS[3 * r + c] = acc;
        }
    double C2[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += JS[3 * r + k] * J[3 * c + k];
            C2[2 * r + c] = acc;
        }
    o->cov[0] = C2[0] + ORC_DILATION;
    o->cov[1] = 0.5 * (C2[1] + C2[2]);
    o->cov[2] = C2[3] + ORC_DILATION;
    const double det = o->cov[0] * o->cov[2] - o->cov[1] * o->cov[1];
    if (!(det > 0.0)) return;
    o->conic[0] = o->cov[2] / det;
    o->conic[1] = -o->cov[1] / det;
    o->conic[2] = o->cov[0] / det;
    /* Pixel-space mean from the unclamped projection. */
    o->mu[0] = cam->fx * x / z + cam->cx;
    o->mu[1] = cam->fy * y / z + cam->cy;

    /* Binning rectangle: the alpha >= 1/255 support is the ellipse
     * d^T conic d <= 2 ln(255 opacity); its bounding box has half extents
     * sqrt(r2 * Sigma2d_xx) and sqrt(r2 * Sigma2d_yy). */
    const double r2 = 2.0 * log(255.0 * o->opacity) * ORC_BIN_R2_REL + ORC_BIN_R2_ABS;
    const double ex = sqrt(r2 * o->cov[0]);
    const double ey = sqrt(r2 * o->cov[2]);
    o->edges[0] = o->mu[0] - ex;
    o->edges[1] = o->mu[0] + ex;
    o->edges[2] = o->mu[1] - ey;
    o->edges[3] = o->mu[1] + ey;
    double u0 = ceil(o->edges[0]), u1 = floor(o->edges[1]);
    double v0 = ceil(o->edges[2]), v1 = floor(o->edges[3]);
    if (u0 < 0.0) u0 = 0.0;
    if (v0 < 0.0) v0 = 0.0;
    if (u1 > cam->width - 1.0) u1 = cam->width - 1.0;
    if (v1 > cam->height - 1.0) v1 = cam->height - 1.0;
    if (!(u0 <= u1 && v0 <= v1)) return;
    o->rect[0] = (int)u0; o->rect[1] = (int)u1;
    o->rect[2] = (int)v0; o->rect[3] = (int)v1;
    o->visible = 1;
}

/* frozen: NULL or [n][5] decisions as in project_one. */
static gproj *project_all(const orc_gaussians *g, const orc_camera *cam, const orc_pose *P,
                          const int *frozen)
{
    gproj *pr = (gproj *)malloc(sizeof(gproj) * (size_t)(g->n > 0 ? g->n : 1));
    if (!pr) return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; ++i)
        project_one(g, i, cam, P, frozen ? frozen + 5 * i : NULL, &pr[i]);
    return pr;
}

int orc_project(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                orc_projection *out)
{
    if (g->sh && (g->sh_degree < 0 || g->sh_degree > ORC_SH_MAX_DEGREE)) return -1;
    gproj *pr = project_all(g, cam, pose, NULL);
    if (!pr) return -2;
    for (int64_t i = 0; i < g->n; ++i) {
        const gproj *o = &pr[i];
        if (out->visible) out->visible[i] = o->visible;
        if (out->clamp) { out->clamp[2 * i] = o->clamp[0]; out->clamp[2 * i + 1] = o->clamp[1]; }
        for (int k = 0; k < 3; ++k) {
            if (out->p_cam) out->p_cam[3 * i + k] = o->p[k];
            if (out->cov2d) out->cov2d[3 * i + k] = o->cov[k];
            if (out->conic) out->conic[3 * i + k] = o->conic[k];
        }
        for (int k = 0; k < 2; ++k)
            if (out->mu) out->mu[2 * i + k] = o->mu[k];
        if (out->depth) out->depth[i] = o->depth;
        if (out->opacity) out->opacity[i] = o->opacity;
        for (int k = 0; k < 4; ++k) {
            if (out->rect) out->rect[4 * i + k] = o->rect[k];
            if (out->rect_edges) out->rect_edges[4 * i + k] = o->edges[k];
        }
    }
    free(pr);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Depth order and per-pixel candidate lists                                */
/* ------------------------------------------------------------------------ */

static const gproj *g_sort_base;

static int cmp_depth_then_index(const void *a, const void *b)
{
    const int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    const double di = g_sort_base[i].depth, dj = g_sort_base[j].depth;
    if (di < dj) return -1;
    if (di > dj) return 1;
    return (i > j) - (i < j);
}

/* Visible Gaussians in ascending (depth, index) order. */
static int64_t *depth_order(const gproj *pr, int64_t n, int64_t *n_vis)
{
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!ord) return NULL;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (pr[i].visible) ord[m++] = i;
    g_sort_base = pr;
    qsort(ord, (size_t)m, sizeof(int64_t), cmp_depth_then_index);
    *n_vis = m;
    return ord;
}

typedef struct {
    int64_t *start;   /* [H*W + 1] */
    int64_t *ids;     /* Gaussian ids, each pixel's run in depth order */
} cand_lists;

/* For candidates mode 1: pixel lists of the Gaussians whose rectangle holds it. */
static int build_candidates(const gproj *pr, const int64_t *ord, int64_t n_vis,
                            const orc_camera *cam, cand_lists *cl)
{
    const int64_t npx = (int64_t)cam->width * cam->height;
    cl->start = (int64_t *)calloc((size_t)npx + 1, sizeof(int64_t));
    if (!cl->start) return -2;
    for (int64_t k = 0; k < n_vis; ++k) {
        const gproj *o = &pr[ord[k]];
        for (int v = o->rect[2]; v <= o->rect[3]; ++v)
            for (int u = o->rect[0]; u <= o->rect[1]; ++u) cl->start[(int64_t)v * cam->width + u + 1]++;
    }
    for (int64_t p = 0; p < npx; ++p) cl->start[p + 1] += cl->start[p];
    cl->ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cl->start[npx] > 0 ? cl->start[npx] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npx > 0 ? npx : 1));
    if (!cl->ids || !fill) { free(fill); return -2; }
    memcpy(fill, cl->start, sizeof(int64_t) * (size_t)npx);
    for (int64_t k = 0; k < n_vis; ++k) {
        const int64_t i = ord[k];
        const gproj *o = &pr[i];
        for (int v = o->rect[2]; v <= o->rect[3]; ++v)
            for (int u = o->rect[0]; u <= o->rect[1]; ++u) cl->ids[fill[(int64_t)v * cam->width + u]++] = i;
    }
    free(fill);
    return 0;
}

static void free_candidates(cand_lists *cl)
{
    free(cl->start);
    free(cl->ids);
}

/* ------------------------------------------------------------------------ */
/* Per-pixel blending (Eq. 3-10)                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    double color[3], depth, opacity, depth_median, uncertainty, t_final, margin, order_margin, stop_order_margin;
    int64_t median;      /* Gaussian id, -1 if T never fell below 0.5 */
    int n;               /* blended Gaussians */
    /* Eq. 13: the blended Gaussian of largest weight alpha T, its weight and
     * depth, and the largest weight among the others */
    int64_t dominant;
    double w_dominant, w_runner_up, d_dominant;
} pixel_out;

/* One blended Gaussian of a pixel, as recorded for the backward pass and
 * for frozen-decision replay. */
typedef struct {
    int64_t id;
    int clamped;         /* alpha was capped at ORC_ALPHA_MAX */
    double alpha, T;     /* alpha_i and the transmittance T_i before it */
    double gauss;        /* exp(power) */
} blend_entry;

static double rel_gap(double a, double thr) { return fabs(a - thr) / thr; }

/* Exponent of the 2-D Gaussian N(mu, Sigma2d) at pixel centre (u, v), up to
 * the normalisation that alpha's opacity factor absorbs (Eq. 5). */
static double gauss_power(const gproj *o, double u, double v)
{
    const double dx = o->mu[0] - u, dy = o->mu[1] - v;
    return -0.5 * (o->conic[0] * dx * dx + o->conic[2] * dy * dy) - o->conic[1] * dx * dy;
}

/*
 * Front-to-back blending at one pixel over candidate ids in depth order.
 * alpha_i = min(0.99, opacity_i * G_i) (Eq. 5), skipped when below 1/255;
 * blending stops before the transmittance (Eq. 4) would fall below 1e-4.
 * Accumulates colour (Eq. 3), depth (Eq. 6), opacity (Eq. 9) and the
 * uncertainty against the sensor depth (Eq. 10); the median Gaussian is the
 * first at which T falls below 0.5 (Eq. 7-8).
 */
static void pixel_forward(const gproj *pr, const int64_t *cand, int64_t ncand, double u,
                          double v, double dobs, int has_dobs, pixel_out *po,
                          blend_entry *trace)
{
    double T = 1.0, prev_depth = -1.0;
    memset(po, 0, sizeof(*po));
    po->median = -1;
    po->dominant = -1;
    po->margin = DBL_MAX;
    po->order_margin = DBL_MAX;
    po->stop_order_margin = DBL_MAX;
    for (int64_t k = 0; k < ncand; ++k) {
        const int64_t i = cand[k];
        const gproj *o = &pr[i];
        const double G = exp(gauss_power(o, u, v));
        const double a_raw = o->opacity * G;
        po->margin = fmin(po->margin, rel_gap(a_raw, ORC_ALPHA_MIN));
        if (a_raw < ORC_ALPHA_MIN) continue;
        po->margin = fmin(po->margin, rel_gap(a_raw, ORC_ALPHA_MAX));
        const int clamped = a_raw > ORC_ALPHA_MAX;
        const double alpha = clamped ? ORC_ALPHA_MAX : a_raw;
        const double Tn = T * (1.0 - alpha);
        po->margin = fmin(po->margin, rel_gap(Tn, ORC_T_STOP));
        if (Tn < ORC_T_STOP) {
            /* The Gaussian that stops the walk, and the next one that would
             * pass the skip test, take part in the result through their order
             * too: were either swapped with its neighbour in depth, a
             * different set of Gaussians would be blended. */
            if (po->n > 0)
                po->stop_order_margin = fmin(po->stop_order_margin, fabs(o->depth - prev_depth) / o->depth);
            for (int64_t k2 = k + 1; k2 < ncand; ++k2) {
                const gproj *o2 = &pr[cand[k2]];
                if (o2->opacity * exp(gauss_power(o2, u, v)) < ORC_ALPHA_MIN) continue;
                po->stop_order_margin = fmin(po->stop_order_margin, fabs(o2->depth - o->depth) / o2->depth);
                break;
            }
            break;
        }
        if (po->n > 0) po->order_margin = fmin(po->order_margin, fabs(o->depth - prev_depth) / o->depth);
        const double w = alpha * T;
        for (int c = 0; c < 3; ++c) po->color[c] += w * o->color[c];
        po->depth += w * o->depth;
        po->opacity += w;
        if (has_dobs) po->uncertainty += w * (o->depth - dobs) * (o->depth - dobs);
        if (w > po->w_dominant) {
            po->w_runner_up = po->w_dominant;
            po->w_dominant = w;
            po->dominant = i;
            po->d_dominant = o->depth;
        } else if (w > po->w_runner_up) {
            po->w_runner_up = w;
        }
        if (po->median < 0) {
            po->margin = fmin(po->margin, rel_gap(Tn, ORC_T_MEDIAN));
            if (Tn < ORC_T_MEDIAN) {
                po->median = i;
                po->depth_median = o->depth;
            }
        }
        if (trace) {
            blend_entry *e = &trace[po->n];
            e->id = i; e->clamped = clamped; e->alpha = alpha; e->T = T; e->gauss = G;
        }
        T = Tn;
        prev_depth = o->depth;
        po->n++;
    }
    po->t_final = T;
}

typedef struct {
    const gproj *pr;
    const int64_t *ord;
    int64_t n_vis;
    cand_lists cl;
    int mode;
} render_ctx;

static void pixel_candidates(const render_ctx *rc, int64_t pix, const int64_t **cand, int64_t *nc)
{
    if (rc->mode == 1) {
        *cand = rc->cl.ids + rc->cl.start[pix];
        *nc = rc->cl.start[pix + 1] - rc->cl.start[pix];
    } else {
        *cand = rc->ord;
        *nc = rc->n_vis;
    }
}

static int render_setup(const orc_gaussians *g, const orc_camera *cam, const orc_pose *P,
                        int mode, render_ctx *rc)
{
    memset(rc, 0, sizeof(*rc));
    rc->mode = mode;
    if (g->sh && (g->sh_degree < 0 || g->sh_degree > ORC_SH_MAX_DEGREE)) return -1;
    rc->pr = project_all(g, cam, P, NULL);
    if (!rc->pr) return -2;
    rc->ord = depth_order(rc->pr, g->n, &rc->n_vis);
    if (!rc->ord) return -2;
    if (mode == 1) return build_candidates(rc->pr, rc->ord, rc->n_vis, cam, &rc->cl);
    return 0;
}

static void render_teardown(render_ctx *rc)
{
    if (rc->mode == 1) free_candidates(&rc->cl);
    free((void *)rc->ord);
    free((void *)rc->pr);
}

int orc_render(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
               const double *depth_obs, int candidates, const int64_t *pixels,
               int64_t n_pixels, orc_images *out)
{
    if (cam->width < 0 || cam->height < 0 || g->n < 0) return -1;
    render_ctx rc;
    int st = render_setup(g, cam, pose, candidates, &rc);
    if (st) { render_teardown(&rc); return st; }
    const int64_t npx = (int64_t)cam->width * cam->height;
    const int64_t count = pixels ? n_pixels : npx;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < count; ++k) {
        const int64_t pix = pixels ? pixels[k] : k;
        const int64_t u = pix % cam->width, v = pix / cam->width;
        const int64_t *cand;
        int64_t nc;
        pixel_candidates(&rc, pix, &cand, &nc);
        pixel_out po;
        pixel_forward(rc.pr, cand, nc, (double)u, (double)v, depth_obs ? depth_obs[pix] : 0.0,
                      depth_obs != NULL, &po, NULL);
        if (out->color)
            for (int c = 0; c < 3; ++c) out->color[c * count + k] = po.color[c];
        if (out->depth) out->depth[k] = po.depth;
        if (out->opacity) out->opacity[k] = po.opacity;
        if (out->depth_median) out->depth_median[k] = po.depth_median;
        if (out->uncertainty) out->uncertainty[k] = depth_obs ? po.uncertainty : 0.0;
        if (out->n_contrib) out->n_contrib[k] = po.n;
        if (out->t_final) out->t_final[k] = po.t_final;
        if (out->median_id) out->median_id[k] = (int32_t)po.median;
        if (out->decision_margin) out->decision_margin[k] = po.margin;
        if (out->order_margin) out->order_margin[k] = po.order_margin;
        if (out->stop_order_margin) out->stop_order_margin[k] = po.stop_order_margin;
    }
    render_teardown(&rc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Admissible results where decisions sit within rounding of a threshold    */
/* ------------------------------------------------------------------------ */

typedef struct {
    const gproj *pr;
    double u, v, dobs;
    int has_dobs;
    double dm, om;          /* decision and order margins (relative)          */
    int max_alts, count;    /* count exceeds max_alts: too many to list       */
    double *out;            /* [max_alts][ORC_ALT_VALUES]                     */
    int64_t *order;         /* the pixel's candidates, reordered by the swaps */
    int64_t n;
} alt_ctx;

typedef struct {
    double T, color[3], depth, opacity, uncertainty, depth_median;
    int has_median;
} alt_state;

static void alt_emit(alt_ctx *a, const alt_state *s)
{
    if (a->count < a->max_alts) {
        double *o = a->out + (size_t)a->count * ORC_ALT_VALUES;
        for (int c = 0; c < 3; ++c) o[c] = s->color[c];
        o[3] = s->depth;
        o[4] = s->opacity;
        o[5] = s->has_median ? s->depth_median : 0.0;
        o[6] = a->has_dobs ? s->uncertainty : 0.0;
        o[7] = s->T;
    }
    a->count++;
}

static double alt_alpha_raw(const alt_ctx *a, int64_t k)
{
    const gproj *o = &a->pr[a->order[k]];
    return o->opacity * exp(gauss_power(o, a->u, a->v));
}

/* Whether a raw alpha is blended under one of the admissible outcomes. */
static int alt_may_blend(const alt_ctx *a, double a_raw)
{
    return a_raw >= ORC_ALPHA_MIN || rel_gap(a_raw, ORC_ALPHA_MIN) < a->dm;
}

/*
 * The walk of pixel_forward (Eq. 3-10) from candidate position k with state s.
 * At a decision inside the margins it follows one outcome by recursion and
 * the other in place.  no_swap: the position whose pair was just exchanged
 * (so the exchange is not undone there).  Each recursion ends in at least one
 * alternative, so the nesting stays below max_alts + 2.
 */
static void alt_walk(alt_ctx *a, int64_t k, alt_state s, int64_t no_swap)
{
    for (; k < a->n; ++k) {
        if (a->count > a->max_alts) return;
        const double a_raw = alt_alpha_raw(a, k);
        if (!alt_may_blend(a, a_raw)) continue;
        /* Order: the next Gaussian that may be blended here, if its depth is
         * within the order margin, may come first (Gaussians skipped at this
         * pixel in between add nothing, wherever they stand). */
        if (k != no_swap) {
            const double d0 = a->pr[a->order[k]].depth;
            for (int64_t k2 = k + 1; k2 < a->n; ++k2) {
                const double d1 = a->pr[a->order[k2]].depth;
                if (!(fabs(d1 - d0) < 2.0 * a->om * fabs(d1))) break;   /* past any near tie */
                if (!alt_may_blend(a, alt_alpha_raw(a, k2))) continue;
                if (fabs(d1 - d0) < a->om * fabs(d1)) {
                    int64_t t = a->order[k];
                    a->order[k] = a->order[k2];
                    a->order[k2] = t;
                    alt_walk(a, k, s, k);
                    t = a->order[k];
                    a->order[k] = a->order[k2];
                    a->order[k2] = t;
                }
                break;
            }
        }
        const gproj *o = &a->pr[a->order[k]];
        if (rel_gap(a_raw, ORC_ALPHA_MIN) < a->dm)
            alt_walk(a, k + 1, s, -1);           /* skipped; below: blended */
        const double alpha = a_raw > ORC_ALPHA_MAX ? ORC_ALPHA_MAX : a_raw;
        const double Tn = s.T * (1.0 - alpha);
        if (rel_gap(Tn, ORC_T_STOP) < a->dm) {
            alt_emit(a, &s);                     /* stopped; below: blended */
        } else if (Tn < ORC_T_STOP) {
            alt_emit(a, &s);
            return;
        }
        const double w = alpha * s.T;
        for (int c = 0; c < 3; ++c) s.color[c] += w * o->color[c];
        s.depth += w * o->depth;
        s.opacity += w;
        if (a->has_dobs) s.uncertainty += w * (o->depth - a->dobs) * (o->depth - a->dobs);
        if (!s.has_median) {
            if (rel_gap(Tn, ORC_T_MEDIAN) < a->dm) {
                alt_state m = s;                 /* the median; below: not yet */
                m.has_median = 1;
                m.depth_median = o->depth;
                m.T = Tn;
                alt_walk(a, k + 1, m, -1);
            } else if (Tn < ORC_T_MEDIAN) {
                s.has_median = 1;
                s.depth_median = o->depth;
            }
        }
        s.T = Tn;
    }
    alt_emit(a, &s);
}

int orc_render_alternatives(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                            const double *depth_obs, int candidates, const int64_t *pixels,
                            int64_t n_pixels, double decision_margin, double order_margin,
                            int32_t max_alts, double *alts, int32_t *n_alts)
{
    if (cam->width < 0 || cam->height < 0 || g->n < 0 || n_pixels < 0 || max_alts < 1) return -1;
    if (!(decision_margin >= 0.0) || !(order_margin >= 0.0)) return -1;
    const int64_t npx = (int64_t)cam->width * cam->height;
    for (int64_t k = 0; k < n_pixels; ++k)
        if (pixels[k] < 0 || pixels[k] >= npx) return -1;
    render_ctx rc;
    int st = render_setup(g, cam, pose, candidates, &rc);
    if (st) { render_teardown(&rc); return st; }
    int failed = 0;
#pragma omp parallel
    {
        int64_t cap = 0;
        int64_t *order = NULL;
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < n_pixels; ++k) {
            const int64_t pix = pixels[k];
            const int64_t *cand;
            int64_t nc;
            pixel_candidates(&rc, pix, &cand, &nc);
            if (nc > cap) {
                free(order);
                cap = nc;
                order = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
                if (!order) {
#pragma omp atomic write
                    failed = 1;
                    cap = 0;
                    continue;
                }
            }
            if (nc > 0) memcpy(order, cand, sizeof(int64_t) * (size_t)nc);
            alt_ctx a;
            a.pr = rc.pr;
            a.u = (double)(pix % cam->width);
            a.v = (double)(pix / cam->width);
            a.has_dobs = depth_obs != NULL;
            a.dobs = depth_obs ? depth_obs[pix] : 0.0;
            a.dm = decision_margin;
            a.om = order_margin;
            a.max_alts = max_alts;
            a.count = 0;
            a.out = alts + (size_t)k * (size_t)max_alts * ORC_ALT_VALUES;
            a.order = order;
            a.n = nc;
            alt_state s;
            memset(&s, 0, sizeof(s));
            s.T = 1.0;
            alt_walk(&a, 0, s, -1);
            n_alts[k] = a.count > max_alts ? max_alts + 1 : a.count;
        }
        free(order);
    }
    render_teardown(&rc);
    return failed ? -2 : 0;
}

int orc_gaussian_uncertainty(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                             const double *depth_obs, int candidates, double *nu_sum,
                             int64_t *nu_count, int32_t *dominant, double *dominant_margin)
{
    if (cam->width < 0 || cam->height < 0 || g->n < 0 || !depth_obs || !nu_sum || !nu_count) return -1;
    render_ctx rc;
    int st = render_setup(g, cam, pose, candidates, &rc);
    if (st) { render_teardown(&rc); return st; }
    const int64_t npx = (int64_t)cam->width * cam->height;
    int64_t *dom = malloc(sizeof(int64_t) * (size_t)(npx ? npx : 1));
    double *contrib = malloc(sizeof(double) * (size_t)(npx ? npx : 1));
    if (!dom || !contrib) { free(dom); free(contrib); render_teardown(&rc); return -2; }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t pix = 0; pix < npx; ++pix) {
        const int64_t *cand;
        int64_t nc;
        pixel_candidates(&rc, pix, &cand, &nc);
        pixel_out po;
        pixel_forward(rc.pr, cand, nc, (double)(pix % cam->width), (double)(pix / cam->width),
                      depth_obs[pix], 1, &po, NULL);
        dom[pix] = -1;
        contrib[pix] = 0.0;
        if (po.dominant >= 0 && depth_obs[pix] > 0.0) {
            const double e = depth_obs[pix] - po.d_dominant;
            dom[pix] = po.dominant;
            contrib[pix] = po.w_dominant * e * e;
        }
        if (dominant) dominant[pix] = (int32_t)po.dominant;
        if (dominant_margin)
            dominant_margin[pix] = po.dominant < 0 ? DBL_MAX
                                                   : (po.w_dominant - po.w_runner_up) / po.w_dominant;
    }
    /* serial scatter: the sums do not depend on the thread count */
    for (int64_t pix = 0; pix < npx; ++pix) {
        if (dom[pix] < 0) continue;
        nu_sum[dom[pix]] += contrib[pix];
        nu_count[dom[pix]] += 1;
    }
    free(dom);
    free(contrib);
    render_teardown(&rc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Backward                                                                 */
/* ------------------------------------------------------------------------ */

/* Gradients with respect to the projected quantities of one Gaussian. */
typedef struct {
    double mu[2], conic[3], opacity, depth, color[3];
} proj_grad;

static void atomic_add(double *dst, double v)
{
#pragma omp atomic
    *dst += v;
}

/*
 * Chain rule through one pixel's blend.  With w_i = alpha_i T_i and any
 * per-Gaussian quantity x blended as X = sum_i w_i x_i, the weights of the
 * Gaussians behind i carry the factor (1 - alpha_i), hence
 *     dX/dalpha_i = T_i x_i - (sum_{j>i} w_j x_j) / (1 - alpha_i).
 * The blended quantities are colour, depth, 1 (opacity) and (d - D)^2.
 */
static void pixel_backward(const gproj *pr, const blend_entry *tr, int n, double u, double v,
                           double dobs, const double g[7], int64_t median, proj_grad *pg)
{
    /* g = dL/d(colour r, g, b, depth, opacity, median depth, uncertainty) */
    double behind[6] = {0, 0, 0, 0, 0, 0};
    for (int k = n - 1; k >= 0; --k) {
        const blend_entry *e = &tr[k];
        const gproj *o = &pr[e->id];
        const double unc = (o->depth - dobs) * (o->depth - dobs);
        const double x[6] = {o->color[0], o->color[1], o->color[2], o->depth, 1.0, unc};
        const double gx[6] = {g[0], g[1], g[2], g[3], g[4], g[6]};
        double dalpha = 0.0;
        for (int c = 0; c < 6; ++c) dalpha += gx[c] * (e->T * x[c] - behind[c] / (1.0 - e->alpha));
        const double w = e->alpha * e->T;
        for (int c = 0; c < 6; ++c) behind[c] += w * x[c];

        proj_grad *d = &pg[e->id];
        for (int c = 0; c < 3; ++c) atomic_add(&d->color[c], w * g[c]);
        double dd = w * g[3] + 2.0 * w * (o->depth - dobs) * g[6];
        if (e->id == median) dd += g[5];
        atomic_add(&d->depth, dd);
        if (!e->clamped) {
            /* alpha = opacity * exp(power) */
            atomic_add(&d->opacity, dalpha * e->gauss);
            const double dpower = dalpha * o->opacity * e->gauss;
            const double dx = o->mu[0] - u, dy = o->mu[1] - v;
            atomic_add(&d->mu[0], -dpower * (o->conic[0] * dx + o->conic[1] * dy));
            atomic_add(&d->mu[1], -dpower * (o->conic[1] * dx + o->conic[2] * dy));
            atomic_add(&d->conic[0], -0.5 * dpower * dx * dx);
            atomic_add(&d->conic[1], -dpower * dx * dy);
            atomic_add(&d->conic[2], -0.5 * dpower * dy * dy);
        }
    }
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/*
 * Chain rule from the projected quantities back to the parameters of one
 * Gaussian and to the pose (left perturbation T <- exp(xi^) T, xi = (rho, phi)).
 */
static void gaussian_backward(const orc_gaussians *g, int64_t i, const orc_camera *cam,
                              const orc_pose *P, const gproj *o, const proj_grad *d,
                              orc_grads *out, double pose_acc[6])
{
    const double x = o->p[0], y = o->p[1], z = o->p[2];
    const double fx = cam->fx, fy = cam->fy;
    /* conic = inverse(Sigma2d); the off-diagonal conic entry b appears twice
     * in the quadratic form, so each matrix entry carries half of db. */
    const double a = o->conic[0], b = o->conic[1], c = o->conic[2];
    const double GQ[4] = {d->conic[0], 0.5 * d->conic[1], 0.5 * d->conic[1], d->conic[2]};
    const double Q[4] = {a, b, b, c};
    double QG[4], A[4];
    for (int r = 0; r < 2; ++r)
        for (int cc = 0; cc < 2; ++cc) QG[2 * r + cc] = Q[2 * r] * GQ[cc] + Q[2 * r + 1] * GQ[2 + cc];
    for (int r = 0; r < 2; ++r)
        for (int cc = 0; cc < 2; ++cc) A[2 * r + cc] = -(QG[2 * r] * Q[cc] + QG[2 * r + 1] * Q[2 + cc]);
    /* A = dL/dSigma2d.  Sigma2d = J Sc J^T + dilation. */
    const double *J = o->J;
    double dSc[9], dJ[6];
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) {
            double acc = 0.0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) acc += J[3 * k + r] * A[2 * k + l] * J[3 * l + cc];
            dSc[3 * r + cc] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int cc = 0; cc < 3; ++cc) {
            double acc = 0.0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 3; ++l) acc += A[2 * r + k] * J[3 * k + l] * o->Sc[3 * l + cc];
            dJ[3 * r + cc] = 2.0 * acc;
        }
    /* Camera-space mean: mu = (fx x/z + cx, fy y/z + cy), depth = z, and J(p). */
    double dp[3];
    dp[0] = d->mu[0] * fx / z;
    dp[1] = d->mu[1] * fy / z;
    dp[2] = -d->mu[0] * fx * x / (z * z) - d->mu[1] * fy * y / (z * z) + d->depth;
    dp[2] += dJ[0] * (-fx / (z * z)) + dJ[4] * (-fy / (z * z));
    const double limx = ORC_TAN_CLAMP * 0.5 * cam->width / fx;
    const double limy = ORC_TAN_CLAMP * 0.5 * cam->height / fy;
    if (o->clamp[0] == 0) {     /* J02 = -fx x / z^2 */
        dp[0] += dJ[2] * (-fx / (z * z));
        dp[2] += dJ[2] * (2.0 * fx * x / (z * z * z));
    } else {                    /* J02 = -fx tx / z with tx fixed */
        dp[2] += dJ[2] * (fx * o->clamp[0] * limx / (z * z));
    }
    if (o->clamp[1] == 0) {
        dp[1] += dJ[5] * (-fy / (z * z));
        dp[2] += dJ[5] * (2.0 * fy * y / (z * z * z));
    } else {
        dp[2] += dJ[5] * (fy * o->clamp[1] * limy / (z * z));
    }
    /* Means: p = W X + t. */
    if (out->means)
        for (int k = 0; k < 3; ++k)
            out->means[3 * i + k] += P->R[k] * dp[0] + P->R[3 + k] * dp[1] + P->R[6 + k] * dp[2];
    /* Sc = W Sigma W^T  =>  dSigma = W^T dSc W. */
    double dSigma[9], tmp[9], Wt[9];
    mat3_transpose(P->R, Wt);
    mat3_mul(Wt, dSc, tmp);
    mat3_mul(tmp, P->R, dSigma);
    /* Sigma = sum_k s_k^2 r_k r_k^T with r_k the columns of Rq (Eq. 1). */
    if (out->log_scales)
        for (int k = 0; k < 3; ++k) {
            double quad = 0.0;
            for (int r = 0; r < 3; ++r)
                for (int cc = 0; cc < 3; ++cc) quad += o->Rq[3 * r + k] * dSigma[3 * r + cc] * o->Rq[3 * cc + k];
            const double ds = 2.0 * o->s[k] * quad;
            out->log_scales[3 * i + k] += ds * o->s[k];
        }
    if (out->quats) {
        /* dRq = 2 dSigma Rq S^2 for symmetric dSigma. */
        double dR[9];
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += dSigma[3 * r + k] * o->Rq[3 * k + cc];
                dR[3 * r + cc] = 2.0 * acc * o->s[cc] * o->s[cc];
            }
        const double w = o->qn[0], qx = o->qn[1], qy = o->qn[2], qz = o->qn[3];
        double dq[4];
        dq[0] = 2.0 * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
        dq[1] = 2.0 * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.0 * qx * dR[4] - w * dR[5] + qz * dR[6]
                       + w * dR[7] - 2.0 * qx * dR[8]);
        dq[2] = 2.0 * (-2.0 * qy * dR[0] + qx * dR[1] + w * dR[2] + qx * dR[3] + qz * dR[5] - w * dR[6]
                       + qz * dR[7] - 2.0 * qy * dR[8]);
        dq[3] = 2.0 * (-2.0 * qz * dR[0] - w * dR[1] + qx * dR[2] + w * dR[3] - 2.0 * qz * dR[4]
                       + qy * dR[5] + qx * dR[6] + qy * dR[7]);
        /* q_hat = q / |q|. */
        double dot = 0.0;
        for (int k = 0; k < 4; ++k) dot += o->qn[k] * dq[k];
        for (int k = 0; k < 4; ++k) out->quats[4 * i + k] += (dq[k] - o->qn[k] * dot) / o->qnorm;
    }
    if (out->opacity_logits)
        out->opacity_logits[i] += d->opacity * o->opacity * (1.0 - o->opacity);
    if (g->sh) {
        /* colour_c = max(0, sum_k sh_kc Y_k(d) + 1/2), d = v / |v|, v = X - C. */
        double Y[ORC_SH_MAX_COEFFS], dY[3 * ORC_SH_MAX_COEFFS], gdir[3] = {0.0, 0.0, 0.0};
        const int K = orc_sh_basis(g->sh_degree, o->dir, Y, dY);
        for (int c = 0; c < 3; ++c) {
            const double dc = o->col_clamped[c] ? 0.0 : d->color[c];
            for (int k = 0; k < K; ++k) {
                if (out->sh) out->sh[(K * i + k) * 3 + c] += dc * Y[k];
                for (int j = 0; j < 3; ++j) gdir[j] += dc * g->sh[(K * i + k) * 3 + c] * dY[3 * k + j];
            }
        }
        /* d = v / |v|: dL/dv = (I - d d^T) dL/dd / |v|. */
        const double dot = gdir[0] * o->dir[0] + gdir[1] * o->dir[1] + gdir[2] * o->dir[2];
        double dv[3];
        for (int j = 0; j < 3; ++j) dv[j] = (gdir[j] - o->dir[j] * dot) / o->vlen;
        if (out->means)
            for (int j = 0; j < 3; ++j) out->means[3 * i + j] += dv[j];
        /* The camera centre C = -R^T t moves to C - R^T rho under exp(xi^) T
         * (rotation alone leaves it in place), so dL/drho += -R dL/dC = R dL/dv. */
        for (int r = 0; r < 3; ++r)
            pose_acc[r] += P->R[3 * r] * dv[0] + P->R[3 * r + 1] * dv[1] + P->R[3 * r + 2] * dv[2];
    } else if (out->rgb) {
        for (int k = 0; k < 3; ++k) out->rgb[3 * i + k] += d->color[k];
    }
    /* Pose: p' = exp(xi^) p gives dp'/drho = I, dp'/dphi = -[p]x; the camera
     * covariance Sc' = exp(phi^) Sc exp(phi^)^T contributes 2 vee-parts of
     * the skew part of M = Sc dSc. */
    double pxdp[3];
    cross3(o->p, dp, pxdp);
    double M[9];
    mat3_mul(o->Sc, dSc, M);
    for (int k = 0; k < 3; ++k) pose_acc[k] += dp[k];
    pose_acc[3] += pxdp[0] + 2.0 * (M[5] - M[7]);
    pose_acc[4] += pxdp[1] + 2.0 * (M[6] - M[2]);
    pose_acc[5] += pxdp[2] + 2.0 * (M[1] - M[3]);
}

static void gather_grad7(const orc_image_grads *dimg, int64_t pix, int64_t npx, double g[7])
{
    for (int c = 0; c < 3; ++c) g[c] = dimg->color ? dimg->color[c * npx + pix] : 0.0;
    g[3] = dimg->depth ? dimg->depth[pix] : 0.0;
    g[4] = dimg->opacity ? dimg->opacity[pix] : 0.0;
    g[5] = dimg->depth_median ? dimg->depth_median[pix] : 0.0;
    g[6] = dimg->uncertainty ? dimg->uncertainty[pix] : 0.0;
}

int orc_backward(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                 const double *depth_obs, int candidates, const orc_image_grads *dimg,
                 orc_grads *out)
{
    if (dimg->uncertainty && !depth_obs) return -1;
    render_ctx rc;
    int st = render_setup(g, cam, pose, candidates, &rc);
    if (st) { render_teardown(&rc); return st; }
    proj_grad *pg = (proj_grad *)calloc((size_t)(g->n > 0 ? g->n : 1), sizeof(proj_grad));
    if (!pg) { render_teardown(&rc); return -2; }
    const int64_t npx = (int64_t)cam->width * cam->height;
#pragma omp parallel
    {
        blend_entry *trace = (blend_entry *)malloc(sizeof(blend_entry) * (size_t)(rc.n_vis > 0 ? rc.n_vis : 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t pix = 0; pix < npx; ++pix) {
            const int64_t u = pix % cam->width, v = pix / cam->width;
            const int64_t *cand;
            int64_t nc;
            pixel_candidates(&rc, pix, &cand, &nc);
            const double dobs = depth_obs ? depth_obs[pix] : 0.0;
            pixel_out po;
            pixel_forward(rc.pr, cand, nc, (double)u, (double)v, dobs, depth_obs != NULL, &po, trace);
            double g7[7];
            gather_grad7(dimg, pix, npx, g7);
            pixel_backward(rc.pr, trace, po.n, (double)u, (double)v, dobs, g7, po.median, pg);
        }
        free(trace);
    }
    double pose_acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < g->n; ++i) {
        if (!rc.pr[i].visible) continue;
        if (out->mu) for (int k = 0; k < 2; ++k) out->mu[2 * i + k] += pg[i].mu[k];
        if (out->conic) for (int k = 0; k < 3; ++k) out->conic[3 * i + k] += pg[i].conic[k];
        if (out->opacity) out->opacity[i] += pg[i].opacity;
        if (out->depth) out->depth[i] += pg[i].depth;
        gaussian_backward(g, i, cam, pose, &rc.pr[i], &pg[i], out, pose_acc);
    }
    if (out->pose)
        for (int k = 0; k < 6; ++k) out->pose[k] += pose_acc[k];
    free(pg);
    render_teardown(&rc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* SE(3) exponential                                                        */
/* ------------------------------------------------------------------------ */

void orc_se3_exp(const double xi[6], double R[9], double t[3])
{
    const double *rho = xi, *phi = xi + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    double A, B, C; /* sin(th)/th, (1-cos th)/th^2, (th - sin th)/th^3 */
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
    double K2[9];
    mat3_mul(K, K, K2);
    double V[9];
    for (int k = 0; k < 9; ++k) {
        const double I = (k % 4 == 0) ? 1.0 : 0.0;
        R[k] = I + A * K[k] + B * K2[k];
        V[k] = I + B * K[k] + C * K2[k];
    }
    for (int r = 0; r < 3; ++r) t[r] = V[3 * r] * rho[0] + V[3 * r + 1] * rho[1] + V[3 * r + 2] * rho[2];
}

/* ------------------------------------------------------------------------ */
/* Frozen-decision finite differences                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t *start;      /* [npx + 1] */
    blend_entry *e;      /* blended Gaussians of every pixel, front to back */
    int64_t *median_pos; /* [npx] position of the median within the pixel's run, -1 */
    int *clamp;          /* [n][5] tangent clamps (x, y), colour clamps (r, g, b) */
} frozen_trace;

/* Linear probe over the frozen branch: re-project with the recorded clamps,
 * then blend every pixel's recorded run with recorded alpha caps. */
static double frozen_probe(const orc_gaussians *g, const orc_camera *cam, const orc_pose *P,
                           const double *depth_obs, const orc_image_grads *dimg,
                           const frozen_trace *ft)
{
    gproj *pr = project_all(g, cam, P, ft->clamp);
    const int64_t npx = (int64_t)cam->width * cam->height;
    double total = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t pix = 0; pix < npx; ++pix) {
        const double u = (double)(pix % cam->width), v = (double)(pix / cam->width);
        const double dobs = depth_obs ? depth_obs[pix] : 0.0;
        double T = 1.0, C[3] = {0, 0, 0}, D = 0, O = 0, U = 0, Dm = 0;
        for (int64_t k = ft->start[pix]; k < ft->start[pix + 1]; ++k) {
            const blend_entry *e = &ft->e[k];
            const gproj *o = &pr[e->id];
            const double alpha = e->clamped ? ORC_ALPHA_MAX : o->opacity * exp(gauss_power(o, u, v));
            const double w = alpha * T;
            for (int c = 0; c < 3; ++c) C[c] += w * o->color[c];
            D += w * o->depth;
            O += w;
            U += w * (o->depth - dobs) * (o->depth - dobs);
            if (k - ft->start[pix] == ft->median_pos[pix]) Dm = o->depth;
            T *= 1.0 - alpha;
        }
        double g7[7];
        gather_grad7(dimg, pix, npx, g7);
        total += g7[0] * C[0] + g7[1] * C[1] + g7[2] * C[2] + g7[3] * D + g7[4] * O + g7[5] * Dm
                 + g7[6] * U;
    }
    free(pr);
    return total;
}

int orc_fd_linear(const orc_gaussians *g, const orc_camera *cam, const orc_pose *pose,
                  const double *depth_obs, const orc_image_grads *dimg, int64_t n_coords,
                  const int32_t *kind, const int64_t *index, const int32_t *comp,
                  double rel_step, double *out)
{
    if (dimg->uncertainty && !depth_obs) return -1;
    const int64_t n = g->n;
    const int64_t npx = (int64_t)cam->width * cam->height;
    /* Record the decision trace at the unperturbed point. */
    render_ctx rc;
    int st = render_setup(g, cam, pose, 1, &rc);
    if (st) { render_teardown(&rc); return st; }
    frozen_trace ft;
    ft.start = (int64_t *)calloc((size_t)npx + 1, sizeof(int64_t));
    ft.median_pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npx > 0 ? npx : 1));
    ft.clamp = (int *)malloc(sizeof(int) * (size_t)(5 * (n > 0 ? n : 1)));
    pixel_out *pos = (pixel_out *)malloc(sizeof(pixel_out) * (size_t)(npx > 0 ? npx : 1));
    for (int64_t i = 0; i < n; ++i) {
        ft.clamp[5 * i] = rc.pr[i].clamp[0];
        ft.clamp[5 * i + 1] = rc.pr[i].clamp[1];
        for (int c = 0; c < 3; ++c) ft.clamp[5 * i + 2 + c] = rc.pr[i].col_clamped[c];
    }
    for (int64_t pix = 0; pix < npx; ++pix) {
        const int64_t *cand;
        int64_t nc;
        pixel_candidates(&rc, pix, &cand, &nc);
        pixel_forward(rc.pr, cand, nc, (double)(pix % cam->width), (double)(pix / cam->width),
                      depth_obs ? depth_obs[pix] : 0.0, depth_obs != NULL, &pos[pix], NULL);
        ft.start[pix + 1] = ft.start[pix] + pos[pix].n;
    }
    ft.e = (blend_entry *)malloc(sizeof(blend_entry) * (size_t)(ft.start[npx] > 0 ? ft.start[npx] : 1));
    for (int64_t pix = 0; pix < npx; ++pix) {
        const int64_t *cand;
        int64_t nc;
        pixel_candidates(&rc, pix, &cand, &nc);
        pixel_out po;
        pixel_forward(rc.pr, cand, nc, (double)(pix % cam->width), (double)(pix / cam->width),
                      depth_obs ? depth_obs[pix] : 0.0, depth_obs != NULL, &po, ft.e + ft.start[pix]);
        ft.median_pos[pix] = -1;
        for (int k = 0; k < po.n; ++k)
            if (ft.e[ft.start[pix] + k].id == po.median) ft.median_pos[pix] = k;
    }
    free(pos);
    render_teardown(&rc);

    /* Private copies of the parameters to perturb. */
    double *buf[7];
    const double *src[7] = {g->means, g->log_scales, g->quats, g->opacity_logits, g->rgb, NULL, g->sh};
    const int width[7] = {3, 3, 4, 1, 3, 0, g->sh ? 3 * sh_count(g) : 0};
    for (int k = 0; k < 7; ++k) {
        buf[k] = (double *)malloc(sizeof(double) * (size_t)(width[k] * (n > 0 ? n : 1) + 1));
        if (src[k]) memcpy(buf[k], src[k], sizeof(double) * (size_t)(width[k] * n));
    }
    orc_gaussians gp = {n, buf[0], buf[1], buf[2], buf[3], g->rgb ? buf[4] : NULL, g->sh ? buf[6] : NULL,
                        g->sh_degree};
    for (int64_t c = 0; c < n_coords; ++c) {
        double vals[2];
        double h = rel_step;
        for (int sgn = 0; sgn < 2; ++sgn) {
            const double s = sgn == 0 ? 1.0 : -1.0;
            if (kind[c] == 5) {
                double xi[6] = {0, 0, 0, 0, 0, 0}, dR[9], dt[3];
                xi[comp[c]] = s * h;
                orc_se3_exp(xi, dR, dt);
                orc_pose pp;
                mat3_mul(dR, pose->R, pp.R);
                for (int r = 0; r < 3; ++r)
                    pp.t[r] = dR[3 * r] * pose->t[0] + dR[3 * r + 1] * pose->t[1] + dR[3 * r + 2] * pose->t[2] + dt[r];
                vals[sgn] = frozen_probe(&gp, cam, &pp, depth_obs, dimg, &ft);
            } else {
                double *slot = &buf[kind[c]][width[kind[c]] * index[c] + comp[c]];
                const double orig = *slot;
                h = rel_step * fmax(1.0, fabs(orig));
                *slot = orig + s * h;
                vals[sgn] = frozen_probe(&gp, cam, pose, depth_obs, dimg, &ft);
                *slot = orig;
            }
        }
        out[c] = (vals[0] - vals[1]) / (2.0 * h);
    }
    for (int k = 0; k < 7; ++k) free(buf[k]);
    free(ft.start);
    free(ft.e);
    free(ft.median_pos);
    free(ft.clamp);
    return 0;
}

int orc_num_threads(void) { return omp_get_max_threads(); }
