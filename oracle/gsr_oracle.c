/*
 * gsr_oracle.c -- TEST INFRASTRUCTURE, not part of the product path.
 *
 * A plain, slow, FP64 CPU reference of the differentiable 3D Gaussian-splatting
 * renderer that RGS-SLAM (arXiv 2601.00705) drives for tracking and mapping.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the HIP path.
 *
 * What it follows:
 *   - Sec. "Gaussian Splatting Representation", Eq. (proj): mu_I = pi(T_WC mu_W),
 *     Sigma_I = J R Sigma_W R^T J^T (first-order linearisation of pi).
 *   - Eq. (alpha): front-to-back alpha compositing over the depth-ordered set
 *     N(p) of Gaussians overlapping pixel p; alpha = opacity x 2-D Gaussian.
 *   - Appendix "Methodology Details / Gaussian Splatting Representation":
 *     Sigma_W = R_i diag(s^2) R_i^T, unit quaternion, log-scales; colour as
 *     real spherical harmonics, Eq. (app-sh).
 *   - Sec. "Minimal Pose Jacobians on SE(3)", Eq. (leftupdate) T <- exp(xi^) T,
 *     Eq. (muCjac) d mu_C / d xi = [I  -[mu_C]x], Eq. (muIjac), Eq. (sigmaIjac)
 *     with dR = [d omega]x R.
 *
 * Readings taken where the paper is silent (each one is listed in the design
 * notes): pixel centres at (px+1/2, py+1/2); unnormalised 2-D Gaussian (peak 1);
 * screen covariance dilated by eps*I; alpha clamped to alpha_max, contributions
 * below alpha_min skipped; compositing stops before the Gaussian that would take
 * T below T_min; background bg * T_final; ordering by camera-space depth with
 * ties broken by Gaussian index; sigmoid opacity; SH direction from the camera
 * centre in world frame.
 *
 * Forward: per tile, the Gaussians whose conservative bounding rectangle covers
 * the tile, sorted by (float32-rounded depth, index); per pixel the plain
 * compositing sum.
 * Backward: per pixel, the blended list is stored and the colour "behind" each
 * entry and the transmittance product after it are built by suffix recursion
 * (no division by 1-alpha), then the chain rule is written out scalar by scalar.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the OpenMP loops (pixel rows, Gaussians, tile lists); 0 keeps
 * the OpenMP default.  Per-thread gradient buffers are merged in thread order,
 * so a result depends on the thread count only through FP64 rounding. */
void or_set_threads(int32_t n)
{
    if (n > 0) omp_set_num_threads(n);
}

int32_t or_get_threads(void) { return (int32_t)omp_get_max_threads(); }

typedef struct {
    int32_t tile_w, tile_h, sh_degree; /* sh_degree < 0: plain RGB colour */
    double z_near, dilation, alpha_min, alpha_max, T_min;
    double bg[3];
    int32_t staging_f32; /* tolerance model only: the renderer stages the projected
                            centre and conic rounded to float32 (see
                            power2_abs_error); no rendered value depends on it */
} or_config;

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
} or_camera;

typedef struct {
    int64_t n;
    const double *mean;          /* [3][n] */
    const double *quat;          /* [4][n]  (w, x, y, z), need not be unit */
    const double *log_scale;     /* [3][n] */
    const double *opacity_logit; /* [n] */
    const double *colour;        /* [3][n] (RGB) or [K][3][n] (SH, K=(d+1)^2) */
} or_scene;

/* Fields of one projected record as returned by or_project. */
enum {
    OP_VALID, OP_U, OP_V, OP_A, OP_B, OP_C, OP_O, OP_R, OP_G, OP_BL, OP_DEPTH,
    OP_RX, OP_RY, OP_COVA, OP_COVB, OP_COVC, OP_MCX, OP_MCY, OP_MCZ,
    OP_TX0, OP_TY0, OP_TX1, OP_TY1, OP_NFIELDS
};

/* ------------------------------------------------------------------------ */
/* small linear algebra, row-major 3x3                                       */

static void quat_to_rot(const double q[4], double R[9])
{
    /* rotation matrix of a unit quaternion (w, x, y, z) */
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* partial derivatives of quat_to_rot w.r.t. w, x, y, z (polynomial form) */
static void quat_to_rot_partials(const double q[4], double dR[4][9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double a[4][9] = {
        { 0, -2 * z, 2 * y,   2 * z, 0, -2 * x,   -2 * y, 2 * x, 0 },
        { 0, 2 * y, 2 * z,    2 * y, -4 * x, -2 * w,   2 * z, 2 * w, -4 * x },
        { -4 * y, 2 * x, 2 * w,   2 * x, 0, 2 * z,   -2 * w, 2 * z, -4 * y },
        { -4 * z, -2 * w, 2 * x,   2 * w, -4 * z, 2 * y,   2 * x, 2 * y, 0 },
    };
    memcpy(dR, a, sizeof(a));
}

/* ------------------------------------------------------------------------ */
/* real spherical harmonics up to degree 3, Eq. (app-sh); index l*l + l + m   */

static int sh_count(int deg) { return deg < 0 ? 0 : (deg + 1) * (deg + 1); }

static void sh_basis(int deg, const double n[3], double Y[16], double dY[16][3])
{
    double x = n[0], y = n[1], z = n[2];
    double pi = M_PI;
    double c0 = 0.5 * sqrt(1.0 / pi);
    double c1 = sqrt(3.0 / (4.0 * pi));
    double c2a = 0.5 * sqrt(15.0 / pi);      /* xy, yz, xz */
    double c2b = 0.25 * sqrt(5.0 / pi);      /* 3z^2 - 1 */
    double c2c = 0.25 * sqrt(15.0 / pi);     /* x^2 - y^2 */
    double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)); /* m = +-3 */
    double c3b = 0.5 * sqrt(105.0 / pi);     /* xyz */
    double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)); /* m = +-1 */
    double c3d = 0.25 * sqrt(7.0 / pi);      /* m = 0 */
    double c3e = 0.25 * sqrt(105.0 / pi);    /* z (x^2 - y^2) */
    memset(Y, 0, 16 * sizeof(double));
    memset(dY, 0, 16 * 3 * sizeof(double));
    Y[0] = c0;
    if (deg < 1) return;
    Y[1] = c1 * y; dY[1][1] = c1;
    Y[2] = c1 * z; dY[2][2] = c1;
    Y[3] = c1 * x; dY[3][0] = c1;
    if (deg < 2) return;
    Y[4] = c2a * x * y;             dY[4][0] = c2a * y; dY[4][1] = c2a * x;
    Y[5] = c2a * y * z;             dY[5][1] = c2a * z; dY[5][2] = c2a * y;
    Y[6] = c2b * (3 * z * z - 1);   dY[6][2] = c2b * 6 * z;
    Y[7] = c2a * x * z;             dY[7][0] = c2a * z; dY[7][2] = c2a * x;
    Y[8] = c2c * (x * x - y * y);   dY[8][0] = c2c * 2 * x; dY[8][1] = -c2c * 2 * y;
    if (deg < 3) return;
    Y[9] = c3a * y * (3 * x * x - y * y);
    dY[9][0] = c3a * 6 * x * y; dY[9][1] = c3a * (3 * x * x - 3 * y * y);
    Y[10] = c3b * x * y * z;
    dY[10][0] = c3b * y * z; dY[10][1] = c3b * x * z; dY[10][2] = c3b * x * y;
    Y[11] = c3c * y * (5 * z * z - 1);
    dY[11][1] = c3c * (5 * z * z - 1); dY[11][2] = c3c * 10 * y * z;
    Y[12] = c3d * z * (5 * z * z - 3);
    dY[12][2] = c3d * (15 * z * z - 3);
    Y[13] = c3c * x * (5 * z * z - 1);
    dY[13][0] = c3c * (5 * z * z - 1); dY[13][2] = c3c * 10 * x * z;
    Y[14] = c3e * z * (x * x - y * y);
    dY[14][0] = c3e * 2 * x * z; dY[14][1] = -c3e * 2 * y * z; dY[14][2] = c3e * (x * x - y * y);
    Y[15] = c3a * x * (x * x - 3 * y * y);
    dY[15][0] = c3a * (3 * x * x - 3 * y * y); dY[15][1] = -c3a * 6 * x * y;
}

/* exported for the SH pins */
void or_sh_basis(int32_t deg, const double *n, double *Y)
{
    double dY[16][3];
    sh_basis(deg, n, Y, dY);
}

/* ------------------------------------------------------------------------ */
/* projection of one Gaussian into one view: Eq. (proj) + extent + rect      */

typedef struct {
    int valid;
    double q[4], qn, R_q[9], s[3], Sigma_w[9], o;
    double mc[3], J[6], M[6], cov[3], det, conic[3];
    double u, v, rx, ry, rgb[3];
    double dir[3], dnorm; /* SH view direction (world) and |mu_W - o_c| */
    int tx0, ty0, tx1, ty1;
} proj_t;

static void project_one(const or_scene *sc, int64_t i, const or_camera *cam,
                        const double *pose, const or_config *cfg, proj_t *p)
{
    int64_t n = sc->n;
    memset(p, 0, sizeof(*p));
    p->tx0 = 1; p->tx1 = 0; p->ty0 = 1; p->ty1 = 0;

    /* activation: unit quaternion, log-scales, sigmoid opacity */
    for (int k = 0; k < 4; ++k) p->q[k] = sc->quat[k * n + i];
    double qn = sqrt(p->q[0] * p->q[0] + p->q[1] * p->q[1] + p->q[2] * p->q[2] + p->q[3] * p->q[3]);
    if (!(qn > 0) || !isfinite(qn)) return;
    p->qn = qn;
    double qh[4] = { p->q[0] / qn, p->q[1] / qn, p->q[2] / qn, p->q[3] / qn };
    quat_to_rot(qh, p->R_q);
    for (int k = 0; k < 3; ++k) p->s[k] = exp(sc->log_scale[k * n + i]);
    /* Sigma_W = R_q diag(s^2) R_q^T */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += p->R_q[r * 3 + k] * p->s[k] * p->s[k] * p->R_q[c * 3 + k];
            p->Sigma_w[r * 3 + c] = acc;
        }
    p->o = 1.0 / (1.0 + exp(-sc->opacity_logit[i]));

    /* camera transform mu_C = R mu_W + t (world-to-camera) */
    const double *R = pose, *t = pose + 9;
    double mw[3] = { sc->mean[i], sc->mean[n + i], sc->mean[2 * n + i] };
    for (int r = 0; r < 3; ++r)
        p->mc[r] = R[r * 3] * mw[0] + R[r * 3 + 1] * mw[1] + R[r * 3 + 2] * mw[2] + t[r];
    double x = p->mc[0], y = p->mc[1], z = p->mc[2];
    if (!(z > cfg->z_near) || !isfinite(x) || !isfinite(y) || !isfinite(z)) return;

    /* calibrated pinhole and its Jacobian at mu_C */
    p->u = cam->fx * x / z + cam->cx;
    p->v = cam->fy * y / z + cam->cy;
    p->J[0] = cam->fx / z; p->J[1] = 0;             p->J[2] = -cam->fx * x / (z * z);
    p->J[3] = 0;           p->J[4] = cam->fy / z;   p->J[5] = -cam->fy * y / (z * z);
    /* M = J R ; Sigma_I = M Sigma_W M^T + eps I */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            p->M[r * 3 + c] = p->J[r * 3] * R[c] + p->J[r * 3 + 1] * R[3 + c] + p->J[r * 3 + 2] * R[6 + c];
    double MS[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            MS[r * 3 + c] = p->M[r * 3] * p->Sigma_w[c] + p->M[r * 3 + 1] * p->Sigma_w[3 + c] +
                            p->M[r * 3 + 2] * p->Sigma_w[6 + c];
    double s00 = MS[0] * p->M[0] + MS[1] * p->M[1] + MS[2] * p->M[2];
    double s01 = MS[0] * p->M[3] + MS[1] * p->M[4] + MS[2] * p->M[5];
    double s11 = MS[3] * p->M[3] + MS[4] * p->M[4] + MS[5] * p->M[5];
    p->cov[0] = s00 + cfg->dilation;
    p->cov[1] = s01;
    p->cov[2] = s11 + cfg->dilation;
    p->det = p->cov[0] * p->cov[2] - p->cov[1] * p->cov[1];
    if (!(p->det > 0) || !isfinite(p->det)) return;
    p->conic[0] = p->cov[2] / p->det;
    p->conic[1] = -p->cov[1] / p->det;
    p->conic[2] = p->cov[0] / p->det;

    /* extent: alpha >= alpha_min  <=>  d^T Sigma_I^-1 d <= 2 ln(o / alpha_min) */
    if (cfg->alpha_min > 0) {
        if (!(p->o >= cfg->alpha_min)) return;
        double k = sqrt(2.0 * log(p->o / cfg->alpha_min));
        p->rx = k * sqrt(p->cov[0]);
        p->ry = k * sqrt(p->cov[2]);
    } else {
        p->rx = INFINITY;
        p->ry = INFINITY;
    }

    /* colour: RGB or SH evaluated at the direction from the camera centre */
    if (cfg->sh_degree < 0) {
        for (int c = 0; c < 3; ++c) p->rgb[c] = sc->colour[c * n + i];
    } else {
        /* camera centre o_c = -R^T t */
        double oc[3];
        for (int c = 0; c < 3; ++c) oc[c] = -(R[c] * t[0] + R[3 + c] * t[1] + R[6 + c] * t[2]);
        double d[3] = { mw[0] - oc[0], mw[1] - oc[1], mw[2] - oc[2] };
        double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (!(dn > 0)) return;
        p->dnorm = dn;
        for (int c = 0; c < 3; ++c) p->dir[c] = d[c] / dn;
        double Y[16], dY[16][3];
        sh_basis(cfg->sh_degree, p->dir, Y, dY);
        int K = sh_count(cfg->sh_degree);
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < K; ++k) acc += sc->colour[(k * 3 + c) * n + i] * Y[k];
            p->rgb[c] = acc;
        }
    }

    /* conservative tile rectangle of the extent box, clipped to the image */
    int tiles_x = (cam->width + cfg->tile_w - 1) / cfg->tile_w;
    int tiles_y = (cam->height + cfg->tile_h - 1) / cfg->tile_h;
    double fx0 = floor((p->u - p->rx) / cfg->tile_w), fx1 = floor((p->u + p->rx) / cfg->tile_w);
    double fy0 = floor((p->v - p->ry) / cfg->tile_h), fy1 = floor((p->v + p->ry) / cfg->tile_h);
    if (!isfinite(p->u) || !isfinite(p->v)) return;
    p->valid = 1;
    if (fx1 < 0 || fy1 < 0 || fx0 > tiles_x - 1 || fy0 > tiles_y - 1) return; /* empty rect */
    p->tx0 = fx0 < 0 ? 0 : (int)fx0;
    p->ty0 = fy0 < 0 ? 0 : (int)fy0;
    p->tx1 = fx1 > tiles_x - 1 ? tiles_x - 1 : (int)fx1;
    p->ty1 = fy1 > tiles_y - 1 ? tiles_y - 1 : (int)fy1;
}

int or_project(const or_scene *sc, const or_camera *cam, const double *pose,
               const or_config *cfg, double *out)
{
    for (int64_t i = 0; i < sc->n; ++i) {
        proj_t p;
        project_one(sc, i, cam, pose, cfg, &p);
        double *o = out + i * OP_NFIELDS;
        o[OP_VALID] = p.valid;
        o[OP_U] = p.u; o[OP_V] = p.v;
        o[OP_A] = p.conic[0]; o[OP_B] = p.conic[1]; o[OP_C] = p.conic[2];
        o[OP_O] = p.o;
        o[OP_R] = p.rgb[0]; o[OP_G] = p.rgb[1]; o[OP_BL] = p.rgb[2];
        o[OP_DEPTH] = p.mc[2];
        o[OP_RX] = p.rx; o[OP_RY] = p.ry;
        o[OP_COVA] = p.cov[0]; o[OP_COVB] = p.cov[1]; o[OP_COVC] = p.cov[2];
        o[OP_MCX] = p.mc[0]; o[OP_MCY] = p.mc[1]; o[OP_MCZ] = p.mc[2];
        o[OP_TX0] = p.tx0; o[OP_TY0] = p.ty0; o[OP_TX1] = p.tx1; o[OP_TY1] = p.ty1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* per-view tile lists sorted front to back                                  */

typedef struct {
    int64_t n_tiles, tiles_x, tiles_y;
    int64_t *start;   /* [n_tiles + 1] */
    int64_t *items;   /* Gaussian indices */
} tile_lists;

/* Front-to-back order of a tile list (Eq. (alpha): N(p) sorted near to far).
 * The order is an integer decision; it is taken on the float32 key the
 * renderer's records carry (FP32 throughout): the camera depth rounded once
 * to float32, ties broken by Gaussian index. */
static int cmp_depth_id(const void *a, const void *b, void *ctx)
{
    const proj_t *P = (const proj_t *)ctx;
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    float da = (float)P[ia].mc[2], db = (float)P[ib].mc[2];
    if (da < db) return -1;
    if (da > db) return 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

static int build_lists(const proj_t *P, int64_t n, const or_camera *cam, const or_config *cfg,
                       tile_lists *L)
{
    L->tiles_x = (cam->width + cfg->tile_w - 1) / cfg->tile_w;
    L->tiles_y = (cam->height + cfg->tile_h - 1) / cfg->tile_h;
    L->n_tiles = L->tiles_x * L->tiles_y;
    L->start = (int64_t *)calloc((size_t)L->n_tiles + 1, sizeof(int64_t));
    if (!L->start) return -1;
    for (int64_t i = 0; i < n; ++i) {
        const proj_t *p = &P[i];
        if (!p->valid) continue;
        for (int ty = p->ty0; ty <= p->ty1; ++ty)
            for (int tx = p->tx0; tx <= p->tx1; ++tx) L->start[ty * L->tiles_x + tx + 1]++;
    }
    for (int64_t t = 0; t < L->n_tiles; ++t) L->start[t + 1] += L->start[t];
    L->items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L->start[L->n_tiles] + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)L->n_tiles);
    if (!L->items || !fill) return -1;
    memcpy(fill, L->start, sizeof(int64_t) * (size_t)L->n_tiles);
    for (int64_t i = 0; i < n; ++i) {
        const proj_t *p = &P[i];
        if (!p->valid) continue;
        for (int ty = p->ty0; ty <= p->ty1; ++ty)
            for (int tx = p->tx0; tx <= p->tx1; ++tx) L->items[fill[ty * L->tiles_x + tx]++] = i;
    }
    free(fill);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < L->n_tiles; ++t)
        qsort_r(L->items + L->start[t], (size_t)(L->start[t + 1] - L->start[t]), sizeof(int64_t),
                cmp_depth_id, (void *)P);
    return 0;
}

static void free_lists(tile_lists *L)
{
    free(L->start);
    free(L->items);
}

/* ------------------------------------------------------------------------ */
/* per-pixel compositing, Eq. (alpha)                                        */

typedef struct {
    int64_t id;
    double alpha, T, G, dx, dy;
    int clamped;
} blend_t;

static double rel_margin(double a, double b)
{
    return fabs(a - b) / (fabs(b) > 0 ? fabs(b) : 1.0);
}

/* Tolerance model for the tests; no rendered value depends on it.  A bound
 * on the error of the exp2-space power p2 = log2(G) when a renderer forms it
 * in float32 from the quadratic form expanded about the centre (xc, yc) of
 * the pixel's tile: with o = (xc, yc) - (u, v), d = pixel - (xc, yc) and
 * k = log2(e) / 2,
 *   p2 = -k (o + d)^T conic (o + d) = c0 + g.d + d^T (-k conic) d,
 * the six coefficients (c0, g, -k conic) each rounded once to float32, and
 * the sum formed by five fused multiply-adds (two along the pixel's column
 * offset dx, one for the dy coefficient, two along dy).  With S the sum of
 * the six terms' magnitudes, the coefficients' roundings err by at most u S
 * (u = 2^-24), the four inner multiply-adds by at most 2 u S (each rounds a
 * partial sum of terms, each term counted at most twice), and the last one by
 * u |p2|: |d p2| <= 3 u S + u |p2|. */
static double power2_abs_error(const proj_t *p, double px, double py, double xc, double yc, double p2,
                               int staging_f32)
{
    const double u = 0x1p-24, k = 0.72134752044448170; /* log2(e) / 2 */
    const double A = p->conic[0], B = p->conic[1], C = p->conic[2];
    const double ox = xc - p->u, oy = yc - p->v, dx = px - xc, dy = py - yc;
    const double S = k * (A * ox * ox + 2.0 * B * ox * oy + C * oy * oy) +
                     2.0 * k * (fabs(A * ox + B * oy) * fabs(dx) + fabs(B * ox + C * oy) * fabs(dy)) +
                     k * (A * dx * dx + 2.0 * fabs(B * dx * dy) + C * dy * dy);
    double e = 3.0 * u * S + u * fabs(p2);
    if (staging_f32) {
        /* the centre (u, v) and the conic rounded to float32 before the
         * expansion: p2 = -k f^T conic f with f = pixel - centre moves by
         * 2 k |(conic f)_x| |du| + 2 k |(conic f)_y| |dv| (|du| <= u |u|)
         * and by k (A fx^2 + 2 |B fx fy| + C fy^2) u for the conic */
        const double fx = px - p->u, fy = py - p->v;
        e += u * (2.0 * k * (fabs(A * fx + B * fy) * fabs(p->u) + fabs(B * fx + C * fy) * fabs(p->v)) +
                  k * (A * fx * fx + 2.0 * fabs(B * fx * fy) + C * fy * fy));
    }
    return e;
}

/* The bound above for a Gaussian given by (u, v, conic), exported for the
 * test that checks it against an emulated float32 evaluation. */
double or_power2_error(double u, double v, double A, double B, double C, double px, double py,
                       double xc, double yc, double p2, int32_t staging_f32)
{
    proj_t p;
    memset(&p, 0, sizeof(p));
    p.u = u;
    p.v = v;
    p.conic[0] = A;
    p.conic[1] = B;
    p.conic[2] = C;
    return power2_abs_error(&p, px, py, xc, yc, p2, staging_f32);
}

/* Composites one pixel; fills rec[] (if non-NULL) with the blended entries.
 * Returns the number of blended entries; *n_pos = list position + 1 of the
 * last blended entry; *margin = smallest relative distance of any decision
 * taken (alpha_min skip, alpha_max clamp, early stop) from its threshold;
 * *clear = smallest ratio, over the same decisions, of that distance to the
 * float32 error bound of the quantity compared (from power2_abs_error for alpha;
 * for T, the bound accumulated over the blends before it, each adding one
 * rounding and alpha / (1 - alpha) times alpha's bound; the float32 rounding
 * of each threshold adds u).  A pixel with *clear > 1 takes every decision
 * the same way in float32 as here. */
static int64_t composite_pixel(const proj_t *P, const int64_t *list, int64_t len, double px,
                               double py, double xc, double yc, const or_config *cfg, double rgb[3],
                               double *T_out, int64_t *n_pos, double *margin, double *clear,
                               blend_t *rec)
{
    const double u32 = 0x1p-24;
    double T = 1.0, C[3] = { 0, 0, 0 }, m = INFINITY, cl = INFINITY, eT = 0.0;
    int64_t nb = 0, last = 0;
    for (int64_t k = 0; k < len; ++k) {
        const proj_t *p = &P[list[k]];
        double dx = px - p->u, dy = py - p->v;
        double power = -0.5 * (p->conic[0] * dx * dx + p->conic[2] * dy * dy) - p->conic[1] * dx * dy;
        double G = exp(power);
        double a_raw = p->o * G;
        double alpha = a_raw < cfg->alpha_max ? a_raw : cfg->alpha_max;
        /* relative error bounds: of alpha = o 2^p2 (p2's error, the
         * exponential within 2 ulp, the opacity's and the product's
         * roundings), and of the alpha_min test, taken as p2 >= log2(alpha_min
         * / o) in float32 (the threshold's, the opacity's and the quotient's
         * roundings, the logarithm within 2 ulp of its value) */
        const double ln2 = 0.69314718055994531;
        double e_p2 = clear ? power2_abs_error(p, px, py, xc, yc, power * 1.4426950408889634, cfg->staging_f32)
                            : 0.0;
        double ea = ln2 * e_p2 + 4.0 * u32;
        if (cfg->alpha_min > 0) {
            double mm = rel_margin(a_raw, cfg->alpha_min);
            if (mm < m) m = mm;
            if (clear) {
                double e = ln2 * e_p2 + 3.0 * u32 + 2.0 * ln2 * u32 * fabs(log2(cfg->alpha_min / p->o));
                if (mm / e < cl) cl = mm / e;
            }
        }
        if (alpha < cfg->alpha_min) continue;
        {
            double mm = rel_margin(a_raw, cfg->alpha_max);
            if (mm < m) m = mm;
            if (clear && cfg->alpha_max < 1.0 && mm / (ea + u32) < cl) cl = mm / (ea + u32);
        }
        double Tn = T * (1.0 - alpha);
        double ga = alpha < 1.0 ? alpha / (1.0 - alpha) : INFINITY;
        if (cfg->T_min > 0) {
            double mm = rel_margin(Tn, cfg->T_min);
            if (mm < m) m = mm;
            if (clear) {
                double e = eT + 2.0 * u32 + ga * ea;
                if (mm / e < cl) cl = mm / e;
            }
        }
        if (Tn < cfg->T_min) break;
        eT += u32 + ga * ea;
        if (rec) {
            rec[nb].id = list[k];
            rec[nb].alpha = alpha;
            rec[nb].T = T;
            rec[nb].G = G;
            rec[nb].dx = dx;
            rec[nb].dy = dy;
            rec[nb].clamped = !(a_raw < cfg->alpha_max);
        }
        for (int c = 0; c < 3; ++c) C[c] += p->rgb[c] * alpha * T;
        T = Tn;
        nb++;
        last = k + 1;
    }
    for (int c = 0; c < 3; ++c) rgb[c] = C[c] + T * cfg->bg[c];
    *T_out = T;
    *n_pos = last;
    if (margin) *margin = m;
    if (clear) *clear = cl;
    return nb;
}

static int64_t view_pixel_offset(const or_camera *cams, int32_t v)
{
    int64_t off = 0;
    for (int32_t u = 0; u < v; ++u) off += (int64_t)cams[u].width * cams[u].height;
    return off;
}

/* Forward render of n_views views.  Images are concatenated per view, each
 * view stored as [3][H][W]; T_final, n_contrib, n_blend, margin, clear as
 * [H][W] (n_contrib, n_blend, margin and clear may be NULL).  Pixel rows run
 * in parallel; every pixel is computed on its own. */
int or_render(const or_scene *sc, int32_t n_views, const or_camera *cams, const double *poses,
              const or_config *cfg, double *rgb, double *T_final, int32_t *n_contrib,
              int32_t *n_blend, double *margin, double *clear)
{
    int64_t n = sc->n;
    proj_t *P = (proj_t *)malloc(sizeof(proj_t) * (size_t)(n > 0 ? n : 1));
    if (!P) return -1;
    for (int32_t v = 0; v < n_views; ++v) {
        const or_camera *cam = &cams[v];
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) project_one(sc, i, cam, poses + 12 * v, cfg, &P[i]);
        tile_lists L;
        if (build_lists(P, n, cam, cfg, &L)) { free(P); return -1; }
        int64_t W = cam->width, H = cam->height, off = view_pixel_offset(cams, v);
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t py = 0; py < H; ++py)
            for (int64_t px = 0; px < W; ++px) {
                int64_t tyi = py / cfg->tile_h, txi = px / cfg->tile_w;
                int64_t t = tyi * L.tiles_x + txi;
                double xc = (double)(txi * cfg->tile_w) + 0.5 * cfg->tile_w;
                double yc = (double)(tyi * cfg->tile_h) + 0.5 * cfg->tile_h;
                double c3[3], T, m, cl;
                int64_t npos;
                int64_t nb = composite_pixel(P, L.items + L.start[t], L.start[t + 1] - L.start[t],
                                             px + 0.5, py + 0.5, xc, yc, cfg, c3, &T, &npos, &m,
                                             clear ? &cl : NULL, NULL);
                int64_t pix = py * W + px;
                for (int c = 0; c < 3; ++c) rgb[3 * off + c * W * H + pix] = c3[c];
                T_final[off + pix] = T;
                if (n_contrib) n_contrib[off + pix] = (int32_t)npos;
                if (n_blend) n_blend[off + pix] = (int32_t)nb;
                if (margin) margin[off + pix] = m;
                if (clear) clear[off + pix] = cl;
            }
        free_lists(&L);
    }
    free(P);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* backward                                                                  */

/* grad2d fields per (view, Gaussian) */
enum { G_U, G_V, G_A, G_B, G_C, G_O, G_R, G_G, G_BL, G_N };

/* Projection backward of one Gaussian in one view: from the screen-space
 * gradient g2[9] to parameter gradients (accumulated when acc_params) and the
 * pose-tangent gradient dxi[6] = (rho, omega). */
static void project_backward(const or_scene *sc, int64_t i, const double *pose, const or_camera *cam,
                             const or_config *cfg, const proj_t *p, const double g2[9],
                             int acc_params, double *d_mean, double *d_quat, double *d_log_scale,
                             double *d_opacity_logit, double *d_colour, double dxi[6])
{
    int64_t n = sc->n;
    const double *R = pose;
    double x = p->mc[0], y = p->mc[1], z = p->mc[2];
    double fx = cam->fx, fy = cam->fy;

    /* conic (A, B, C) = (c, -b, a) / det  ->  d(a, b, c) */
    double a = p->cov[0], b = p->cov[1], c = p->cov[2], D = p->det, D2 = D * D;
    double dA = g2[G_A], dB = g2[G_B], dC = g2[G_C];
    double da = dA * (-c * c / D2) + dB * (b * c / D2) + dC * (1.0 / D - a * c / D2);
    double db = dA * (2.0 * b * c / D2) + dB * (-1.0 / D - 2.0 * b * b / D2) + dC * (2.0 * a * b / D2);
    double dc = dA * (1.0 / D - a * c / D2) + dB * (a * b / D2) + dC * (-a * a / D2);
    /* symmetric gradient matrix of Sigma_I (b appears twice) */
    double Gm[4] = { da, 0.5 * db, 0.5 * db, dc };

    /* Sigma_I = M Sigma_W M^T: dSigma_W = M^T G M, dM = 2 G M Sigma_W */
    double dSw[9];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            double acc = 0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) acc += p->M[k * 3 + r] * Gm[k * 2 + l] * p->M[l * 3 + q];
            dSw[r * 3 + q] = acc;
        }
    double GM[6], dM[6];
    for (int k = 0; k < 2; ++k)
        for (int q = 0; q < 3; ++q) GM[k * 3 + q] = Gm[k * 2] * p->M[q] + Gm[k * 2 + 1] * p->M[3 + q];
    for (int k = 0; k < 2; ++k)
        for (int q = 0; q < 3; ++q) {
            double acc = 0;
            for (int l = 0; l < 3; ++l) acc += GM[k * 3 + l] * p->Sigma_w[l * 3 + q];
            dM[k * 3 + q] = 2.0 * acc;
        }
    /* M = J R: dJ = dM R^T, dR_cam = J^T dM */
    double dJ[6], dRc[9];
    for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 3; ++l)
            dJ[k * 3 + l] = dM[k * 3] * R[l * 3] + dM[k * 3 + 1] * R[l * 3 + 1] + dM[k * 3 + 2] * R[l * 3 + 2];
    for (int l = 0; l < 3; ++l)
        for (int q = 0; q < 3; ++q) dRc[l * 3 + q] = p->J[l] * dM[q] + p->J[3 + l] * dM[3 + q];

    /* J(mu_C) and (u, v)(mu_C) -> d mu_C */
    double dmc[3];
    dmc[0] = dJ[2] * (-fx / (z * z)) + g2[G_U] * (fx / z);
    dmc[1] = dJ[5] * (-fy / (z * z)) + g2[G_V] * (fy / z);
    dmc[2] = dJ[0] * (-fx / (z * z)) + dJ[2] * (2.0 * fx * x / (z * z * z)) + dJ[4] * (-fy / (z * z)) +
             dJ[5] * (2.0 * fy * y / (z * z * z)) + g2[G_U] * (-fx * x / (z * z)) +
             g2[G_V] * (-fy * y / (z * z));

    /* world mean via mu_C = R mu_W + t */
    double dmw[3];
    for (int q = 0; q < 3; ++q) dmw[q] = R[q] * dmc[0] + R[3 + q] * dmc[1] + R[6 + q] * dmc[2];

    /* pose tangent, Eq. (muCjac) and the rotation term of Eq. (sigmaIjac):
     * d rho = d mu_C, d omega = mu_C x d mu_C + vee(P - P^T), P = dR_cam R^T */
    double Pm[9];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
            Pm[r * 3 + q] = dRc[r * 3] * R[q * 3] + dRc[r * 3 + 1] * R[q * 3 + 1] + dRc[r * 3 + 2] * R[q * 3 + 2];
    dxi[0] += dmc[0];
    dxi[1] += dmc[1];
    dxi[2] += dmc[2];
    dxi[3] += y * dmc[2] - z * dmc[1] + (Pm[7] - Pm[5]);
    dxi[4] += z * dmc[0] - x * dmc[2] + (Pm[2] - Pm[6]);
    dxi[5] += x * dmc[1] - y * dmc[0] + (Pm[3] - Pm[1]);

    /* colour */
    double dcol[3] = { g2[G_R], g2[G_G], g2[G_BL] };
    if (cfg->sh_degree >= 0) {
        double Y[16], dY[16][3];
        sh_basis(cfg->sh_degree, p->dir, Y, dY);
        int K = sh_count(cfg->sh_degree);
        double gdir[3] = { 0, 0, 0 };
        for (int k = 0; k < K; ++k)
            for (int ch = 0; ch < 3; ++ch) {
                double coef = sc->colour[(k * 3 + ch) * n + i];
                for (int q = 0; q < 3; ++q) gdir[q] += dcol[ch] * coef * dY[k][q];
            }
        /* dir = d / |d|, d = mu_W - o_c */
        double dot = gdir[0] * p->dir[0] + gdir[1] * p->dir[1] + gdir[2] * p->dir[2];
        double dd[3];
        for (int q = 0; q < 3; ++q) dd[q] = (gdir[q] - p->dir[q] * dot) / p->dnorm;
        for (int q = 0; q < 3; ++q) dmw[q] += dd[q];
        /* o_c = -R^T t moves by -R^T rho under the left twist: d rho += R dd */
        for (int r = 0; r < 3; ++r) dxi[r] += R[r * 3] * dd[0] + R[r * 3 + 1] * dd[1] + R[r * 3 + 2] * dd[2];
        if (acc_params)
            for (int k = 0; k < K; ++k)
                for (int ch = 0; ch < 3; ++ch) d_colour[(k * 3 + ch) * n + i] += dcol[ch] * Y[k];
    } else if (acc_params) {
        for (int ch = 0; ch < 3; ++ch) d_colour[ch * n + i] += dcol[ch];
    }
    if (!acc_params) return;

    for (int q = 0; q < 3; ++q) d_mean[q * n + i] += dmw[q];
    d_opacity_logit[i] += g2[G_O] * p->o * (1.0 - p->o);

    /* Sigma_W = R_q diag(s^2) R_q^T */
    for (int k = 0; k < 3; ++k) {
        double acc = 0;
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) acc += p->R_q[r * 3 + k] * dSw[r * 3 + q] * p->R_q[q * 3 + k];
        d_log_scale[k * n + i] += 2.0 * p->s[k] * p->s[k] * acc;
    }
    double dRq[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0;
            for (int q = 0; q < 3; ++q) acc += dSw[r * 3 + q] * p->R_q[q * 3 + k];
            dRq[r * 3 + k] = 2.0 * acc * p->s[k] * p->s[k];
        }
    double qh[4] = { p->q[0] / p->qn, p->q[1] / p->qn, p->q[2] / p->qn, p->q[3] / p->qn };
    double pd[4][9];
    quat_to_rot_partials(qh, pd);
    double dqh[4];
    for (int k = 0; k < 4; ++k) {
        double acc = 0;
        for (int e = 0; e < 9; ++e) acc += dRq[e] * pd[k][e];
        dqh[k] = acc;
    }
    /* through the normalisation q_hat = q / |q| */
    double dot = dqh[0] * qh[0] + dqh[1] * qh[1] + dqh[2] * qh[2] + dqh[3] * qh[3];
    for (int k = 0; k < 4; ++k) d_quat[k * n + i] += (dqh[k] - qh[k] * dot) / p->qn;
}

/* Backward of or_render for an upstream gradient dL_drgb (same layout as
 * rgb) and optionally dL_dT (same layout as T_final).  Parameter gradients are
 * overwritten and summed over the views whose pose_only flag is 0; d_xi [V][6]
 * receives the gradient at xi = 0 of T(xi) = exp(xi^) T, xi = (rho, omega).
 * grad2d (nullable) receives the screen-space gradient [V][n][9]. */
int or_backward(const or_scene *sc, int32_t n_views, const or_camera *cams, const double *poses,
                const or_config *cfg, const double *dL_drgb, const double *dL_dT,
                const uint8_t *pose_only, double *d_mean, double *d_quat, double *d_log_scale,
                double *d_opacity_logit, double *d_colour, double *d_xi, double *grad2d_out,
                double *grad2d_abs_out)
{
    int64_t n = sc->n;
    int K = cfg->sh_degree < 0 ? 1 : sh_count(cfg->sh_degree);
    memset(d_mean, 0, sizeof(double) * 3 * (size_t)n);
    memset(d_quat, 0, sizeof(double) * 4 * (size_t)n);
    memset(d_log_scale, 0, sizeof(double) * 3 * (size_t)n);
    memset(d_opacity_logit, 0, sizeof(double) * (size_t)n);
    memset(d_colour, 0, sizeof(double) * 3 * (size_t)K * (size_t)n);
    memset(d_xi, 0, sizeof(double) * 6 * (size_t)n_views);

    const int nthr = omp_get_max_threads();
    proj_t *P = (proj_t *)malloc(sizeof(proj_t) * (size_t)(n > 0 ? n : 1));
    double *g2 = (double *)malloc(sizeof(double) * G_N * (size_t)(n > 0 ? n : 1));
    /* per-thread screen-space gradients, summed in thread order after each view */
    double *g2t = (double *)malloc(sizeof(double) * G_N * (size_t)(n > 0 ? n : 1) * (size_t)nthr);
    double *xit = (double *)malloc(sizeof(double) * 6 * (size_t)nthr);
    /* optional: the sum of the magnitudes of the elementary products behind
     * each screen-space gradient (those of dL/dalpha included), per thread,
     * for the tests' cancellation measure */
    double *abt = grad2d_abs_out ? (double *)malloc(sizeof(double) * G_N * (size_t)(n > 0 ? n : 1) * (size_t)nthr)
                                 : NULL;
    if (!P || !g2 || !g2t || !xit || (grad2d_abs_out && !abt)) return -1;
    for (int32_t v = 0; v < n_views; ++v) {
        const or_camera *cam = &cams[v];
        const double *pose = poses + 12 * v;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) project_one(sc, i, cam, pose, cfg, &P[i]);
        tile_lists L;
        if (build_lists(P, n, cam, cfg, &L)) return -1;
        int64_t maxlen = 1;
        for (int64_t t = 0; t < L.n_tiles; ++t)
            if (L.start[t + 1] - L.start[t] > maxlen) maxlen = L.start[t + 1] - L.start[t];
        memset(g2t, 0, sizeof(double) * G_N * (size_t)n * (size_t)nthr);
        if (abt) memset(abt, 0, sizeof(double) * G_N * (size_t)n * (size_t)nthr);
        int64_t W = cam->width, H = cam->height, off = view_pixel_offset(cams, v);
        int failed = 0;
#pragma omp parallel num_threads(nthr)
        {
            const int tid = omp_get_thread_num();
            double *tg2 = g2t + (size_t)tid * G_N * (size_t)n;
            double *tab = abt ? abt + (size_t)tid * G_N * (size_t)n : NULL;
            blend_t *rec = (blend_t *)malloc(sizeof(blend_t) * (size_t)maxlen);
            if (!rec) {
#pragma omp atomic write
                failed = 1;
            }
#pragma omp for schedule(dynamic, 1)
            for (int64_t py = 0; py < H; ++py) {
                if (!rec) continue;
                for (int64_t px = 0; px < W; ++px) {
                    int64_t t = (py / cfg->tile_h) * L.tiles_x + px / cfg->tile_w;
                    double c3[3], Tf;
                    int64_t npos;
                    int64_t nb = composite_pixel(P, L.items + L.start[t], L.start[t + 1] - L.start[t],
                                                 px + 0.5, py + 0.5, 0.0, 0.0, cfg, c3, &Tf, &npos, NULL,
                                                 NULL, rec);
                    int64_t pix = py * W + px;
                    double g[3], gT = dL_dT ? dL_dT[off + pix] : 0.0;
                    for (int c = 0; c < 3; ++c) g[c] = dL_drgb[3 * off + c * W * H + pix];
                    /* suffix recursion: B = colour composited behind the entry,
                     * Q = product of (1 - alpha) after the entry */
                    double B[3] = { cfg->bg[0], cfg->bg[1], cfg->bg[2] }, Q = 1.0;
                    for (int64_t k = nb - 1; k >= 0; --k) {
                        const blend_t *e = &rec[k];
                        const proj_t *p = &P[e->id];
                        double *gg = tg2 + G_N * e->id;
                        double *ga = tab ? tab + G_N * e->id : NULL;
                        double dalpha = -gT * e->T * Q;
                        /* the magnitudes of dalpha's elementary products (its
                         * own cancellation enters the measure too) */
                        double dalpha_abs = fabs(gT * e->T * Q);
                        for (int c = 0; c < 3; ++c) {
                            gg[G_R + c] += g[c] * e->alpha * e->T;
                            if (ga) ga[G_R + c] += fabs(g[c] * e->alpha * e->T);
                            dalpha += g[c] * e->T * (p->rgb[c] - B[c]);
                            dalpha_abs += fabs(g[c] * e->T) * (fabs(p->rgb[c]) + fabs(B[c]));
                        }
                        for (int c = 0; c < 3; ++c) B[c] = p->rgb[c] * e->alpha + (1.0 - e->alpha) * B[c];
                        Q *= 1.0 - e->alpha;
                        if (e->clamped) continue; /* alpha = alpha_max: no dependence */
                        /* alpha = o exp(power) */
                        double dpow = dalpha * e->alpha;
                        gg[G_O] += dalpha * e->G;
                        gg[G_A] += dpow * (-0.5 * e->dx * e->dx);
                        gg[G_B] += dpow * (-e->dx * e->dy);
                        gg[G_C] += dpow * (-0.5 * e->dy * e->dy);
                        /* dx = px - u, dy = py - v */
                        gg[G_U] += dpow * (p->conic[0] * e->dx + p->conic[1] * e->dy);
                        gg[G_V] += dpow * (p->conic[1] * e->dx + p->conic[2] * e->dy);
                        if (ga) {
                            const double dpa = dalpha_abs * e->alpha;
                            ga[G_O] += dalpha_abs * e->G;
                            ga[G_A] += dpa * 0.5 * e->dx * e->dx;
                            ga[G_B] += dpa * fabs(e->dx * e->dy);
                            ga[G_C] += dpa * 0.5 * e->dy * e->dy;
                            ga[G_U] += dpa * (fabs(p->conic[0] * e->dx) + fabs(p->conic[1] * e->dy));
                            ga[G_V] += dpa * (fabs(p->conic[1] * e->dx) + fabs(p->conic[2] * e->dy));
                        }
                    }
                }
            }
            free(rec);
        }
        if (failed) return -1;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < G_N * n; ++j) {
            double acc = 0.0;
            for (int th = 0; th < nthr; ++th) acc += g2t[(size_t)th * G_N * (size_t)n + (size_t)j];
            g2[j] = acc;
        }
        free_lists(&L);
        if (grad2d_out) memcpy(grad2d_out + (size_t)v * n * G_N, g2, sizeof(double) * G_N * (size_t)n);
        if (grad2d_abs_out) {
            double *dst = grad2d_abs_out + (size_t)v * n * G_N;
#pragma omp parallel for schedule(static)
            for (int64_t j = 0; j < G_N * n; ++j) {
                double acc2 = 0.0;
                for (int th = 0; th < nthr; ++th) acc2 += abt[(size_t)th * G_N * (size_t)n + (size_t)j];
                dst[j] = acc2;
            }
        }
        int acc = !(pose_only && pose_only[v]);
        /* each Gaussian writes only its own parameter gradients; the pose
         * gradient is summed per thread, then in thread order */
        memset(xit, 0, sizeof(double) * 6 * (size_t)nthr);
#pragma omp parallel num_threads(nthr)
        {
            double *txi = xit + 6 * omp_get_thread_num();
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                if (!P[i].valid) continue;
                project_backward(sc, i, pose, cam, cfg, &P[i], g2 + G_N * i, acc, d_mean, d_quat,
                                 d_log_scale, d_opacity_logit, d_colour, txi);
            }
        }
        for (int th = 0; th < nthr; ++th)
            for (int k = 0; k < 6; ++k) d_xi[6 * v + k] += xit[6 * th + k];
    }
    free(abt);
    free(xit);
    free(g2t);
    free(g2);
    free(P);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* binning contract in float32                                               */

/* Binning of already-projected float32 records into (tile | depth) keys.
 * A slot is live iff rx >= 0, ry >= 0 and u and v are not NaN; the depth is
 * only a sort key (its raw float32 bit pattern).
 * Candidate tiles are those of the slot's rectangle, computed with
 * single-precision IEEE operations only:
 *   x0 = floor((u - rx) / tile_w), x1 = floor((u + rx) / tile_w)  (same in y),
 * empty if x1 < 0, y1 < 0, x0 > tiles_x - 1 or y0 > tiles_y - 1, otherwise
 * clipped to the view's tile grid.  A candidate tile is kept iff tile_hit()
 * finds the slot's quadratic form at or below its threshold qthr somewhere on
 * the box spanned by the tile's pixel centres.
 * Key = (global tile << 32) | bits(depth), value = slot index (view * n +
 * Gaussian); pairs are ordered by key, then slot; rectangle tiles are visited
 * row by row.  ranges[2 t], ranges[2 t + 1] = [first, last + 1) of global
 * tile t, or 0, 0.  Returns the number of pairs; writes at most `capacity`. */
static const uint64_t *g_bin_keys;
static int cmp_pair(const void *a, const void *b)
{
    uint32_t ia = *(const uint32_t *)a, ib = *(const uint32_t *)b;
    uint64_t ka = g_bin_keys[ia], kb = g_bin_keys[ib];
    if (ka != kb) return ka < kb ? -1 : 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

/* q(dx, dy) = A dx^2 + 2 B dx dy + C dy^2, d = pixel centre - (u, v): is its
 * minimum over the box of the tile's pixel centres <= qthr?  Inside the box
 * the minimum is 0; otherwise it lies on an edge, where the minimiser along
 * the edge is clamped to the edge.  Float32 operations in this exact order. */
static int tile_hit(float u, float v, float A, float B, float C, float qthr, int64_t tx, int64_t ty,
                    int32_t tw, int32_t th)
{
    float x0 = ((float)(tx * tw) + 0.5f) - u;
    float x1 = ((float)(tx * tw + tw - 1) + 0.5f) - u;
    float y0 = ((float)(ty * th) + 0.5f) - v;
    float y1 = ((float)(ty * th + th - 1) + 0.5f) - v;
    if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return 1;
    float iA = 1.0f / A, iC = 1.0f / C, B2 = 2.0f * B;
    float m = INFINITY;
    float ex[2] = { x0, x1 }, ey[2] = { y0, y1 };
    for (int e = 0; e < 2; ++e) {
        float X = ex[e];
        float ys = -(B * X) * iC;
        ys = ys < y0 ? y0 : (ys > y1 ? y1 : ys);
        float q = (A * X) * X + (B2 * X) * ys + (C * ys) * ys;
        m = q < m ? q : m;
    }
    for (int e = 0; e < 2; ++e) {
        float Y = ey[e];
        float xs = -(B * Y) * iA;
        xs = xs < x0 ? x0 : (xs > x1 ? x1 : xs);
        float q = (A * xs) * xs + (B2 * xs) * Y + (C * Y) * Y;
        m = q < m ? q : m;
    }
    return m <= qthr;
}

int64_t or_bin_f32(int32_t n_views, const int32_t *widths, const int32_t *heights, int64_t n,
                   const float *u, const float *v, const float *rx, const float *ry,
                   const float *A, const float *B, const float *C, const float *qthr,
                   const float *depth, int32_t tile_w, int32_t tile_h, int64_t capacity,
                   uint64_t *keys, uint32_t *vals, uint32_t *ranges)
{
    int64_t total_tiles = 0;
    int64_t *base = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_views + 1));
    for (int32_t w = 0; w < n_views; ++w) {
        base[w] = total_tiles;
        total_tiles += (int64_t)((widths[w] + tile_w - 1) / tile_w) * ((heights[w] + tile_h - 1) / tile_h);
    }
    base[n_views] = total_tiles;
    /* pass 1: count */
    int64_t M = 0;
    for (int32_t w = 0; w < n_views; ++w) {
        int tiles_x = (widths[w] + tile_w - 1) / tile_w, tiles_y = (heights[w] + tile_h - 1) / tile_h;
        for (int64_t i = 0; i < n; ++i) {
            int64_t s = (int64_t)w * n + i;
            float uu = u[s], vv = v[s], rxx = rx[s], ryy = ry[s];
            if (!(rxx >= 0.0f) || !(ryy >= 0.0f) || uu != uu || vv != vv) continue;
            float x0 = floorf((uu - rxx) / (float)tile_w), x1 = floorf((uu + rxx) / (float)tile_w);
            float y0 = floorf((vv - ryy) / (float)tile_h), y1 = floorf((vv + ryy) / (float)tile_h);
            if (x1 < 0.0f || y1 < 0.0f || x0 > (float)(tiles_x - 1) || y0 > (float)(tiles_y - 1)) continue;
            int64_t tx0 = x0 < 0.0f ? 0 : (int64_t)x0, ty0 = y0 < 0.0f ? 0 : (int64_t)y0;
            int64_t tx1 = x1 > (float)(tiles_x - 1) ? tiles_x - 1 : (int64_t)x1;
            int64_t ty1 = y1 > (float)(tiles_y - 1) ? tiles_y - 1 : (int64_t)y1;
            for (int64_t ty = ty0; ty <= ty1; ++ty)
                for (int64_t tx = tx0; tx <= tx1; ++tx)
                    M += tile_hit(uu, vv, A[s], B[s], C[s], qthr[s], tx, ty, tile_w, tile_h);
        }
    }
    uint64_t *k_all = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(M + 1));
    uint32_t *v_all = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(M + 1));
    uint32_t *idx = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(M + 1));
    int64_t m = 0;
    for (int32_t w = 0; w < n_views; ++w) {
        int tiles_x = (widths[w] + tile_w - 1) / tile_w, tiles_y = (heights[w] + tile_h - 1) / tile_h;
        for (int64_t i = 0; i < n; ++i) {
            int64_t s = (int64_t)w * n + i;
            float uu = u[s], vv = v[s], rxx = rx[s], ryy = ry[s], dd = depth[s];
            if (!(rxx >= 0.0f) || !(ryy >= 0.0f) || uu != uu || vv != vv) continue;
            float x0 = floorf((uu - rxx) / (float)tile_w), x1 = floorf((uu + rxx) / (float)tile_w);
            float y0 = floorf((vv - ryy) / (float)tile_h), y1 = floorf((vv + ryy) / (float)tile_h);
            if (x1 < 0.0f || y1 < 0.0f || x0 > (float)(tiles_x - 1) || y0 > (float)(tiles_y - 1)) continue;
            int64_t tx0 = x0 < 0.0f ? 0 : (int64_t)x0, ty0 = y0 < 0.0f ? 0 : (int64_t)y0;
            int64_t tx1 = x1 > (float)(tiles_x - 1) ? tiles_x - 1 : (int64_t)x1;
            int64_t ty1 = y1 > (float)(tiles_y - 1) ? tiles_y - 1 : (int64_t)y1;
            uint32_t bits;
            memcpy(&bits, &dd, 4);
            for (int64_t ty = ty0; ty <= ty1; ++ty)
                for (int64_t tx = tx0; tx <= tx1; ++tx) {
                    if (!tile_hit(uu, vv, A[s], B[s], C[s], qthr[s], tx, ty, tile_w, tile_h)) continue;
                    uint64_t tile = (uint64_t)(base[w] + ty * tiles_x + tx);
                    k_all[m] = (tile << 32) | bits;
                    v_all[m] = (uint32_t)s;
                    idx[m] = (uint32_t)m;
                    m++;
                }
        }
    }
    /* comparator sort: key ascending, then emission order (= slot ascending) */
    g_bin_keys = k_all;
    qsort(idx, (size_t)M, sizeof(uint32_t), cmp_pair);
    for (int64_t t = 0; t < 2 * total_tiles; ++t) ranges[t] = 0;
    for (int64_t j = 0; j < M; ++j) {
        uint64_t key = k_all[idx[j]];
        uint64_t tile = key >> 32;
        if (j < capacity) {
            keys[j] = key;
            vals[j] = v_all[idx[j]];
        }
        if (j == 0 || (k_all[idx[j - 1]] >> 32) != tile) ranges[2 * tile] = (uint32_t)j;
        if (j == M - 1 || (k_all[idx[j + 1]] >> 32) != tile) ranges[2 * tile + 1] = (uint32_t)(j + 1);
    }
    free(k_all);
    free(v_all);
    free(idx);
    free(base);
    return M;
}
