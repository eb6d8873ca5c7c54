/*
 * gsr.h -- C ABI of libgsr, an MI355X (gfx950) differentiable tile-based
 * 3D Gaussian-splatting rasterizer: the renderer that RGS-SLAM
 * (arXiv 2601.00705) optimises during tracking and mapping.
 *
 * The operations follow the paper:
 *   - gsr_project: Eq. (proj) of Sec. "Gaussian Splatting Representation":
 *     mu_I = pi(R mu_W + t), Sigma_I = J R Sigma_W R^T J^T (J the pinhole
 *     Jacobian at mu_C), with Sigma_W = R_q diag(s^2) R_q^T from a unit
 *     quaternion and log-scales (appendix, Gaussian Splatting
 *     Representation) and colour as RGB or real SH, Eq. (app-sh).
 *   - gsr_bin: the front-to-back ordered sets N(p) of Eq. (alpha) ("sorted
 *     from near to far", Sec. Alpha Compositing for Color), built per tile.
 *   - gsr_render_fwd: alpha compositing, Eq. (alpha).
 *   - gsr_loss_l1: the gradient seed of the L1 photometric residual,
 *     Eq. (photometric).
 *   - gsr_loss_track: the tracking loss of the appendix (Tracking and Camera
 *     Pose Optimization), Eqs. (app-bright), (app-ls), (app-trackloss),
 *     (app-weight), and its gradient seed for gsr_render_bwd.
 *   - gsr_loss_mapping: the mapping loss of the appendix's optimisation
 *     settings, L1 plus lambda_dssim (1 - SSIM), and its gradient seed.
 *   - gsr_adam_step, gsr_covis, gsr_prune, gsr_compact, gsr_nearest,
 *     gsr_merge, gsr_keep_list: map maintenance,
 *     the optimiser step of the appendix's settings with the anchor of Eq.
 *     (app-ema), the co-visibility score of Eq. (iou), and the pruning rule
 *     and merging of Sec. "Insertion, Lightweight Merging, and Pruning".
 *   - gsr_spatial_order: a storage order of the map (a layout choice; the
 *     method's sums do not depend on it) under which projection waves and
 *     binning chunks hold Gaussians that are neighbours in space.
 *   - gsr_seed_triangulate, gsr_seed_scale, gsr_seed_frame: the one-shot
 *     Gaussian seeding of Sec. "Dense Feature Matching" (Eq. (conf),
 *     two-view linear triangulation) and the appendix's initialisation
 *     (Eqs. (app-sigma-init), (app-alpha-init), colour median), producing
 *     Gaussians in the layout gsr_project reads.
 *   - gsr_render_bwd: gradients for colour, opacity, mean, covariance
 *     parameters (the differentiability statement after Eq. (alpha)) and for
 *     the pose twist of Eq. (leftupdate), via Eqs. (muCjac), (muIjac),
 *     (sigmaIjac).
 *
 * Conventions (readings where the paper is silent):
 *   - pose: world-to-camera [R | t], 12 floats per view, R row-major then t;
 *     x_c = R x_w + t.
 *   - pose tangent xi = (rho, omega): T(xi) = exp(xi^) T, xi^ = [[omega]x rho;
 *     0 0]; gradients are taken at xi = 0.
 *   - pixel (px, py) is sampled at (px + 1/2, py + 1/2); the 2-D Gaussian is
 *     unnormalised (peak 1); Sigma_I gets + dilation * I.
 *   - alpha = min(alpha_max, o exp(-d^T Sigma_I^-1 d / 2)), o = sigmoid(logit);
 *     entries with alpha < alpha_min are skipped; compositing stops before an
 *     entry that would take the transmittance below T_min; output colour is
 *     C + T_final * bg.
 *   - ordering: camera-space depth z ascending, ties by Gaussian index.
 *   - SH: real basis without Condon-Shortley phase, index l*l + l + m, at the
 *     unit direction from the camera centre (-R^T t) to the world mean.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller
 * unless stated otherwise.  Parameter planes are structure-of-arrays:
 * mean [3][n], quat [4][n] (w, x, y, z, any non-zero norm), log_scale [3][n],
 * opacity_logit [n], colour [3][n] (RGB) or [K][3][n] (SH, K = (d+1)^2).
 * Images of the views are concatenated in view order; view v occupies
 * 3 * H_v * W_v floats laid out [3][H_v][W_v] (rgb, dL_drgb) or H_v * W_v
 * values [H_v][W_v] (T_final, n_contrib, n_blend, dL_dT).
 *
 * The library allocates no device memory and never synchronises, except
 * gsr_plan_bind and gsr_pair_count, which say so.  All work is enqueued on the
 * given stream (a hipStream_t; NULL = the null stream).  Calls on different
 * plans are independent; calls on one plan must be ordered by the caller.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_MAX_VIEWS 64
#define GSR_MAX_DEVICES 64   /* device indices the no-allocation entry point serves */

typedef enum {
    GSR_OK = 0,
    GSR_EINVAL = -1,       /* invalid argument; nothing was enqueued */
    GSR_ECAPACITY = -2,    /* pair capacity exceeded (see gsr_pair_count) */
    GSR_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
    GSR_EUNSUPPORTED = -4, /* valid but unsupported configuration */
    GSR_ESTATE = -5        /* plan not bound to a workspace */
} gsr_status;

/* Pinhole camera of one view (host struct). */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
} gsr_camera;

/* Renderer settings (host struct). */
typedef struct {
    int32_t tile_w, tile_h; /* powers of two, tile_w <= 64; tile_w * tile_h in
                               {64, 128, 256, 512} (1, 2, 4 or 8 pixels per lane) */
    int32_t batch;          /* records staged in LDS per step: 64, 128 or 256 (0 = 128) */
    int32_t sh_degree;      /* -1: RGB colour; 0..3: SH degree */
    float z_near;           /* cull mu_C.z <= z_near */
    float dilation;         /* eps added to the diagonal of Sigma_I (px^2) */
    float alpha_min;        /* skip threshold (0 disables it and the extent cull) */
    float alpha_max;        /* upper clamp, in (0, 1] */
    float T_min;            /* early-stop transmittance (0 disables it) */
    float bg[3];            /* background colour weighted by T_final */
    int32_t deterministic;  /* 1: the backward accumulates the screen-space
                               gradients exactly in fixed point (integer
                               atomics), so that every backward output is
                               bitwise reproducible whatever the order in
                               which tiles run; 0: FP64 atomics (reproducible
                               to ~1e-16 relative).  1 adds 288 bytes of
                               workspace per slot. */
    int32_t precision;      /* GSR_PRECISION_FP32 (0, the default) or
                               GSR_PRECISION_MIXED (1).  Mixed: the staging
                               record each tile reads per pair is 32 bytes
                               (float32 centre, conic and opacity, binary16
                               colour) instead of 64 (double centre and conic,
                               float32 opacity and colour), and gsr_render_fwd
                               writes, and gsr_loss_l1 reads, the image as
                               IEEE binary16; T_final, n_contrib and every
                               gradient stay float32.  gsr_loss_track and
                               gsr_loss_mapping need float32 images and return
                               GSR_EUNSUPPORTED for a mixed plan. */
} gsr_config;

#define GSR_PRECISION_FP32 0
#define GSR_PRECISION_MIXED 1

/* Gaussian parameters (device planes, see above). */
typedef struct {
    int64_t n;
    const float *mean, *quat, *log_scale, *opacity_logit, *colour;
} gsr_gaussians;

/* Parameter gradients (device planes with the shapes of gsr_gaussians).
 * Written, not accumulated; summed over the views that are not pose-only. */
typedef struct {
    float *d_mean, *d_quat, *d_log_scale, *d_opacity_logit, *d_colour;
} gsr_grads;

/* Byte offsets of the planes inside a bound workspace. */
typedef struct {
    size_t counters;  /* struct { uint64 pairs; uint32 overflow; ... } */
    size_t geom;      /* float4 [V*n]: (u, v, rx, ry); rx < 0 or NaN = culled */
    size_t conic_o;   /* float4 [V*n]: (A, B, C, o), A = (Sigma_I^-1)_00 ... */
    size_t rgb_d;     /* float4 [V*n]: (r, g, b, depth) */
    size_t qthr;      /* float [V*n]: binning level of d^T conic d per slot */
    size_t stage;     /* 64-byte records [V*n]: double u, v, A, B, C; float o, r, g, b
                         (unrounded centre and conic the compositing stages from);
                         mixed precision: 32-byte records float u, v, A, B, C, o;
                         binary16 r, g, b (same offset, half the bytes used) */
    size_t grad2d;    /* double [V*n][9]: d(u, v, A, B, C, o, r, g, b) per slot */
    size_t keys;      /* uint64 [capacity]: sorted (tile << 32 | depth bits) */
    size_t vals;      /* uint32 [capacity]: sorted slot = view * n + index */
    size_t ranges;    /* uint32 [tiles][2]: [first, last + 1) per global tile */
    size_t stamps;    /* uint64 [V + 1]: device wall-clock ticks (see
                         gsr_device_clock_hz) at which the last backward tile
                         of view v finished, for v < V, and at which the last
                         gsr_project began, at [V]: per-view latency of a step */
    size_t live_mask; /* uint64 [ceil(n / 64)][V]: bit k of word [w][v] set
                         when slot (v, 64 w + k) is live: its tile rectangle
                         is not empty (written by gsr_project, read by gsr_bin) */
    size_t total;     /* workspace bytes */
} gsr_layout;

/* Sizes derived by a plan (host struct). */
typedef struct {
    int64_t n, slots, capacity, total_pixels;
    int32_t n_views, total_tiles, sort_passes, tile_bits;
} gsr_plan_info;

typedef struct gsr_plan gsr_plan; /* opaque host object */

/* Creates a plan for n Gaussians rendered into n_views (1..GSR_MAX_VIEWS)
 * views.  cams: host array [n_views].  pair_capacity: maximum number of
 * (tile, Gaussian) pairs one binning may produce (< 2^32); the workspace
 * holds two key/value buffers of that size.  Requires n * n_views < 2^32.
 * Returns GSR_EINVAL on invalid arguments. */
gsr_status gsr_plan_create(int64_t n, int32_t n_views, const gsr_camera *cams, const gsr_config *cfg,
                           int64_t pair_capacity, gsr_plan **out);
void gsr_plan_destroy(gsr_plan *plan);

/* Workspace bytes the plan needs (256-byte aligned device memory). */
size_t gsr_plan_workspace_bytes(const gsr_plan *plan);

/* Binds a caller-owned device workspace of at least gsr_plan_workspace_bytes
 * bytes, uploads the view table and capacity into it, marks every slot
 * culled (NaN geom, clear live_mask; empty tile ranges), and synchronises
 * `stream` once.  The workspace must stay alive while the plan is used.  The
 * first bind also creates the plan's own second stream (non-blocking,
 * default priority) and two ordering events, released by
 * gsr_plan_destroy. */
gsr_status gsr_plan_bind(gsr_plan *plan, void *workspace, size_t bytes, void *stream);

gsr_status gsr_plan_layout(const gsr_plan *plan, gsr_layout *out);
gsr_status gsr_plan_get_info(const gsr_plan *plan, gsr_plan_info *out);

/* Eq. (proj): projects every Gaussian into every view (poses: device
 * [n_views][12]), in double precision.  Writes the float geom / conic_o /
 * rgb_d / qthr records (correctly rounded) and the staging records of the
 * live slots, and zeroes their screen-space gradient accumulators.  A culled
 * slot's geom holds a culled marker (rx and ry -1, or NaN for a slot not
 * live at any projection since the workspace was bound); the projection
 * writes it only where live_mask shows the slot live before, so a caller
 * that writes geom itself keeps live_mask set for those slots. */
gsr_status gsr_project(gsr_plan *plan, const gsr_gaussians *g, const float *poses, void *stream);

/* Builds the depth-ordered per-tile lists from the geom / conic_o / qthr /
 * rgb_d records of the slots that live_mask marks (candidate tiles: the
 * slot's rectangle; kept: the tiles whose pixel-centre box reaches
 * d^T conic d <= qthr).  gsr_project writes the records and the mask; a
 * caller that writes records itself also sets the mask bit of every slot
 * with a non-empty rectangle (other bits add no pair):
 * pair emission, stable LSD radix sort of (tile | depth) keys with slot
 * values, tile ranges.  When the pair count exceeds the capacity, a device
 * flag is set, no pair is written, gsr_render_fwd writes NaN images and
 * gsr_render_bwd writes NaN gradients; gsr_pair_count reports it.  The sort
 * of segments longer than 8192 pairs runs on the plan's second stream,
 * forked from `stream` after the tile ranges and joined back before gsr_bin
 * returns its work to `stream` (the fork and join are recorded too when
 * `stream` is being captured into a graph). */
gsr_status gsr_bin(gsr_plan *plan, void *stream);

/* Eq. (alpha) for every view.  rgb, T_final, n_contrib required; n_blend
 * (number of blended entries per pixel) may be NULL.  n_contrib is the list
 * position + 1 of the last blended entry of the pixel's tile list; it is
 * what gsr_render_bwd replays.  rgb holds float32 values, or IEEE binary16
 * (uint16_t bit patterns, rounded to nearest) for a mixed-precision plan. */
gsr_status gsr_render_fwd(gsr_plan *plan, void *rgb, float *T_final, int32_t *n_contrib, int32_t *n_blend,
                          void *stream);

/* Gradient of the mean absolute photometric error, Eq. (photometric):
 * dL_drgb = sign(rgb - target) / (3 * total pixels), sign(0) = 0.  rgb as
 * gsr_render_fwd writes it (binary16 for a mixed-precision plan); target and
 * dL_drgb float32. */
gsr_status gsr_loss_l1(gsr_plan *plan, const void *rgb, const float *target, float *dL_drgb, void *stream);

/* Tracking loss of every view, appendix (Tracking and Camera Pose
 * Optimization).  With I_hat the render (rgb), I the observation (target),
 * both [3][H][W] per view, and the sums running over the view's pixels and
 * channels:
 *   (g, b) = argmin_{g,b} sum (I - g I_hat - b)^2               Eq. (app-ls)
 *   loss   = sum_pixels w sum_channels |I - (g I_hat + b)|      Eqs. (app-bright), (app-trackloss)
 *   w      = clip((1 - T_final) / tau_alpha, 0, 1)
 *            * clip(||grad I||_2 / tau_grad, 0, 1)              Eq. (app-weight)
 * ||grad I||_2: Frobenius norm over the channels of the observation's
 * central differences (one-sided at the border, zero along an axis of
 * extent 1).  (g, b) is the least-squares solution as a function of the
 * render; a render without variance takes g = 1, b = mean(I) - mean(I_hat).
 * Outputs (device): loss [n_views] and exposure [n_views][2] = (g, b) in
 * double; dL_drgb (like rgb) = d(sum of the losses)/d rgb, including the
 * dependence of (g, b) on the render (d|r|/dr = 0 at r = 0); dL_dT (like
 * T_final, may be NULL) = the gradient through the opacity weight (the
 * clip's derivative taken as 0 outside the open interval (0, 1)).  Both feed
 * gsr_render_bwd.  tau_alpha, tau_grad: positive and finite, else
 * GSR_EINVAL.  Uses the plan's workspace; deterministic (fixed-order sums). */
gsr_status gsr_loss_track(gsr_plan *plan, const float *rgb, const float *T_final, const float *target,
                          double tau_alpha, double tau_grad, double *loss, double *exposure, float *dL_drgb,
                          float *dL_dT, void *stream);

/* Mapping loss of the appendix's optimisation settings (an L1 term and an
 * SSIM term weighted by lambda_dssim = 0.2 there), over every pixel and
 * channel of every view, x the render (rgb) and y the target:
 *   loss = (1 - lambda) mean |x - y| + lambda (1 - mean SSIM(x, y)).
 * SSIM per channel (Wang et al. 2004): 11 x 11 Gaussian window of standard
 * deviation 1.5 (weights summing to 1), C1 = 0.01^2, C2 = 0.03^2, zeros
 * outside the image.  Outputs: loss (device, one double) and dL_drgb (like
 * rgb, overwritten) = d loss / d rgb (d|r|/dr = 0 at r = 0), which feeds
 * gsr_render_bwd.  lambda outside [0, 1]: GSR_EINVAL.  Uses the plan's
 * workspace; deterministic (fixed-order sums); the arithmetic is FP32 with
 * the loss summed in double. */
gsr_status gsr_loss_mapping(gsr_plan *plan, const float *rgb, const float *target, double lambda, double *loss,
                            float *dL_drgb, void *stream);

/* Backward of gsr_render_fwd (call after it, on the same plan, without an
 * intervening gsr_project or gsr_bin).  T_final and n_contrib are the buffers
 * the forward wrote (read only).  dL_dT may be NULL (zero).  pose_only: HOST array
 * [n_views] of 0/1 or NULL; views flagged 1 contribute to d_xi only.  It is
 * read when the call is made and passed to the kernels by value, so a call
 * captured into a graph keeps the flags it was captured with: replays see
 * later changes to the poses and parameters (device memory) but not to
 * pose_only (capture again to change which views are pose-only).  grads
 * may be NULL (pose gradients only); d_xi: device [n_views][6] or NULL.
 * g and poses must be the values given to gsr_project. */
gsr_status gsr_render_bwd(gsr_plan *plan, const gsr_gaussians *g, const float *poses, const float *T_final,
                          const int32_t *n_contrib, const float *dL_drgb, const float *dL_dT,
                          const uint8_t *pose_only, gsr_grads *grads, float *d_xi, void *stream);

/* The two stages of gsr_render_bwd, callable separately (same arguments and
 * rules).  gsr_raster_bwd: backward of Eq. (alpha) into per-slot
 * screen-space gradient accumulators (grad2d in the layout).
 * gsr_project_bwd: backward of Eq. (proj) and of the pose twist, Eqs.
 * (muCjac)-(sigmaIjac), from those accumulators to grads and d_xi. */
gsr_status gsr_raster_bwd(gsr_plan *plan, const float *T_final, const int32_t *n_contrib, const float *dL_drgb,
                          const float *dL_dT, void *stream);
gsr_status gsr_project_bwd(gsr_plan *plan, const gsr_gaussians *g, const float *poses, const uint8_t *pose_only,
                           gsr_grads *grads, float *d_xi, void *stream);

/* ---- one-shot seeding (independent of any plan) ---------------------- */

#define GSR_SEED_MAX_NEIGHBOURS 8

/* One keyframe of a seeding call (host struct; image is a device pointer). */
typedef struct {
    double P[12];          /* 3x4 projection matrix K [R | t], row-major; pixel
                              positions with pixel centres at +1/2 */
    double centre[3];      /* camera centre, world coordinates */
    int32_t width, height; /* image size */
    const float *image;    /* device [3][height][width]: the observed keyframe */
    double gain, bias;     /* its exposure (observed = gain * radiance + bias) */
} gsr_seed_view;

typedef struct {
    double max_reproj;     /* px; a kept point's reprojection error is below it */
    double min_parallax;   /* radians; a kept point's baseline angle is at least it */
    double alpha_lo, alpha_hi; /* Eq. (app-alpha-init) bounds, 0 < lo <= hi < 1 */
} gsr_seed_config;

/* Seeds one Gaussian candidate per reference pixel of keyframe views[0] from
 * its correspondences in the n_neighbours keyframes views[1..] (Sec. "Dense
 * Feature Matching", Multi-view Triangulation, and the appendix's
 * initialisation).  For every neighbour the two-view linear system
 * (rows x P^3 - P^1, y P^3 - P^2 of both views) is solved in double for the
 * right singular vector of its smallest singular value; the hypothesis with
 * the lowest reprojection error (RMS of the two reprojection distances, in
 * front of both cameras) is kept, ties going to the larger baseline angle
 * (the angle at X between the rays to both camera centres).  It is valid
 * when that error is below max_reproj and the angle at least min_parallax.
 * Inputs (device): x_ref [2][n] reference pixel positions, x_nb [K][2][n]
 * matched positions, kappa [K][n] per-neighbour confidences in [0, 1].
 * Outputs (device): mean [3][n] (the kept hypothesis, also for an invalid
 * one; 0 if there is none), colour [3][n] (median over the supporting views
 * -- the reference and every neighbour whose match lies within max_reproj of
 * the point's projection -- of the bilinear samples corrected by
 * (sample - bias) / gain; the mean of the middle two for an even count; 0
 * when invalid), opacity_logit [n] (logit of alpha_lo + (alpha_hi -
 * alpha_lo) kappa_bar, Eq. (app-alpha-init)), valid [n] (0/1); optional
 * (NULL allowed): best [n] (neighbour index or -1), err [n] (px, +inf if no
 * hypothesis), angle [n] (radians), kappa_bar [n] (Eq. (conf), the mean of
 * kappa over the neighbours).  n < 2^31, 1 <= n_neighbours <=
 * GSR_SEED_MAX_NEIGHBOURS; bad arguments give GSR_EINVAL. */
gsr_status gsr_seed_triangulate(int64_t n, int32_t n_neighbours, const gsr_seed_view *views,
                                const gsr_seed_config *cfg, const float *x_ref, const float *x_nb,
                                const float *kappa, float *mean, float *colour, float *opacity_logit,
                                int32_t *valid, int32_t *best, float *err, float *angle, float *kappa_bar,
                                void *stream);

/* Isotropic initial scale of the valid seeds: log_scale [3][n] (device) =
 * log(max(d, floor_scale)) on every axis, d the mean distance to the 3
 * nearest other valid seeds (all of them when fewer exist; floor_scale when
 * none); 0 for invalid seeds.  mean [3][n], valid [n] as written by
 * gsr_seed_triangulate.  workspace: caller-owned device memory of
 * gsr_seed_scale_workspace_bytes(n) bytes (0 for n out of range), reused
 * freely between calls; calls that share it must be ordered. */
size_t gsr_seed_scale_workspace_bytes(int64_t n);
gsr_status gsr_seed_scale(int64_t n, const float *mean, const int32_t *valid, float floor_scale, void *workspace,
                          size_t workspace_bytes, float *log_scale, void *stream);

/* Anisotropic initial covariance of the valid seeds, Eq. (app-sigma-init):
 * Sigma = U diag(s_perp^2, s_perp^2, s_par^2) U^T with U = [t1 t2 v].
 * Readings where the paper is silent: the plane is fitted to the valid
 * seeds within `radius` of the seed (itself included; distances of the FP32
 * positions compared in double) by the eigen-decomposition of their scatter
 * about their mean, v the eigenvector of the smallest eigenvalue (the
 * normal), t1 that of the largest, t2 = v x t1; fewer than three seeds in
 * the radius: v = the unit ray from centre_ref to the seed, t1 any unit
 * perpendicular.  s_perp = det(J J^T)^(-1/4), J the 2 x 3 Jacobian of the
 * pixel position under P_ref with respect to the world point (the radius of
 * the circle of equal area to the back-projected one-pixel footprint);
 * s_par = c_par s_perp max(1, err) / max(sin(angle), 1e-6); both at least
 * floor_scale (s_par from the floored s_perp).  FP64 arithmetic.
 * Inputs: mean [3][n], valid [n], err [n] and angle [n] as written by
 * gsr_seed_triangulate (device); P_ref (3 x 4, row-major) and centre_ref [3]
 * of the reference keyframe (host).  Outputs (device): quat [4][n], the
 * unit quaternion (w, x, y, z) of U, and log_scale [3][n] = (log s_perp,
 * log s_perp, log s_par); the identity and zeros for invalid seeds.
 * workspace: gsr_seed_scale_workspace_bytes(n) bytes of device memory.
 * The search hashes the seeds by cells of `radius` and visits the 3 x 3 x 3
 * cells around each seed, so its cost grows with the number of seeds within
 * about two radii.  Bad arguments (n out of range, a non-positive or non-finite
 * radius, c_par or floor_scale, a non-finite P_ref or centre_ref, a null
 * buffer, a small workspace): GSR_EINVAL, nothing enqueued. */
gsr_status gsr_seed_frame(int64_t n, const float *mean, const int32_t *valid, const float *err, const float *angle,
                          const double *P_ref, const double *centre_ref, double radius, double c_par,
                          float floor_scale, void *workspace, size_t workspace_bytes, float *quat, float *log_scale,
                          void *stream);

/* Nearest other valid Gaussian of each valid Gaussian (Euclidean distance of
 * the centres; ties go to the lower index), the neighbour search behind the
 * merging of Sec. "Insertion, Lightweight Merging, and Pruning".  mean
 * [3][n], valid [n] (device; 0 excludes a Gaussian both as a query and as a
 * neighbour).  Output nn_index [n] (device): the neighbour's index, -1 for
 * an invalid Gaussian or one with no valid other.  workspace: device,
 * gsr_seed_scale_workspace_bytes(n) bytes (the same search).  n out of
 * [0, 2^31) or a null buffer: GSR_EINVAL, nothing enqueued. */
gsr_status gsr_nearest(int64_t n, const float *mean, const int32_t *valid, void *workspace, size_t workspace_bytes,
                       int32_t *nn_index, void *stream);

/* ---- map maintenance (independent of any plan) ----------------------- */

/* Five parameter planes in the layout of gsr_gaussians: mean [3][n],
 * quat [4][n], log_scale [3][n], opacity_logit [n], colour [colour_rows][n]
 * (3 for RGB, 3 (d+1)^2 for SH); device pointers. */
typedef struct {
    float *mean, *quat, *log_scale, *opacity_logit, *colour;
} gsr_planes;

typedef struct {
    float lr[5];           /* learning rate of each plane (mean, quat, log_scale,
                              opacity_logit, colour): the scheduled value of this
                              step; the appendix's settings are 1e-3 for
                              positions and rotations, 2e-3 for colour and
                              opacity */
    double beta1, beta2;   /* in [0, 1); the appendix's 0.9, 0.999 (double, so
                              that 1 - beta is formed exactly before rounding
                              to the FP32 arithmetic) */
    float eps;             /* > 0; 1e-8 */
    float max_grad_norm;   /* global L2 clipping norm (the appendix's 1.0); <= 0:
                              no clipping */
    float ema;             /* eta of Eq. (app-ema) in [0, 1] */
    int32_t step;          /* t >= 1, for the bias corrections */
} gsr_adam_config;

#define GSR_ADAM_WORKSPACE_BYTES 16384

/* One optimiser step of the appendix's optimisation settings (Adam, Kingma
 * and Ba, Algorithm 1, with per-plane learning rates and gradient norm
 * clipping), then the anchor update of Eq. (app-ema) on the new means:
 *   c = min(1, max_grad_norm / (||g||_2 + 1e-6)) over all planes,
 *   m = b1 m + (1 - b1) c g,  v = b2 v + (1 - b2) (c g)^2,
 *   p -= lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps),
 *   anchor = (1 - ema) anchor + ema mean.
 * params, m, v are updated in place; grads are read only (their planes given
 * through the same struct).  anchor: device [3][n] or NULL.  workspace:
 * device, GSR_ADAM_WORKSPACE_BYTES, 8-byte aligned.  norm: device double [1]
 * or NULL, receives ||g||_2 before clipping.  FP32 state and arithmetic, the
 * norm in double and in a fixed order (deterministic).  Invalid settings or
 * a null plane: GSR_EINVAL, nothing enqueued. */
gsr_status gsr_adam_step(int64_t n, int32_t colour_rows, const gsr_planes *params, const gsr_planes *grads,
                         const gsr_planes *m, const gsr_planes *v, float *anchor, const gsr_adam_config *cfg,
                         void *workspace, double *norm, void *stream);

/* Co-visibility score of Eq. (iou) between a key frame and n_frames frames
 * of the same size: a pixel is visible when its accumulated opacity 1 - T
 * exceeds tau (compared in float32).  T_key [pixels], T_frames
 * [n_frames][pixels] (device, e.g. T_final of gsr_render_fwd).  Outputs
 * (device): counts [n_frames][2] = (|V_key & V_f|, |V_key | V_f|), exact;
 * iou [n_frames] = intersection / union (0 for an empty union). */
gsr_status gsr_covis(int64_t pixels, int32_t n_frames, const float *T_key, const float *T_frames, float tau,
                     uint64_t *counts, double *iou, void *stream);

typedef struct {
    int32_t m_min;         /* observation count below which a Gaussian goes */
    float v_min;           /* cumulative visibility below which it goes */
    float sigma_max;       /* trace of the world covariance above sigma_max^2 */
    float alpha_min;       /* opacity below which it goes */
} gsr_prune_config;

/* Pruning rule of Sec. "Insertion, Lightweight Merging, and Pruning": the
 * Gaussian i is dropped when m_obs[i] < m_min, v_vis[i] < v_min,
 * exp(2 s0) + exp(2 s1) + exp(2 s2) > sigma_max^2 (the trace of
 * R diag(s^2) R^T) or sigmoid(opacity_logit[i]) < alpha_min, decided in
 * double.  m_obs, v_vis: the caller's statistics [n]; log_scale [3][n],
 * opacity_logit [n].  Outputs (device): keep_index [n], the kept indices in
 * increasing order in its first *kept entries, and kept [1].  workspace:
 * device, gsr_prune_workspace_bytes(n) bytes. */
size_t gsr_prune_workspace_bytes(int64_t n);
gsr_status gsr_prune(int64_t n, const int32_t *m_obs, const float *v_vis, const float *log_scale,
                     const float *opacity_logit, const gsr_prune_config *cfg, int32_t *keep_index, int64_t *kept,
                     void *workspace, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): gsr_prune
 * without a workspace.  Same rule, arguments, outputs and errors as
 * gsr_prune; the pruning scan keeps its per-block counts in a fixed device
 * array of the library (256 KiB, one per GPU, held until the process ends)
 * instead, so the call allocates nothing.  n may not exceed
 * GSR_PRUNE_NOALLOC_MAX_N (2^27): larger n returns GSR_EINVAL with nothing
 * enqueued.  All calls on one GPU share that array: calls that overlap on one
 * GPU (different streams or threads) race and must be ordered by the
 * caller.  The first call on each device looks up the array's address there
 * (hipGetSymbolAddress) with that device current. */
#define GSR_PRUNE_NOALLOC_MAX_N (1ll << 27)
gsr_status gsr_prune_noalloc(int64_t n, const int32_t *m_obs, const float *v_vis, const float *log_scale,
                             const float *opacity_logit, const gsr_prune_config *cfg, int32_t *keep_index,
                             int64_t *kept, void *stream);

/* Compaction after gsr_prune: dst[r][j] = src[r][keep_index[j]] for
 * j < *kept (device value), r < rows; src and dst [rows][n] (device, not
 * overlapping); columns from *kept on are left as they are. */
gsr_status gsr_compact(int64_t n, int32_t rows, const float *src, const int32_t *keep_index, const int64_t *kept,
                       float *dst, void *stream);

/* Spatial storage order of a map.  The paper fixes no order for the
 * Gaussians: every sum of Eqs. (alpha) and (color) runs over the
 * depth-ordered set N(p), whatever the storage order, which only breaks ties
 * of equal depth (by index).  This order is a layout choice that makes the
 * Gaussians of a projection wave, and of a binning chunk, neighbours in
 * space.  index[j] (device, [n]) receives the Gaussian to store at position
 * j, a permutation of 0 .. n-1 to apply with gsr_compact (kept = n) to every
 * plane of the map and of its optimiser state.  Definition, for means [3][n]
 * (device, x, y, z planes):
 *   1. lo_a, hi_a: the least and greatest coordinate a over the Gaussians
 *      whose three coordinates are finite; w = max over a of hi_a - lo_a
 *      (double);
 *   2. cells: with w = m 2^e, m in [0.5, 1), q_a = min(1023,
 *      floor((x_a - lo_a) 2^(10 - e))) in double; all 0 when w = 0;
 *   3. code: the Morton interleave of q_x, q_y, q_z (bit k of q_x at bit
 *      3k, of q_y at 3k + 1, of q_z at 3k + 2); 2^30 for a Gaussian with a
 *      non-finite coordinate;
 *   4. rank: place in the ascending order of (code, index);
 *   5. with F = floor(n / brick) and P the least integer
 *      >= max(1, floor(0.6180339887498949 F + 0.5)) coprime with F, position
 *      j brick + k (j < F, k < brick) holds the Gaussian of rank
 *      ((j P) mod F) brick + k, and positions from F brick on the Gaussian
 *      of their own rank.
 * So a brick of consecutive positions holds neighbours along the curve,
 * and consecutive bricks come from far apart (brick >= n: the plain curve
 * order).  The result is deterministic.  workspace: device, 256-byte
 * aligned, gsr_spatial_order_workspace_bytes(n) bytes (0 for n out of
 * range), not overlapping mean or index.  Errors: GSR_EINVAL for null
 * pointers, n outside [1, 2^31), brick < 1, a short or misaligned
 * workspace or overlapping buffers; nothing enqueued. */
size_t gsr_spatial_order_workspace_bytes(int64_t n);
gsr_status gsr_spatial_order(int64_t n, const float *mean, int32_t brick, int32_t *index, void *workspace,
                             size_t workspace_bytes, void *stream);

/* Merging of Sec. "Insertion, Lightweight Merging, and Pruning" (readings
 * where the paper is silent): i and j = nn_index[i] merge when they are
 * mutual nearest neighbours (nn_index[j] == i), their centres lie within
 * radius * min(sbar_i, sbar_j), sbar = exp(mean of the three log_scales)
 * (highly overlapping footprints), and the first three colour rows differ
 * by at most colour_tol each (similar colours).  The pair becomes one
 * Gaussian at the lower index with the v_vis-weighted mean (equal weights
 * when both are 0) of mean, colour rows, opacity (as sigmoid) and world
 * covariance R diag(s^2) R^T, split back into a unit quaternion and
 * log-scales by its eigen-decomposition (FP64 arithmetic); the higher index
 * is marked dropped.  params: the input planes; out: separate output planes
 * of the same shapes, not overlapping the input (every column written: a
 * copy for Gaussians not merged).  nn_index [n] from gsr_nearest; v_vis [n].
 * keep [n] (device): 1 kept, 0 merged away, for gsr_keep_list.  Errors:
 * GSR_EINVAL for null planes, aliasing planes, colour_rows out of [3, 48] or
 * a negative or non-finite radius or colour_tol; nothing enqueued. */
gsr_status gsr_merge(int64_t n, int32_t colour_rows, const gsr_planes *params, const float *v_vis,
                     const int32_t *nn_index, double radius, double colour_tol, gsr_planes *out, int32_t *keep,
                     void *stream);

/* Ordered list of the set entries of a 0/1 mask [n] (device): keep_index
 * receives the indices i with mask[i] != 0 in increasing order in its first
 * *kept entries, for gsr_compact.  workspace: device,
 * gsr_prune_workspace_bytes(n) bytes.  n must lie in [1, 2^31). */
gsr_status gsr_keep_list(int64_t n, const int32_t *mask, int32_t *keep_index, int64_t *kept, void *workspace,
                         void *stream);

/* Rate of the device wall clock of the current device (the clock of the
 * layout's stamps), in ticks per second. */
gsr_status gsr_device_clock_hz(double *hz);

/* Synchronises `stream`, then reports the pair count of the last binning
 * and whether it exceeded the capacity. */
gsr_status gsr_pair_count(gsr_plan *plan, int64_t *required, int32_t *overflow, void *stream);

/* Device time of the library's kernels, for benchmarks and profiling.
 * While timing is on, each launch group below is bracketed by two HIP events
 * recorded on the launch stream (not while that stream is being captured
 * into a graph, where nothing is recorded).  The events are host objects of
 * the plan; no device memory is allocated.  Switching timing on clears the
 * totals.  gsr_plan_read_timing waits for the events recorded so far (it
 * synchronises with them) and reports, for one group, the summed
 * milliseconds and the number of timed launches since timing was switched
 * on.  Returns GSR_EINVAL for an unknown group. */
typedef enum {
    GSR_T_PROJECT = 0,  /* gsr_project's kernel */
    GSR_T_BIN_EMIT,     /* pair counting, offsets and emission */
    GSR_T_BIN_SORT,     /* ordering of the pairs */
    GSR_T_BIN_RANGES,   /* tile ranges and the tiles' processing order */
    GSR_T_RASTER_FWD,   /* compositing forward kernel */
    GSR_T_LOSS_L1,      /* gsr_loss_l1's kernel */
    GSR_T_CLEAR_GRAD2D, /* zeroing of the screen-space gradient accumulators */
    GSR_T_RASTER_BWD,   /* compositing backward kernel */
    GSR_T_PROJECT_BWD,  /* projection backward and the pose reduction */
    GSR_T_LOSS_TRACK,   /* gsr_loss_track's kernels */
    GSR_T_LOSS_MAP,     /* gsr_loss_mapping's kernels */
    GSR_T_COUNT
} gsr_timer;

gsr_status gsr_plan_set_timing(gsr_plan *plan, int32_t enable);
gsr_status gsr_plan_read_timing(gsr_plan *plan, int32_t timer, double *total_ms, int64_t *launches);

const char *gsr_status_str(gsr_status s);
/* Detail of the last failure on the calling thread ("" if none). */
const char *gsr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */
