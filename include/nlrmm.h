/*
 * nlrmm.h -- C ABI of the MI355X (gfx950) NL-RMM-GKS hot path.
 *
 * The library computes the operator applications of NL-RMM-GKS (Okunola, Pasha,
 * Kilmer, Nagy, de Sturler, "Nonlinear RMM-GKS for large-scale dynamic and
 * streaming inverse problems with uncertain forward operators") for the forward
 * model b = H(p) u + e of Section 1 (eq. "nonlinear_forward"), where H(p) is the
 * parallel-beam Radon transform at per-view angles theta = p (Section 6.2 uses a
 * global shift of the nominal angles; per-view angles are the general case).
 *
 * Discretisation (the paper leaves it to a toolbox; this is the library's model):
 *   weight a[v][j][pix] = |pixel square ∩ {s0 + j ds <= p.n(theta_v) < s0 + (j+1) ds}| / ds,
 *   n(theta) = (cos theta, sin theta).  The sinogram is the bin-averaged line integral
 *   of the piecewise-constant image.  The angle derivative is exact for this model.
 *
 * Conventions for every entry point
 *   - Pointers named x, y, theta, V, AV, ... are DEVICE pointers owned by the caller;
 *     the library never frees or reallocates them.  Host pointers are marked (host).
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = default
 *     stream) and returns without synchronising.
 *   - Return value: 0 on success, a negative NLRMM_E* code on failure (never throws).
 *     Arguments are validated on the host before anything is launched; on error
 *     nothing is enqueued and outputs are untouched.
 *   - Numerical events detected on the device (Krylov breakdown, DP bracket clamp,
 *     Armijo failure, non-finite values) are OR-ed into a caller-provided device
 *     int32 status word (NLRMM_ST_* bits) and never force a host synchronisation.
 *   - One context per stream; calls on one context must not overlap.
 *
 * Memory layouts (row-major, last index fastest)
 *   image    x[col][frame][iy][ix]   pixel (ix, iy) = [x0 + ix d, x0 + (ix+1) d] x
 *                                                     [y0 + iy d, y0 + (iy+1) d]
 *   sinogram y[col][view][bin]       views of frame f: view_off[f] .. view_off[f+1]-1
 *   angles   theta[view]             float64 radians
 */
#ifndef NLRMM_H
#define NLRMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NLRMM_OK 0
#define NLRMM_EINVAL -1   /* null pointer or out-of-range scalar argument */
#define NLRMM_ESHAPE -2   /* inconsistent or unsupported sizes */
#define NLRMM_EHIP -3     /* a HIP runtime call failed */
#define NLRMM_ENOMEM -4   /* device workspace allocation failed */
#define NLRMM_ENOTSUP -5  /* unsupported option combination */

#define NLRMM_ST_BREAKDOWN 1      /* new Krylov direction numerically in span(V) */
#define NLRMM_ST_DP_LOW 2         /* discrepancy principle clamped to the bracket's low end */
#define NLRMM_ST_DP_HIGH 4        /* ... to the bracket's high end */
#define NLRMM_ST_ARMIJO 8         /* no Armijo step accepted; angles unchanged */
#define NLRMM_ST_NONFINITE 16     /* a NaN or Inf was produced */
#define NLRMM_ST_COMPRESS_SKIP 32 /* u already in span(V W): compressed basis has kmin-1 columns */

/* Image grid and detector.  Square pixels of width d.
 * Limits checked on the host by every entry point (NLRMM_ESHAPE when violated, before
 * anything is launched):
 *   all entry points       1 <= nx, ny <= 16384, 1 <= nbins <= 65536, d > 0, ds > 0, finite;
 *   forward family         nx, ny <= 4096 (nlrmm_project, nlrmm_project_dtheta,
 *                          nlrmm_project_residual, nlrmm_autotune_project);
 *   backward family        at most 4 bin edges inside one pixel footprint,
 *                          ceil(d sqrt(2) / ds - 1e-12) <= 4, and a staged window of
 *                          ceil(15 d sqrt(2) / ds) + that count + 4 <= 64 bins per 16-pixel
 *                          tile, i.e. ds >= about 0.38 d (nlrmm_backproject(_acc),
 *                          nlrmm_backproject_dtheta, nlrmm_autotune_backproject);
 *   solver, gks_expand     both families.
 * nlrmm_check_geom reports these limits without a device. */
typedef struct {
    int32_t nx, ny;   /* pixels along x (fastest index) and y */
    double x0, y0;    /* lower-left corner of the image */
    double d;         /* pixel width, > 0 */
    int32_t nbins;    /* detector bins */
    double s0, ds;    /* bin j covers [s0 + j ds, s0 + (j+1) ds), ds > 0 */
} nlrmm_geom;

#define NLRMM_OPS_FORWARD 1    /* projection, angle derivative, data residual */
#define NLRMM_OPS_BACKWARD 2   /* backprojection and the derivative's transpose */

/* Frames with their own images and uneven view counts (dynamic problems). */
typedef struct {
    int32_t nframes;          /* >= 1 */
    int64_t nviews;           /* total number of views V >= 1 */
    const int64_t *view_off;  /* DEVICE [nframes+1] prefix offsets, view_off[0] = 0,
                                 view_off[nframes] = nviews; may be NULL iff nframes == 1 */
} nlrmm_batch;

typedef struct nlrmm_ctx nlrmm_ctx;   /* opaque: device workspace and launch cache */

const char *nlrmm_strerror(int code);
int nlrmm_version(void);

/* Host-only shape check (no context, no device work): NLRMM_OK when the operator families
 * in `ops` (NLRMM_OPS_* bits) accept `geom`, NLRMM_ESHAPE when a size limit above is
 * exceeded, NLRMM_EINVAL for a NULL or non-finite geometry or unknown bits.  The entry
 * points run the same check first. */
int nlrmm_check_geom(int32_t ops, const nlrmm_geom *geom);

/* Create a context on HIP device `device`.  Allocates nothing yet; workspace grows on
 * the first call that needs it (outside graph capture).  *out receives the handle. */
int nlrmm_ctx_create(nlrmm_ctx **out, int device);
void nlrmm_ctx_destroy(nlrmm_ctx *ctx);

/* Autotuner of the projector launch shapes (the batching design: tile and ray-block shapes
 * chosen by measurement).  nlrmm_autotune_project computes y = A(theta) x exactly like
 * nlrmm_project while timing each forward block shape (1, 2, 4 or 8 waves sharing each
 * detector edge's image lines) with HIP events on `stream`, and keeps the fastest for this
 * geometry, batch and column-group size in the context; nlrmm_autotune_backproject does the
 * same for the backprojection's view split (1, 2, 4, 8 or 16 partial images, bounded by 16 views
 * per split and frame) and leaves x = A(theta)^T y.  Candidates differ only in the order of
 * FP64 partial sums.  Both synchronize `stream` and return NLRMM_EINVAL while it is being
 * captured.  Later calls with the same shapes (operators, solver, graph captures) use the
 * choice.  nlrmm_ctx_set_tune_file loads choices stored in `path` (lines of
 * "kind nx ny nbins nframes nviews ncols choice"; kind 0 forward with choice 1, 2, 4 or 8,
 * kind 1 backprojection with choice 1, 2, 4, 8 or 16; other lines are skipped) and appends
 * every new choice there; NULL stops appending.  A stored view split above what the shape
 * allows (16 views per split and frame) is clamped to that bound when the backprojection is
 * launched.  nlrmm_tune_query returns the stored choice for a shape in *choice (0 when none:
 * the built-in default is used). */
int nlrmm_autotune_project(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                           int32_t ncols, const float *x, const double *theta, float *y,
                           void *stream);
int nlrmm_autotune_backproject(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                               int32_t ncols, const float *y, const double *theta, float *x,
                               void *stream);
int nlrmm_ctx_set_tune_file(nlrmm_ctx *ctx, const char *path);
int nlrmm_tune_query(nlrmm_ctx *ctx, int32_t kind, const nlrmm_geom *geom,
                     const nlrmm_batch *batch, int32_t ncols, int32_t *choice);

/* Measurement aid (no part of the method).  With timing enabled (enable >= 1), every
 * projection records a pair of HIP events on its launch stream around its forward-weights
 * kernel (which = 0), and every backprojection around its pixel-tile kernel (which = 1); the
 * pair of the most recent launch is kept (for a multi-group projection, the last group's).
 * enable = R > 1 launches the timed kernel R times back to back between the two events
 * (capped at 1000; the results are unchanged because the repeated kernel recomputes the same
 * outputs; a backprojection that adds into x is launched once), so that the events' own cost
 * is spread over R launches.  nlrmm_ctx_kernel_ms waits for the stop event and returns the
 * duration per launch in milliseconds; NLRMM_EINVAL if no such launch has been recorded
 * since timing was enabled.  Events are created by nlrmm_ctx_set_timing (so enable it
 * outside graph capture) and freed by nlrmm_ctx_destroy.  enable = 0 turns timing off.
 * enable = -P (P = 1 .. 1000) selects per-launch accumulation instead: every P-th eligible
 * launch (one-column projections without the derivative, reductions or an early-exit flag;
 * one-column backprojections) records its own event pair around the single kernel launch, up
 * to 4096 launches per kernel; nlrmm_ctx_kernel_avg waits for the last one, returns the average
 * duration of the recorded launches in milliseconds and their number, and starts a new
 * accumulation (NLRMM_EINVAL unless this mode is on). */
int nlrmm_ctx_set_timing(nlrmm_ctx *ctx, int enable);
int nlrmm_ctx_kernel_ms(nlrmm_ctx *ctx, int which, float *ms);
int nlrmm_ctx_kernel_avg(nlrmm_ctx *ctx, int which, float *avg_ms, int32_t *launches);

/* Forward projection y = A(theta) x (the forward operator H(p)u of Section 1,
 * eq. "nonlinear_forward"; applied to every column for the basis block A V of
 * Section 3.2).
 *   x     [ncols][nframes][ny][nx] float32
 *   theta [nviews] float64
 *   y     [ncols][nviews][nbins] float32, overwritten
 * Edge-driven evaluation with FP64 accumulation; deterministic (no atomics). */
int nlrmm_project(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                  int32_t ncols, const float *x, const double *theta, float *y, void *stream);

/* Backprojection x = A(theta)^T y, the exact transpose of nlrmm_project (the H^T in the
 * GKS residual H^T(Hu - b) of Section 3.2).  Pixel-driven gather, no atomics.
 *   y [ncols][nviews][nbins] float32 ; x [ncols][nframes][ny][nx] float32, overwritten */
int nlrmm_backproject(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                      int32_t ncols, const float *y, const double *theta, float *x,
                      void *stream);

/* Backprojection that allocates nothing (no hipMalloc, hipFree or allocating library call),
 * for callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Same operator, arguments, layouts and results as
 * nlrmm_backproject (bitwise: the same view split and summation order).  The view split's
 * partial images (split x ncols x nframes x ny x nx float32, none when the shape runs
 * without a split) are kept in a fixed device array of NLRMM_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends; a shape whose split needs
 * more returns NLRMM_ESHAPE before anything is launched.  The context itself must have been
 * created beforehand (nlrmm_ctx_create allocates no device memory).  All calls on one GPU
 * share that array: calls that overlap in time on one GPU (different streams or host
 * threads) race on it and must be serialised by the caller. */
#define NLRMM_NOALLOC_SCRATCH_BYTES (64u << 20)
int nlrmm_backproject_noalloc(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                              int32_t ncols, const float *y, const double *theta, float *x,
                              void *stream);

/* Transpose of the angle derivative: x = D(theta)^T r = sum_v (dA_v/dtheta_v)^T r_v, the
 * H_p^T r term of the full-space sensitivity equation of Section 4.2 (eq. "sensitivity") for
 * a global angle offset (per-view terms: r zero outside view v).  Per view, bin j carries
 * (M(e_j) - M(e_{j+1})) / ds with M the chord first moment (the weights of
 * nlrmm_project_dtheta), gathered per pixel; no atomics.
 *   r [ncols][nviews][nbins] float32 ; x [ncols][nframes][ny][nx] float32, overwritten */
int nlrmm_backproject_dtheta(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                             int32_t ncols, const float *r, const double *theta, float *x,
                             void *stream);

/* Angle derivative of the projection, D[v][j] = d y[v][j] / d theta_v: the Jacobian
 * columns H_{p_i} u of Alg. "update_param" (view v's column has nonzeros only on view
 * v's rows).  Optional outputs (any may be NULL, at least one must be given):
 *   dy     [ncols][nviews][nbins] float32 : D itself
 *   yproj  [ncols][nviews][nbins] float32 : the projection A(theta) x (fused)
 *   gdot   [ncols][nviews] float64        : <D_v, g_v> with g [nviews][nbins] float32
 *                                           (requires g); the AltMin gradient when g is
 *                                           the residual A(theta)u - b
 *   dnorm2 [ncols][nviews] float64        : ||D_v||^2 (the diagonal of J^T J)
 * The per-view reductions are computed in FP64 without writing D. */
int nlrmm_project_dtheta(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                         int32_t ncols, const float *x, const double *theta, float *dy,
                         float *yproj, const float *g, double *gdot, double *dnorm2,
                         void *stream);

/* Backprojection that adds into x (x += A(theta)^T y) when accumulate != 0; otherwise
 * identical to nlrmm_backproject.  Used to sum the adjoints of measurement blocks. */
int nlrmm_backproject_acc(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                          int32_t ncols, const float *y, const double *theta, float *x,
                          int32_t accumulate, void *stream);

/* Data residual of the forward model (eq. "nonlinear_forward"): r = A(theta) x - b for one
 * image, computed in the projection kernel (the projection itself is never stored).
 *   b [nviews][nbins] float32; r [nviews][nbins] float32 or NULL;
 *   rnorm2 [nviews] float64 or NULL: ||r_v||^2 per view (FP64 accumulation). */
int nlrmm_project_residual(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                           const float *x, const double *theta, const float *b, float *r,
                           double *rnorm2, void *stream);

/* ------------------------------------------------------------------------------------
 * Fan-beam family: the CT geometry of Section 6.2 (a point source at distance R from the
 * rotation centre; the paper leaves the distances to its toolbox, this is the library's
 * model).  View theta has n = (cos, sin), t = (-sin, cos), the source at S = -R t and the
 * detector on the line through the rotation centre (the origin of the image coordinates)
 * along n, bin j covering s in [s0 + j ds, s0 + (j+1) ds); the ray of detector coordinate s
 * runs from S through s n.  Near each pixel centre c the rays are taken as parallel along
 * the ray through c (direction t(alpha), alpha = theta - gamma, tan gamma = (c.n)/(R + c.t)),
 * which meets the detector at s_c = R (c.n) / (R + c.t), and a shift w across the rays at c
 * moves s by m w, m = R |c - S| / (R + c.t)^2.  The weight is the strip-area weight of the
 * pixel for direction alpha, centred at s_c and scaled by m:
 *   a[v][j][pix] = (m / ds) (Phi_alpha((e_{j+1} - s_c) / m) - Phi_alpha((e_j - s_c) / m)),
 * Phi_alpha the pixel's cumulative footprint across direction alpha.  It is exact to first
 * order in the pixel size and becomes the parallel-beam model above as R grows.
 * Arguments, layouts and the frame batching are those of the parallel-beam family; R is a
 * host scalar with R >= 1.5 x the largest distance of an image corner from the origin
 * (NLRMM_EINVAL otherwise: the source stays well outside the image).  Any geometry accepted
 * by nlrmm_check_geom(0, .) is accepted; ncols * nframes <= 65535.
 * Projection and derivative: bin-driven gather; transposes: pixel-driven gather; no atomics,
 * deterministic.  The derivative is the exact angle derivative of this model (the chord
 * terms of Section 4's Jacobian H_p u for per-view angles).
 * ------------------------------------------------------------------------------------ */

/* y = A_fan(theta) x.  x [ncols][nframes][ny][nx] float32 -> y [ncols][nviews][nbins]. */
int nlrmm_fan_project(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                      int32_t ncols, const float *x, const double *theta, double R, float *y,
                      void *stream);

/* x = A_fan(theta)^T y, the transpose of nlrmm_fan_project (up to FP32 rounding). */
int nlrmm_fan_backproject(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                          int32_t ncols, const float *y, const double *theta, double R,
                          float *x, void *stream);

/* dy[v][j] = d (A_fan(theta) x)[v][j] / d theta_v. */
int nlrmm_fan_project_dtheta(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                             int32_t ncols, const float *x, const double *theta, double R,
                             float *dy, void *stream);

/* x = D_fan(theta)^T r, the transpose of nlrmm_fan_project_dtheta. */
int nlrmm_fan_backproject_dtheta(nlrmm_ctx *ctx, const nlrmm_geom *geom,
                                 const nlrmm_batch *batch, int32_t ncols, const float *r,
                                 const double *theta, double R, float *x, void *stream);

/* ------------------------------------------------------------------------------------
 * Photoacoustic circular-means family (Section 6.3, "Photoacoustic Tomography with Sensor
 * Radius Uncertainty": circles of radii r_j(p) = r_j + p around every sensor, one global
 * radial shift p).  The paper leaves the operator to its toolbox; the library's model:
 * n_sensors sensors at angles 2 pi a / n_sensors on the circle of radius sensor_radius around
 * the image origin; radii r_j(p) = (j + 1) radius_step + p (radius_step = 2 / n_radii gives
 * the paper's r_j = 2 j / n_c); between pixel centres the image is its bilinear interpolant
 * (0 for indices outside the grid) and a circle integral is the n_samples-point trapezoid
 * rule:
 *   y[a][j] = (2 pi r / K) sum_k I(s_a + r (cos, sin)(2 pi k / K)),   K = n_samples.
 * The derivative in p is that of the sum, (2 pi / K) sum_k [I + r grad I . e_k].  Sample
 * positions, cells and weights FP64, pixel values FP32, sums FP64; deterministic (the
 * transpose is a gather).  Layouts: x [ncols][ny][nx] float32, y [ncols][n_sensors][n_radii]
 * float32; p a host double.  Limits: n_samples <= 8192, ncols * n_sensors * n_radii <= 2^26
 * (NLRMM_ESHAPE); a non-finite p or radius, a negative sensor radius or a radius step <= 0
 * gives NLRMM_EINVAL.
 * ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t n_sensors, n_radii, n_samples;
    double sensor_radius, radius_step;
} nlrmm_pat_geom;

/* y = A_pat(p) x: the circle integrals of every column. */
int nlrmm_pat_project(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_pat_geom *pat,
                      int32_t ncols, const float *x, double p, float *y, void *stream);

/* dy = d(A_pat(p) x)/dp: the Jacobian column of the global radial shift (Alg.
 * "update_param" with one parameter). */
int nlrmm_pat_project_dp(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_pat_geom *pat,
                         int32_t ncols, const float *x, double p, float *dy, void *stream);

/* x = A_pat(p)^T y, the transpose of nlrmm_pat_project (up to FP32 rounding of the inputs). */
int nlrmm_pat_backproject(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_pat_geom *pat,
                          int32_t ncols, const float *y, double p, float *x, void *stream);

/* ------------------------------------------------------------------------------------
 * Krylov side of MM-GKS / RMM-GKS (Section 3; supplementary Algs. "enlarge", "compress").
 * Basis blocks are column-contiguous FP32: V [ncols][n] with n = nframes*ny*nx, and
 * A V [ncols][m] with m = nviews*nbins.  Grams are FP64 row-major with leading dim ldg.
 * Psi is the anisotropic TV operator of Section 2.2: per frame the forward differences
 * along x (ny rows of nx-1) then along y (ny-1 rows of nx), unscaled; with temporal == 1
 * and nframes > 1 the frame differences ((nframes-1) blocks of ny*nx) follow.  The entry
 * points below that take no velocity field accept temporal 0 or 1 (temporal 2, the
 * optical-flow rows, goes through the nlrmm_theta_* family: NLRMM_EINVAL or NLRMM_ENOTSUP
 * here).
 * ------------------------------------------------------------------------------------ */

/* MM weights w = ((Psi u)^2 + eps^2)^(-1/2) (Section 3.1, the squared diagonal of P_eps).
 *   u [nframes][ny][nx] float32 -> w [npsi] float32 (npsi as described above). */
int nlrmm_tv_weights(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, int32_t temporal,
                     const float *u, double eps, float *w, void *stream);

/* Weighted regulariser Gram G = (P Psi V)^T (P Psi V) = (Psi V)^T diag(w) (Psi V) for the
 * first ell (<= 64) columns of V: the R_Psi^T R_Psi of the projected problem (Section 3.2).
 * Psi V is computed on the fly.  precision: 0 = FP64 products and accumulation (VALU);
 * 1 = FP32 MFMA (32x32x2) with FP32 accumulation per 64-pixel chunk, FP64 across chunks;
 * 2 = BF16 MFMA operands (32x32x8), same accumulation.  G [ell][ldg] float64 overwritten. */
int nlrmm_gram_psi(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, int32_t temporal,
                   int32_t ell, const float *V, const float *w, double *G, int32_t ldg,
                   int32_t precision, void *stream);

/* ------------------------------------------------------------------------------------
 * Dynamic regulariser Theta with optical-flow motion rows (Section 7, "Optical Flow
 * Regularization", eqs. "of_forward" and "Theta_OF").  temporal: 0 none, 1 frame differences
 * u(t+1) - u(t) (ANISO-TV), 2 motion rows: for every frame pair t (t = 0 .. nframes-2) the
 * forward consistency u(t) - M(s(t)) u(t+1), then for every pair the reverse consistency
 * u(t+1) - M(-s(t)) u(t), M(s) the bilinear warp that samples a frame at (k + s_x, l + s_y)
 * (pixel units, the position clamped to [0, nx-1] x [0, ny-1]).  Theta u = [Psi u; rows]
 * with the spatial rows of Psi as described above (so its length is nframes * (ny (nx-1) +
 * (ny-1) nx) plus (nframes-1) nx ny for temporal 1, 2 (nframes-1) nx ny for temporal 2).
 *   flow  DEVICE [nframes-1][2][ny][nx] float32: s_x then s_y of every pair (temporal 2 with
 *         nframes > 1 needs it and nx, ny >= 2; otherwise it may be NULL).
 * ------------------------------------------------------------------------------------ */

/* Velocity estimation (SOLVE-OF, eq. "of_forward") of every frame pair of u
 * [nframes][ny][nx]: s(t) minimises ||Y s + u_t||^2 + gamma ||L s||^2 + ridge ||s||^2, with
 * Y = [diag(d_x u(t)), diag(d_y u(t))] (central differences in pixel units, one-sided at the
 * borders), u_t = u(t+1) - u(t) and L the forward differences of each component (none across
 * the border); the l2/l2 form of the paper's lp/lq problem, gamma fixed (the paper selects it
 * by GCV) and a ridge for flat regions.  iters conjugate-gradient steps on the normal
 * equations from s = 0 for all pairs at once (FP32 vectors, FP64 inner products);
 * deterministic.  Uses the context's scratch workspace (grown as needed, refused under
 * capture).  flow [nframes-1][2][ny][nx] overwritten; nframes == 1: nothing to do. */
int nlrmm_of_estimate(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, const float *u,
                      double gamma, double ridge, int32_t iters, float *flow, void *stream);

/* out = Theta u (all rows, layout above). */
int nlrmm_theta_apply(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, int32_t temporal,
                      const float *flow, const float *u, float *out, void *stream);

/* MM weights w = ((Theta u)^2 + eps^2)^(-1/2) (Section 3.1), one per row of Theta u. */
int nlrmm_theta_weights(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes,
                        int32_t temporal, const float *flow, const float *u, double eps,
                        float *w, void *stream);

/* r += lambda Theta^T (w * Theta u), the regulariser part of the normal-equation residual
 * (w NULL: the weights of u formed with eps).  lambda DEVICE double scalar.  The motion rows'
 * transpose scatters into 64-bit fixed-point accumulators (2^-36 units) in the context's
 * scratch workspace: the result does not depend on the order of the atomic adds. */
int nlrmm_theta_grad_add(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes,
                         int32_t temporal, const float *flow, const float *u, const float *w,
                         double eps, const double *lambda, float *r, void *stream);

/* Weighted regulariser Gram (Theta V)^T diag(w) (Theta V) for the first ell columns of V, as
 * nlrmm_gram_psi (same precisions) with the temporal rows of `temporal` and `flow`. */
int nlrmm_gram_theta(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, int32_t temporal,
                     const float *flow, int32_t ell, const float *V, const float *w, double *G,
                     int32_t ldg, int32_t precision, void *stream);

/* Projected MM-GKS solve (eq. "reduced_problem") from its Grams:
 *   GA = (AV)^T AV, GP = (P Psi V)^T P Psi V, rb = (AV)^T b   (FP64, ell <= 56),
 *   scal = DEVICE {||b||^2, target}.
 * lambda: lam_fix >= 0 uses it; otherwise the discrepancy principle ||A V z - b|| = target
 * on the reduced problem (Section 3.2), searched on the log-bracket
 * [1e-10, 1e10] * tr(GA)/tr(GP) and clamped to its ends (NLRMM_ST_DP_LOW / _HIGH).
 * Outputs (DEVICE): z [ell]; out[0] = lambda, out[1] = ||A V z - b||^2 of the model. */
int nlrmm_gks_solve(nlrmm_ctx *ctx, int32_t ell, const double *GA, const double *GP,
                    int32_t ldg, const double *rb, const double *scal, double lam_fix, double *z,
                    double *out, int32_t *status, void *stream);

/* One generalized-Krylov expansion (Alg. "enlarge", after u = V z):
 *   r = A^T (A V z - b) + lambda Psi^T (w * Psi u),  u = V z,
 *   r <- r - V V^T r twice (CGS2, FP64 dot products), v = r / ||r||,
 * appended as column ell of V; column ell of A V is set to A(theta) v; the Gram GA gains
 * row/column ell and rb gains entry ell.  Breakdown (||r_perp|| <= breakdown_tol ||r||)
 * sets NLRMM_ST_BREAKDOWN (the column is still written).  Capacity: V and AV must hold
 * ell+1 columns, GA (ell+1) x ldg.  lambda is a DEVICE scalar, z DEVICE [ell]. */
int nlrmm_gks_expand(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                     const double *theta, int32_t ell, int32_t temporal, float *V, float *AV,
                     const double *z, const float *b, const float *w, const double *lambda,
                     double *GA, int32_t ldg, double *rb, double breakdown_tol,
                     int32_t *status, void *stream);

/* Recycling compression (Alg. "compress", Section 3.3): W = right singular vectors of the
 * kmin-1 largest singular values of H = [R_A; sqrt(lambda) R_Psi] (eigenvectors of
 * GA + lambda GP, sign: largest-magnitude entry positive), c = z - W W^T z and
 *   V <- V [W, c/||c||],  A V <- A V [W, c/||c||],  z <- [W^T z; ||c||]
 * (u = V z is unchanged).  GA and rb are transformed accordingly.  When ||c|| <= 1e-12 ||z||
 * the last column is zero and NLRMM_ST_COMPRESS_SKIP is set.  n, m: column lengths of V
 * and A V.  lambda DEVICE scalar; z DEVICE [ell] in, [kmin] out.  precision of the basis
 * products V [W, c] and A V [W, c]: 0 FP32 operands with FP64 accumulation, 2 BF16 operands
 * with FP32 accumulation on the matrix cores (the mixed-precision path); other values
 * return NLRMM_ENOTSUP.  The eigen-problem is FP64 in both. */
int nlrmm_recycle_compress(nlrmm_ctx *ctx, int64_t n, int64_t m, int32_t ell, int32_t kmin,
                           float *V, float *AV, double *GA, const double *GP, int32_t ldg,
                           double *rb, const double *lambda, double *z, int32_t precision,
                           int32_t *status, void *stream);

/* ------------------------------------------------------------------------------------
 * Outer driver: NL-RMM-GKS (Alg. "nl_rmmgks_two_solves", high-regularisation solve off).
 * ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t kmin, kmax;      /* recycling window (2 <= kmin <= 16, kmin < kmax <= 55) */
    int32_t solves;          /* projected solves per Enlarge; <= 0 means kmax - kmin */
    double eps;              /* smoothing of the l1 penalty (> 0) */
    double tau;              /* discrepancy-principle factor: target = tau * delta */
    double lam_fix;          /* >= 0: fixed lambda; < 0: discrepancy principle */
    int32_t param_update;    /* 0: angles fixed (RMM-GKS); 1: AltMin Gauss-Newton (Alg. "update_param");
                                2: variable projection (Section 4.2, Alg. "update_varpro");
                                3: one global offset by the full-space sensitivity equation
                                (Section 4.2, eqs. "sensitivity", "GN_system"): u_p by
                                sens_iters conjugate-gradient steps at the image u_{k+1}, the
                                step dp = -g / (h + mu_rel h) for every view, Armijo on the
                                reduced objective with u(p) in the compressed basis (needs
                                param_mode 1 and kmax + 1 - kmin >= 6, else NLRMM_ENOTSUP) */
    int32_t param_mode;      /* 0: one angle per view; 1: one global shift of all views */
    int32_t maxiter_p;       /* Gauss-Newton iterations per outer iteration */
    double mu_rel;           /* damping mu = mu_rel * mean(||D_v||^2) */
    double c1, beta, alpha0; /* Armijo constant, backtracking factor, first step */
    int32_t armijo_trials;   /* <= 32 */
    double breakdown_tol;    /* Krylov breakdown threshold */
    int32_t temporal;        /* dynamic problems: 0 none, 1 frame differences (ANISO-TV, operator
                                D1 of Section 7), 2 optical-flow motion rows (see of_* below) */
    int32_t gram_precision;  /* regulariser Gram: 0 FP64, 1 FP32 MFMA, 2 BF16 MFMA (nlrmm_gram_psi) */
    int32_t compress_precision; /* compression basis products: 0 FP32/FP64-accumulate, 2 BF16 MFMA */
    double lam_hi;           /* > 0: the optional high-regularisation solve of Section 4.3 (Alg.
                                "nl_rmmgks_two_solves"): after Compress, one RMM-GKS cycle with
                                lambda fixed at lam_hi (solves projected solves from the
                                compressed basis and u_{k+1}) gives u_hat, which the parameter
                                update uses instead of u_{k+1} (VarPro: with its compressed basis
                                and lam_hi); the image, basis, lambda and residual carried to the
                                next outer iteration stay those of the primary solve.  <= 0: off */
    int32_t sens_iters;      /* conjugate-gradient steps of the sensitivity solve (param_update 3);
                                <= 0: 50 */
    /* optical-flow temporal regulariser (temporal = 2, dynamic problems; Section 7, the OF
       branch of Alg. "dyn_nl_rmmgks"): at the start of every of_every-th outer iteration the
       velocities of all frame pairs are estimated from the current image by of_iters
       conjugate-gradient steps on eq. "of_forward" (l2/l2 form, of_gamma, of_ridge; see
       nlrmm_of_estimate), and Theta = [Psi; M_hat] (eq. "Theta_OF") is used until the next
       estimate.  Not combined with param_update 3 (NLRMM_ENOTSUP).  Defaults when <= 0:
       of_iters 200, of_gamma 0.05, of_ridge 1e-3, of_every 1. */
    int32_t of_iters;
    double of_gamma, of_ridge;
    int32_t of_every;
} nlrmm_solver_cfg;

typedef struct nlrmm_solver nlrmm_solver;

/* Allocate the solver state for images of nframes frames and up to max_views views
 * (basis V [kmax+1][n], A V [kmax+1][max_views*nbins], FP64 projected quantities). */
int nlrmm_solver_create(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes,
                        int64_t max_views, const nlrmm_solver_cfg *cfg, nlrmm_solver **out);
void nlrmm_solver_destroy(nlrmm_solver *solver);

/* Start basis: kmin+1 Golub-Kahan right vectors of A(theta) from b (full CGS2), u = 0. */
int nlrmm_solver_init(nlrmm_solver *solver, const nlrmm_batch *batch, const double *theta,
                      const float *b, void *stream);

/* Parameter initialisation by a coarse grid search over one global angle offset (the paper's
 * experiments section, "Parameter initialization"): a Golub-Kahan basis V of ell0 vectors
 * from b at the angles theta (the bidiagonalisation of nlrmm_solver_init), then for each
 * candidate offset shifts[c] the residual of the reduced least-squares problem
 * res2[c] = min_z ||A(theta + shifts[c]) V z - b||^2 (FP64 data Gram, Cholesky), and
 * theta += shifts[best] with best the smallest residual (first index on ties).
 * theta DEVICE [views], updated in place; shifts DEVICE [ncand] (radians); res2 DEVICE
 * [ncand] or NULL (then ncand <= max_views); best DEVICE int32 or NULL.  1 <= ell0 <=
 * min(kmax + 1, 56).  The solver's basis and image are left in an unspecified state: call
 * nlrmm_solver_init at the chosen angles afterwards.  A rank-deficient basis leaves a
 * candidate's residual at ||b||^2. */
int nlrmm_solver_grid_search(nlrmm_solver *solver, const nlrmm_batch *batch, double *theta,
                             const float *b, const double *shifts, int32_t ncand, int32_t ell0,
                             double *res2, int32_t *best, void *stream);

/* Full-space sensitivity of the variable-projection reduced problem for one global angle
 * offset p (Section 4.2, eq. "sensitivity"; the paper uses the RMM-GKS image for the closed
 * form u(p)): with u the solver's current image, w its regulariser weights, lam the current
 * lambda, r = A(theta) u - b and A_p u = D u (the angle derivative summed over views),
 *   (A^T A + lam Psi^T diag(w) Psi) u_p = -(D^T r + A^T D u)
 * by `iters` conjugate-gradient steps from 0, then J_r = D u + A u_p and the Gauss-Newton
 * scalars out = [g, h, dp] with g = J_r^T r + lam (Psi u_p)^T w Psi u, h = J_r^T J_r +
 * lam (Psi u_p)^T w Psi u_p, dp = -g / h (eq. "GN_system" for one parameter; 0 when h = 0).
 * theta, b DEVICE; out DEVICE [3] float64; up DEVICE [n] float32 or NULL (receives u_p).
 * Needs six spare basis columns (kmax + 1 - current columns >= 6); the basis, image and
 * lambda carried between outer iterations are unchanged (the weights buffer is
 * overwritten with the weights of u). */
int nlrmm_solver_offset_sensitivity(nlrmm_solver *solver, const nlrmm_batch *batch,
                                    const double *theta, const float *b, int32_t iters,
                                    double *out, float *up, void *stream);

/* One outer iteration on the views of `batch` (all views, or one streaming block):
 * rebase A V = A(theta_k) V; Enlarge (solves projected solves, one append between
 * consecutive solves); Compress; UPDATE-PARAM (theta updated in place); weights from the
 * new image; residual with the old operator A(theta_k); CGS2; append.  delta is the noise
 * norm of these views (discrepancy target tau*delta).  theta, b DEVICE. */
int nlrmm_solver_outer(nlrmm_solver *solver, const nlrmm_batch *batch, double *theta,
                       const float *b, double delta, void *stream);

/* Launch policy.  per_frame = 0 (default): every operator application covers all frames
 * and columns in one launch.  per_frame = 1: one launch per (column, frame) on that frame's
 * views (the plain per-frame path, same arithmetic); view_off_host (host) [nframes+1]
 * gives the frames' view offsets. */
int nlrmm_solver_set_launch(nlrmm_solver *solver, int32_t per_frame, const int64_t *view_off_host,
                            int32_t nframes);

/* DEVICE pointers into the solver: image u [n], basis V, scalars scal[16]
 * ({||b||^2, target, lambda, model residual^2, ..., [8] GN f0, g^T d, alpha, mu, f}),
 * status word; ell = current number of basis columns. */
int nlrmm_solver_state(nlrmm_solver *solver, float **u, float **V, double **scal,
                       int32_t **status, int32_t *ell);

/* Asynchronous device-to-device copies of the solver state into caller buffers (any may be
 * NULL): u_out [n] float32, scal_out [16] float64, status_out [1] int32. */
int nlrmm_solver_read(nlrmm_solver *solver, float *u_out, double *scal_out, int32_t *status_out,
                      void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NLRMM_H */
