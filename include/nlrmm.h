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

/* Image grid and detector.  Square pixels of width d. */
typedef struct {
    int32_t nx, ny;   /* pixels along x (fastest index) and y, 1 .. 16384 */
    double x0, y0;    /* lower-left corner of the image */
    double d;         /* pixel width, > 0 */
    int32_t nbins;    /* detector bins, 1 .. 65536 */
    double s0, ds;    /* bin j covers [s0 + j ds, s0 + (j+1) ds), ds > 0 */
} nlrmm_geom;

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

/* Create a context on HIP device `device`.  Allocates nothing yet; workspace grows on
 * the first call that needs it (outside graph capture).  *out receives the handle. */
int nlrmm_ctx_create(nlrmm_ctx **out, int device);
void nlrmm_ctx_destroy(nlrmm_ctx *ctx);

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

#ifdef __cplusplus
}
#endif
#endif /* NLRMM_H */
