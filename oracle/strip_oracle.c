/*
 * FP64 CPU oracle of the angle-parameterised parallel-beam projector.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the test-suite, the package smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header or constant generator with the HIP library.
 *
 * Operator (the paper's forward model H(p)u + e = b, Section 1, eq.
 * "nonlinear_forward", with p the per-view angles and H the Radon transform
 * of Section 6.2 at perturbed angles; the discretisation is this project's
 * reading because the paper delegates it to a toolbox):
 *
 *   a[v][j][pix] = |Q_pix  ∩  {e_j <= p.n(theta_v) < e_{j+1}}| / ds
 *
 * Q_pix is the pixel square, n = (cos, sin), e_j = s0 + j ds the bin edges.
 * The area is Phi(e_{j+1} - c) - Phi(e_j - c) where c = centre.n and Phi(v)
 * is the integral of the pixel's chord-length profile (a trapezoid).  The
 * angle derivative (Leibniz rule on the moving strip boundaries) is
 *
 *   d a[v][j][pix] / d theta_v = (M(e_j) - M(e_{j+1})) / ds,
 *   M(e) = integral over the chord {p in Q : p.n = e} of (p.t) dtau,
 *   t = (-sin, cos),
 *
 * evaluated here by Liang-Barsky clipping of the line against the square.
 *
 * Layouts: image x[col][frame][l][k] (k along x fastest, N x N per frame),
 * sinogram y[col][view][bin]; views of frame f are view_off[f] ..
 * view_off[f+1]-1; angles in radians.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double c, s;      /* cos, sin of the view angle */
    double wo, wi;    /* outer / inner half-widths of the pixel footprint */
    double rho;       /* ramp width = wo - wi */
    double h;         /* plateau chord length */
    double D, D2;     /* pixel width and area */
} view_t;

static view_t view_make(double theta, double D)
{
    view_t q;
    q.c = cos(theta);
    q.s = sin(theta);
    double p = D * fabs(q.c), r = D * fabs(q.s);
    q.wo = 0.5 * (p + r);
    q.wi = 0.5 * fabs(p - r);
    q.rho = q.wo - q.wi;
    q.h = D / fmax(fabs(q.c), fabs(q.s));
    q.D = D;
    q.D2 = D * D;
    return q;
}

/* Area of the pixel on the side p.n < centre.n + v (cumulative footprint). */
static double phi(double v, const view_t *q)
{
    if (v <= -q->wo) return 0.0;
    if (v >= q->wo) return q->D2;
    if (v < -q->wi) {                       /* left ramp: a corner triangle */
        double t = v + q->wo;
        return q->h * t * t / (2.0 * q->rho);
    }
    if (v <= q->wi)                         /* plateau */
        return 0.5 * q->h * q->rho + q->h * (v + q->wi);
    double t = q->wo - v;                   /* right ramp */
    return q->D2 - q->h * t * t / (2.0 * q->rho);
}

/* First moment along t of the chord at offset v from the pixel centre, whose
 * own t-coordinate is tc: integral of (tc + tau) over the clipped chord. */
static double chord_moment(double v, double tc, const view_t *q)
{
    const double H = 0.5 * q->D;
    double lo = -INFINITY, hi = INFINITY;
    /* x(tau) = v c - tau s must lie in [-H, H] */
    if (q->s != 0.0) {
        double a = (v * q->c - H) / q->s, b = (v * q->c + H) / q->s;
        lo = fmax(lo, fmin(a, b));
        hi = fmin(hi, fmax(a, b));
    } else if (fabs(v * q->c) > H) {
        return 0.0;
    }
    /* y(tau) = v s + tau c must lie in [-H, H] */
    if (q->c != 0.0) {
        double a = (-H - v * q->s) / q->c, b = (H - v * q->s) / q->c;
        lo = fmax(lo, fmin(a, b));
        hi = fmin(hi, fmax(a, b));
    } else if (fabs(v * q->s) > H) {
        return 0.0;
    }
    if (!(hi > lo)) return 0.0;
    return tc * (hi - lo) + 0.5 * (hi * hi - lo * lo);
}

typedef struct {
    int N, nb;
    double s0, ds;
} geom_t;

/* Bins touched by the footprint [cc - wo, cc + wo], clipped to the detector. */
static void bin_range(double cc, const view_t *q, const geom_t *g, int *jlo, int *jhi)
{
    int a = (int)floor((cc - q->wo - g->s0) / g->ds);
    int b = (int)floor((cc + q->wo - g->s0) / g->ds);
    if (a < 0) a = 0;
    if (b > g->nb - 1) b = g->nb - 1;
    *jlo = a;
    *jhi = b;
}

static int frame_of(int v, int nframes, const int64_t *view_off)
{
    int f = 0;
    while (f + 1 < nframes && v >= view_off[f + 1]) ++f;
    return f;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* y = A(theta) x for every column. */
int ora_project(int N, int nb, double s0, double ds, int nframes, const int64_t *view_off,
                int ncols, const double *x, const double *theta, double *y, int nthreads)
{
    const geom_t g = {N, nb, s0, ds};
    const double D = 2.0 / N;
    const int V = (int)view_off[nframes];
    const int64_t npix = (int64_t)N * N;
    set_threads(nthreads);
    for (int col = 0; col < ncols; ++col) {
        const double *xc = x + (int64_t)col * nframes * npix;
        double *yc = y + (int64_t)col * V * nb;
#pragma omp parallel for schedule(dynamic, 1)
        for (int v = 0; v < V; ++v) {
            const view_t q = view_make(theta[v], D);
            const double *xf = xc + (int64_t)frame_of(v, nframes, view_off) * npix;
            double *row = yc + (int64_t)v * nb;
            for (int j = 0; j < nb; ++j) row[j] = 0.0;
            for (int l = 0; l < N; ++l) {
                const double yl = -1.0 + (l + 0.5) * D;
                for (int k = 0; k < N; ++k) {
                    const double xv = xf[(int64_t)l * N + k];
                    const double xk = -1.0 + (k + 0.5) * D;
                    const double cc = xk * q.c + yl * q.s;
                    int jlo, jhi;
                    bin_range(cc, &q, &g, &jlo, &jhi);
                    for (int j = jlo; j <= jhi; ++j) {
                        const double e0 = s0 + j * ds, e1 = s0 + (j + 1) * ds;
                        const double w = (phi(e1 - cc, &q) - phi(e0 - cc, &q)) / ds;
                        row[j] += w * xv;
                    }
                }
            }
        }
    }
    return 0;
}

/* x = A(theta)^T y for every column (exact transpose of ora_project). */
int ora_backproject(int N, int nb, double s0, double ds, int nframes, const int64_t *view_off,
                    int ncols, const double *y, const double *theta, double *x, int nthreads)
{
    const geom_t g = {N, nb, s0, ds};
    const double D = 2.0 / N;
    const int V = (int)view_off[nframes];
    const int64_t npix = (int64_t)N * N;
    set_threads(nthreads);
    view_t *qs = (view_t *)malloc(sizeof(view_t) * (size_t)(V > 0 ? V : 1));
    for (int v = 0; v < V; ++v) qs[v] = view_make(theta[v], D);
    for (int col = 0; col < ncols; ++col) {
        const double *yc = y + (int64_t)col * V * nb;
        double *xc = x + (int64_t)col * nframes * npix;
        for (int f = 0; f < nframes; ++f) {
            double *xf = xc + (int64_t)f * npix;
#pragma omp parallel for schedule(dynamic, 1)
            for (int l = 0; l < N; ++l) {
                const double yl = -1.0 + (l + 0.5) * D;
                for (int k = 0; k < N; ++k) {
                    const double xk = -1.0 + (k + 0.5) * D;
                    double acc = 0.0;
                    for (int64_t v = view_off[f]; v < view_off[f + 1]; ++v) {
                        const view_t *q = &qs[v];
                        const double cc = xk * q->c + yl * q->s;
                        int jlo, jhi;
                        bin_range(cc, q, &g, &jlo, &jhi);
                        for (int j = jlo; j <= jhi; ++j) {
                            const double e0 = s0 + j * ds, e1 = s0 + (j + 1) * ds;
                            const double w = (phi(e1 - cc, q) - phi(e0 - cc, q)) / ds;
                            acc += w * yc[v * nb + j];
                        }
                    }
                    xf[(int64_t)l * N + k] = acc;
                }
            }
        }
    }
    free(qs);
    return 0;
}

/* Dy[v][j] = d y[v][j] / d theta_v for every column. */
int ora_dtheta(int N, int nb, double s0, double ds, int nframes, const int64_t *view_off,
               int ncols, const double *x, const double *theta, double *dy, int nthreads)
{
    const geom_t g = {N, nb, s0, ds};
    const double D = 2.0 / N;
    const int V = (int)view_off[nframes];
    const int64_t npix = (int64_t)N * N;
    set_threads(nthreads);
    for (int col = 0; col < ncols; ++col) {
        const double *xc = x + (int64_t)col * nframes * npix;
        double *dc = dy + (int64_t)col * V * nb;
#pragma omp parallel for schedule(dynamic, 1)
        for (int v = 0; v < V; ++v) {
            const view_t q = view_make(theta[v], D);
            const double *xf = xc + (int64_t)frame_of(v, nframes, view_off) * npix;
            double *row = dc + (int64_t)v * nb;
            for (int j = 0; j < nb; ++j) row[j] = 0.0;
            for (int l = 0; l < N; ++l) {
                const double yl = -1.0 + (l + 0.5) * D;
                for (int k = 0; k < N; ++k) {
                    const double xv = xf[(int64_t)l * N + k];
                    const double xk = -1.0 + (k + 0.5) * D;
                    const double cc = xk * q.c + yl * q.s;
                    const double tc = -xk * q.s + yl * q.c;
                    int jlo, jhi;
                    bin_range(cc, &q, &g, &jlo, &jhi);
                    for (int j = jlo; j <= jhi; ++j) {
                        const double e0 = s0 + j * ds, e1 = s0 + (j + 1) * ds;
                        const double dw = (chord_moment(e0 - cc, tc, &q) -
                                           chord_moment(e1 - cc, tc, &q)) / ds;
                        row[j] += dw * xv;
                    }
                }
            }
        }
    }
    return 0;
}

/* x = D(theta)^T r with D the angle derivative above: x[pix] = sum over views v of frame f
 * and bins j of (M(e_j) - M(e_{j+1})) / ds * r[v][j] (the same weights as ora_dtheta,
 * gathered per pixel), for every column. */
int ora_dtheta_t(int N, int nb, double s0, double ds, int nframes, const int64_t *view_off,
                 int ncols, const double *r, const double *theta, double *x, int nthreads)
{
    const geom_t g = {N, nb, s0, ds};
    const double D = 2.0 / N;
    const int V = (int)view_off[nframes];
    const int64_t npix = (int64_t)N * N;
    set_threads(nthreads);
    view_t *qs = (view_t *)malloc(sizeof(view_t) * (size_t)(V > 0 ? V : 1));
    for (int v = 0; v < V; ++v) qs[v] = view_make(theta[v], D);
    for (int col = 0; col < ncols; ++col) {
        const double *rc = r + (int64_t)col * V * nb;
        double *xc = x + (int64_t)col * nframes * npix;
        for (int f = 0; f < nframes; ++f) {
            double *xf = xc + (int64_t)f * npix;
#pragma omp parallel for schedule(dynamic, 1)
            for (int l = 0; l < N; ++l) {
                const double yl = -1.0 + (l + 0.5) * D;
                for (int k = 0; k < N; ++k) {
                    const double xk = -1.0 + (k + 0.5) * D;
                    double acc = 0.0;
                    for (int64_t v = view_off[f]; v < view_off[f + 1]; ++v) {
                        const view_t *q = &qs[v];
                        const double cc = xk * q->c + yl * q->s;
                        const double tc = -xk * q->s + yl * q->c;
                        int jlo, jhi;
                        bin_range(cc, q, &g, &jlo, &jhi);
                        for (int j = jlo; j <= jhi; ++j) {
                            const double e0 = s0 + j * ds, e1 = s0 + (j + 1) * ds;
                            const double dw = (chord_moment(e0 - cc, tc, q) -
                                               chord_moment(e1 - cc, tc, q)) / ds;
                            acc += dw * rc[v * nb + j];
                        }
                    }
                    xf[(int64_t)l * N + k] = acc;
                }
            }
        }
    }
    free(qs);
    return 0;
}

/* Dense A(theta) (V*nb x N*N) and dA/dtheta (same shape) for tiny grids. */
int ora_dense(int N, int nb, double s0, double ds, int V, const double *theta,
              double *A, double *dA)
{
    const geom_t g = {N, nb, s0, ds};
    const double D = 2.0 / N;
    const int64_t npix = (int64_t)N * N;
    memset(A, 0, sizeof(double) * (size_t)V * nb * npix);
    if (dA) memset(dA, 0, sizeof(double) * (size_t)V * nb * npix);
    for (int v = 0; v < V; ++v) {
        const view_t q = view_make(theta[v], D);
        for (int l = 0; l < N; ++l) {
            const double yl = -1.0 + (l + 0.5) * D;
            for (int k = 0; k < N; ++k) {
                const double xk = -1.0 + (k + 0.5) * D;
                const double cc = xk * q.c + yl * q.s;
                const double tc = -xk * q.s + yl * q.c;
                int jlo, jhi;
                bin_range(cc, &q, &g, &jlo, &jhi);
                for (int j = jlo; j <= jhi; ++j) {
                    const double e0 = s0 + j * ds, e1 = s0 + (j + 1) * ds;
                    const int64_t row = (int64_t)v * nb + j, colx = (int64_t)l * N + k;
                    A[row * npix + colx] = (phi(e1 - cc, &q) - phi(e0 - cc, &q)) / ds;
                    if (dA)
                        dA[row * npix + colx] =
                            (chord_moment(e0 - cc, tc, &q) - chord_moment(e1 - cc, tc, &q)) / ds;
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Fan beam (the paper's CT geometry, Section 6.2; its toolbox geometry is not stated, so this
 * is a reading).  The source is at distance R from the rotation centre, at S = -R t(theta),
 * t = (-sin, cos); the ray of detector coordinate s passes through S and the point s n(theta)
 * of the line through the centre along n = (cos, sin).  Near a pixel centre c the rays are
 * locally parallel: the ray through c has direction t(alpha), alpha = theta - gamma,
 * tan gamma = (c.n) / b with b = R + c.t, and crosses the detector line at s_c = R (c.n) / b;
 * a shift w across the rays at c moves s by m w with m = R l / b^2, l = |c - S| =
 * sqrt((c.n)^2 + b^2).  The weight is the parallel-beam strip weight of the pixel for the
 * direction alpha, with its footprint centred at s_c and scaled by m, and the bin value the
 * s-average over the bin of the chord length:
 *   a[v][j][pix] = (m / ds) [Phi_alpha((e_{j+1} - s_c) / m) - Phi_alpha((e_j - s_c) / m)].
 * It is exact to first order in the pixel size, and as R -> infinity (gamma -> 0, m -> 1) it
 * is the strip-area model above.  The angle derivative of F(e) = m Phi_alpha(v),
 * v = (e - s_c) / m, is
 *   dF/dtheta = m' Phi_alpha(v) - L(v) (s_c' + v m') - m L(v) mu(v) alpha',
 * L the chord length at offset v and L mu its first moment along t(alpha) about the centre
 * (the change of Phi_alpha with its angle at fixed offset), with
 *   s_c' = R (c.t b + (c.n)^2) / b^2,   gamma' = (c.t b + (c.n)^2) / l^2,   alpha' = 1 - gamma',
 *   m' = R (c.n) (2 l^2 - R b) / (l b^3)
 * (d(c.n)/dtheta = c.t, d(c.t)/dtheta = -c.n);  d a / d theta = (dF(e_{j+1}) - dF(e_j)) / ds.
 * ------------------------------------------------------------------------------------ */

/* Chord length through the pixel at offset v from its centre (Liang-Barsky, as above). */
static double chord_len(double v, const view_t *q)
{
    const double H = 0.5 * q->D;
    double lo = -INFINITY, hi = INFINITY;
    if (q->s != 0.0) {
        double a = (v * q->c - H) / q->s, b = (v * q->c + H) / q->s;
        lo = fmax(lo, fmin(a, b));
        hi = fmin(hi, fmax(a, b));
    } else if (fabs(v * q->c) > H) {
        return 0.0;
    }
    if (q->c != 0.0) {
        double a = (-H - v * q->s) / q->c, b = (H - v * q->s) / q->c;
        lo = fmax(lo, fmin(a, b));
        hi = fmin(hi, fmax(a, b));
    } else if (fabs(v * q->s) > H) {
        return 0.0;
    }
    return hi > lo ? hi - lo : 0.0;
}

/* A view record for the local ray direction alpha given its cosine and sine. */
static view_t view_from_cs(double c, double s, double D)
{
    view_t q;
    q.c = c;
    q.s = s;
    double p = D * fabs(c), r = D * fabs(s);
    q.wo = 0.5 * (p + r);
    q.wi = 0.5 * fabs(p - r);
    q.rho = q.wo - q.wi;
    q.h = D / fmax(fabs(c), fabs(s));
    q.D = D;
    q.D2 = D * D;
    return q;
}

typedef struct {
    view_t a;                /* the pixel's local ray direction alpha */
    double sc, m;            /* projection and magnification */
    double dsc, dm, dalpha;  /* their angle derivatives, and alpha' */
} fanpix_t;

static fanpix_t fan_pixel(double xk, double yl, const view_t *q, double R)
{
    fanpix_t f;
    const double cn = xk * q->c + yl * q->s;
    const double ct = -xk * q->s + yl * q->c;
    const double b = R + ct;
    const double l2 = cn * cn + b * b, l = sqrt(l2);
    const double cg = b / l, sg = cn / l;   /* cos, sin gamma */
    f.a = view_from_cs(q->c * cg + q->s * sg, q->s * cg - q->c * sg, q->D);
    f.sc = R * cn / b;
    f.m = R * l / (b * b);
    f.dsc = R * (ct * b + cn * cn) / (b * b);
    f.dm = R * cn * (2.0 * l2 - R * b) / (l * b * b * b);
    f.dalpha = 1.0 - (ct * b + cn * cn) / l2;
    return f;
}

/* Bins touched by the footprint [s_c - m wo, s_c + m wo], clipped to the detector. */
static void fan_bin_range(const fanpix_t *f, const geom_t *g, int *jlo, int *jhi)
{
    int a = (int)floor((f->sc - f->m * f->a.wo - g->s0) / g->ds);
    int b = (int)floor((f->sc + f->m * f->a.wo - g->s0) / g->ds);
    if (a < 0) a = 0;
    if (b > g->nb - 1) b = g->nb - 1;
    *jlo = a;
    *jhi = b;
}

static double fan_weight(int j, const fanpix_t *f, const geom_t *g)
{
    const double e0 = g->s0 + j * g->ds, e1 = g->s0 + (j + 1) * g->ds;
    return f->m * (phi((e1 - f->sc) / f->m, &f->a) - phi((e0 - f->sc) / f->m, &f->a)) / g->ds;
}

/* d/dtheta of F(e) = m Phi_alpha((e - s_c) / m) */
static double fan_dF(double e, const fanpix_t *f)
{
    const double v = (e - f->sc) / f->m;
    const double L = chord_len(v, &f->a);
    const double Lmu = chord_moment(v, 0.0, &f->a);
    return f->dm * phi(v, &f->a) - L * (f->dsc + v * f->dm) - f->m * Lmu * f->dalpha;
}

static double fan_dweight(int j, const fanpix_t *f, const geom_t *g)
{
    const double e0 = g->s0 + j * g->ds, e1 = g->s0 + (j + 1) * g->ds;
    return (fan_dF(e1, f) - fan_dF(e0, f)) / g->ds;
}

/* y = A_fan(theta) x (mode 0) or D_fan(theta) x = d(A_fan x)/dtheta per view (mode 1). */
static int fan_apply(int mode, int N, int nb, double s0, double ds, double R, int nframes,
                     const int64_t *view_off, int ncols, const double *x, const double *theta,
                     double *y, int nthreads)
{
    const geom_t g = {N, nb, s0, ds};
    const double D = 2.0 / N;
    const int V = (int)view_off[nframes];
    const int64_t npix = (int64_t)N * N;
    set_threads(nthreads);
    for (int col = 0; col < ncols; ++col) {
        const double *xc = x + (int64_t)col * nframes * npix;
        double *yc = y + (int64_t)col * V * nb;
#pragma omp parallel for schedule(dynamic, 1)
        for (int v = 0; v < V; ++v) {
            const view_t q = view_make(theta[v], D);
            const double *xf = xc + (int64_t)frame_of(v, nframes, view_off) * npix;
            double *yv = yc + (int64_t)v * nb;
            for (int j = 0; j < nb; ++j) yv[j] = 0.0;
            for (int l = 0; l < N; ++l) {
                const double yl = -1.0 + (l + 0.5) * D;
                for (int k = 0; k < N; ++k) {
                    const double xv = xf[(int64_t)l * N + k];
                    if (xv == 0.0) continue;
                    const double xk = -1.0 + (k + 0.5) * D;
                    const fanpix_t f = fan_pixel(xk, yl, &q, R);
                    int jlo, jhi;
                    fan_bin_range(&f, &g, &jlo, &jhi);
                    for (int j = jlo; j <= jhi; ++j)
                        yv[j] += xv * (mode == 0 ? fan_weight(j, &f, &g) : fan_dweight(j, &f, &g));
                }
            }
        }
    }
    return 0;
}

int ora_fan_project(int N, int nb, double s0, double ds, double R, int nframes,
                    const int64_t *view_off, int ncols, const double *x, const double *theta,
                    double *y, int nthreads)
{
    return fan_apply(0, N, nb, s0, ds, R, nframes, view_off, ncols, x, theta, y, nthreads);
}

int ora_fan_dtheta(int N, int nb, double s0, double ds, double R, int nframes,
                   const int64_t *view_off, int ncols, const double *x, const double *theta,
                   double *y, int nthreads)
{
    return fan_apply(1, N, nb, s0, ds, R, nframes, view_off, ncols, x, theta, y, nthreads);
}

/* x = A_fan(theta)^T y (mode 0) or D_fan(theta)^T y (mode 1), per pixel over views. */
static int fan_apply_t(int mode, int N, int nb, double s0, double ds, double R, int nframes,
                       const int64_t *view_off, int ncols, const double *y,
                       const double *theta, double *x, int nthreads)
{
    const geom_t g = {N, nb, s0, ds};
    const double D = 2.0 / N;
    const int V = (int)view_off[nframes];
    const int64_t npix = (int64_t)N * N;
    set_threads(nthreads);
    view_t *qs = (view_t *)malloc(sizeof(view_t) * (size_t)(V > 0 ? V : 1));
    for (int v = 0; v < V; ++v) qs[v] = view_make(theta[v], D);
    for (int col = 0; col < ncols; ++col) {
        const double *yc = y + (int64_t)col * V * nb;
        double *xc = x + (int64_t)col * nframes * npix;
        for (int fr = 0; fr < nframes; ++fr) {
            double *xf = xc + (int64_t)fr * npix;
#pragma omp parallel for schedule(dynamic, 1)
            for (int l = 0; l < N; ++l) {
                const double yl = -1.0 + (l + 0.5) * D;
                for (int k = 0; k < N; ++k) {
                    const double xk = -1.0 + (k + 0.5) * D;
                    double acc = 0.0;
                    for (int64_t v = view_off[fr]; v < view_off[fr + 1]; ++v) {
                        const fanpix_t f = fan_pixel(xk, yl, &qs[v], R);
                        int jlo, jhi;
                        fan_bin_range(&f, &g, &jlo, &jhi);
                        for (int j = jlo; j <= jhi; ++j)
                            acc += yc[v * nb + j] *
                                   (mode == 0 ? fan_weight(j, &f, &g) : fan_dweight(j, &f, &g));
                    }
                    xf[(int64_t)l * N + k] = acc;
                }
            }
        }
    }
    free(qs);
    return 0;
}

int ora_fan_backproject(int N, int nb, double s0, double ds, double R, int nframes,
                        const int64_t *view_off, int ncols, const double *y, const double *theta,
                        double *x, int nthreads)
{
    return fan_apply_t(0, N, nb, s0, ds, R, nframes, view_off, ncols, y, theta, x, nthreads);
}

int ora_fan_dtheta_t(int N, int nb, double s0, double ds, double R, int nframes,
                     const int64_t *view_off, int ncols, const double *y, const double *theta,
                     double *x, int nthreads)
{
    return fan_apply_t(1, N, nb, s0, ds, R, nframes, view_off, ncols, y, theta, x, nthreads);
}

int ora_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
