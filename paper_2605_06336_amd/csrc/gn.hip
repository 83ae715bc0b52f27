// Gauss-Newton angle update (Alg. "update_param") and small device-side helpers.
//
// Per-view angles: the Jacobian column of theta_v is non-zero only on view v's rows, so
// J^T J is diagonal with entries h_v = ||D_v||^2 and the damped step is
//   d_v = -g_v / (h_v + mu),  g_v = <D_v, r_v>,  r = A(theta) u - b,
// with mu = mu_rel * mean(h).  A single global shift (the paper's experiments) uses
// g = sum g_v, h = sum h_v.  The Armijo backtracking (one alpha for all angles) is run
// as a fixed sequence of trial projections; a device flag set by the first accepted
// trial makes the remaining trials return immediately, so no host round trip is needed.
#include "internal.h"
#include "krylov.h"

#include <math.h>

namespace nlrmm {
namespace {

constexpr int BLK = 256;

__device__ double block_sum2(double v, double *sbuf)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sbuf[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < BLK / 64; ++i) t += sbuf[i];
    return t;
}

__global__ __launch_bounds__(BLK) void gn_prepare_k(const double *__restrict__ g,
                                                    const double *__restrict__ h,
                                                    const double *__restrict__ rn2, int64_t V,
                                                    int scalar_mode, double mu_rel,
                                                    double *__restrict__ dir,
                                                    double *__restrict__ sc, int *accepted)
{
    __shared__ double sbuf[BLK / 64];
    const int tid = threadIdx.x;
    double sg = 0.0, sh = 0.0, sr = 0.0;
    for (int64_t v = tid; v < V; v += BLK) {
        sg += g[v];
        sh += h[v];
        sr += rn2[v];
    }
    sg = block_sum2(sg, sbuf);
    sh = block_sum2(sh, sbuf);
    sr = block_sum2(sr, sbuf);
    double gd = 0.0, mu;
    if (scalar_mode) {
        mu = mu_rel * sh;
        const double d = -sg / (sh + mu);
        for (int64_t v = tid; v < V; v += BLK) dir[v] = d;
        gd = sg * d;
    } else {
        mu = mu_rel * sh / (double)V;
        double part = 0.0;
        for (int64_t v = tid; v < V; v += BLK) {
            const double d = -g[v] / (h[v] + mu);
            dir[v] = d;
            part += g[v] * d;
        }
        gd = block_sum2(part, sbuf);
    }
    if (tid == 0) {
        sc[0] = 0.5 * sr;   // f0
        sc[1] = gd;         // g^T d
        sc[2] = 0.0;        // accepted alpha
        sc[3] = mu;
        *accepted = 0;
    }
}

__global__ __launch_bounds__(BLK) void armijo_check_k(const double *__restrict__ part_r,
                                                      int64_t nparts,
                                                      const double *__restrict__ alphas, int q,
                                                      double c1, double *__restrict__ sc,
                                                      int *accepted)
{
    __shared__ double sbuf[BLK / 64];
    if (*accepted) return;   // uniform
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nparts; i += BLK) s += part_r[i];
    s = block_sum2(s, sbuf);
    if (threadIdx.x == 0) {
        const double f = 0.5 * s;
        const double a = alphas[q];
        if (f <= sc[0] + c1 * a * sc[1]) {
            *accepted = 1;
            sc[2] = a;
            sc[4] = f;
        }
    }
}

__global__ void gn_apply_k(double *__restrict__ theta, const double *__restrict__ dir, int64_t V,
                           const double *__restrict__ sc, const int *__restrict__ accepted,
                           int *status)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double a = *accepted ? sc[2] : 0.0;
    if (v < V) theta[v] += a * dir[v];
    if (v == 0 && !*accepted) atomicOr(status, NLRMM_ST_ARMIJO);
}

__global__ void scatter_gram_k(const double *__restrict__ col, int ell, double *__restrict__ G,
                               int ldg, double *__restrict__ rb)
{
    // col = [G[0..ell][ell], rb[ell]] from one multi-dot launch
    const int i = threadIdx.x;
    if (i <= ell) {
        G[i * ldg + ell] = col[i];
        G[ell * ldg + i] = col[i];
    }
    if (i == 0) rb[ell] = col[ell + 1];
}

__global__ void symmetrize_k(double *G, int ldg, int ell)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ell * ell) return;
    const int i = t / ell, j = t % ell;
    if (i > j) G[i * ldg + j] = G[j * ldg + i];
}

__global__ void copy_f64_k(const double *__restrict__ s, double *__restrict__ d, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

__global__ void fill_f64_k(double *d, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = v;
}

__global__ void fill_f32_k(float *d, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = v;
}

__global__ void fill_i32_k(int *d, int64_t n, int v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = v;
}

// dst = src / sqrt(norm2[0]); norm_out[0] = sqrt(norm2[0])
__global__ void scale_into_k(const float *__restrict__ src, const double *__restrict__ norm2,
                             int64_t n, float *__restrict__ dst, double *norm_out, int *status)
{
    const double nr = sqrt(fmax(norm2[0], 0.0));
    const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (norm_out) norm_out[0] = nr;
        if (!(nr > 0.0) || !isfinite(nr)) atomicOr(status, NLRMM_ST_NONFINITE);
    }
    if (i < n) dst[i] = (float)((double)src[i] * inv);
}


// Residual of the reduced least-squares problem of one grid candidate:
// min_z ||A V z - b||^2 = ||b||^2 - rb^T G^-1 rb with G = (A V)^T A V = L L^T and rb =
// (A V)^T b, i.e. ||b||^2 - ||L^-1 rb||^2 (one thread; ell <= 56).  A non-positive pivot
// (rank-deficient basis) leaves the candidate's residual at ||b||^2.
__global__ void grid_residual_k(const double *__restrict__ G, int ldg,
                                const double *__restrict__ rb, const double *__restrict__ bnorm2,
                                int ell, double *__restrict__ res2)
{
    __shared__ double L[56][56];
    __shared__ double y[56];
    if (threadIdx.x != 0) return;
    double fit = 0.0;
    bool ok = true;
    for (int i = 0; i < ell && ok; ++i) {
        for (int j = 0; j <= i; ++j) {
            double sum = G[i * ldg + j];
            for (int k = 0; k < j; ++k) sum -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(sum > 0.0)) {
                    ok = false;
                    break;
                }
                L[i][i] = sqrt(sum);
            } else {
                L[i][j] = sum / L[j][j];
            }
        }
        if (!ok) break;
        double t = rb[i];
        for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
        y[i] = t / L[i][i];
        fit += y[i] * y[i];
    }
    res2[0] = ok ? bnorm2[0] - fit : bnorm2[0];
}

// The smallest residual of the candidates (first index on ties) and theta_v += s_best.
__global__ void grid_pick_k(const double *__restrict__ res2, int ncand,
                            const double *__restrict__ shifts, double *__restrict__ theta,
                            int64_t V, int *__restrict__ best)
{
    __shared__ int sbest;
    if (threadIdx.x == 0) {
        int k = 0;
        for (int c = 1; c < ncand; ++c)
            if (res2[c] < res2[k]) k = c;
        sbest = k;
        if (best != nullptr) best[0] = k;
    }
    __syncthreads();
    const double sh = shifts[sbest];
    for (int64_t v = threadIdx.x; v < V; v += blockDim.x) theta[v] += sh;
}


// Conjugate-gradient coefficients kept on the device (c: [0] rr, [1] p^T M p, [2] new rr,
// [3] alpha, [4] -alpha, [5] beta): mode 0 alpha = rr / p^T M p; mode 1 beta = new rr / rr
// and rr <- new rr.  A zero denominator (converged) gives a zero coefficient.
__global__ void cg_coef_k(double *c, int mode)
{
    if (threadIdx.x != 0) return;
    if (mode == 0) {
        const double a = c[1] != 0.0 ? c[0] / c[1] : 0.0;
        c[3] = a;
        c[4] = -a;
    } else {
        c[5] = c[0] != 0.0 ? c[2] / c[0] : 0.0;
        c[0] = c[2];
    }
}

// Gauss-Newton step of one global offset from the sensitivity dots: d1 = [J_r^T J_r,
// r^T J_r], d2 = [u_p^T Psi^T w Psi u, u_p^T Psi^T w Psi u_p]; out = [g, h, dp = -g / h].
__global__ void offset_gn_k(const double *d1, const double *d2, const double *lamp,
                            double *out)
{
    if (threadIdx.x != 0) return;
    const double lam = lamp[0];
    const double g = d1[1] + lam * d2[0];
    const double h = d1[0] + lam * d2[1];
    out[0] = g;
    out[1] = h;
    out[2] = h > 0.0 ? -g / h : 0.0;
}

// Direction of the Gauss-Newton step of one global offset, the same for every view: from
// gh = [g, h] of the sensitivity solve, dp = -g / (h + mu) with mu = mu_rel h (0 when h <= 0);
// the Gauss-Newton scalars sc get g dp (the Armijo slope) and mu.
__global__ void offset_dir_k(const double *__restrict__ gh, double mu_rel, int64_t V,
                             double *__restrict__ dir, double *__restrict__ sc)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double g = gh[0], h = gh[1];
    const double mu = mu_rel * h;
    const double dp = h + mu > 0.0 ? -g / (h + mu) : 0.0;
    if (v < V) dir[v] = dp;
    if (v == 0) {
        sc[1] = g * dp;
        sc[3] = mu;
    }
}

// Image of an Armijo trial of the global-offset step, to first order in the offset:
// out = u + (alphas[q] dp) u_p with dp = dir[0] (skipped once a trial was accepted).
__global__ void lin_image_k(const float *__restrict__ u, const float *__restrict__ up, int64_t n,
                            const double *__restrict__ alphas, int q,
                            const double *__restrict__ dir, const int *__restrict__ accepted,
                            float *__restrict__ out)
{
    if (*accepted) return;   // uniform
    const double c = alphas[q] * dir[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)((double)u[i] + c * (double)up[i]);
}

// Reduced objective of the global-offset step, f = 1/2 sum_v ||r_v||^2 + lam/2 reg (rn2 the
// per-view squared residuals, reg = ||sqrt(w) Psi u||^2, summed in a fixed order): with q < 0
// it is f0 (sc[0]) and clears the acceptance flag; otherwise the Armijo test of trial q
// against sc[0] + c1 alphas[q] sc[1] (skipped once a trial was accepted).
__global__ __launch_bounds__(BLK) void sens_objective_k(const double *__restrict__ rn2, int64_t V,
                                                        const double *__restrict__ reg,
                                                        const double *__restrict__ lamp,
                                                        const double *__restrict__ alphas, int q,
                                                        double c1, double *__restrict__ sc,
                                                        int *accepted)
{
    __shared__ double sbuf[BLK / 64];
    if (q >= 0 && *accepted) return;   // uniform
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < V; i += BLK) s += rn2[i];
    s = block_sum2(s, sbuf);
    if (threadIdx.x == 0) {
        const double f = 0.5 * s + 0.5 * lamp[0] * reg[0];
        if (q < 0) {
            sc[0] = f;
            *accepted = 0;
        } else {
            const double a = alphas[q];
            if (f <= sc[0] + c1 * a * sc[1]) {
                *accepted = 1;
                sc[2] = a;
                sc[4] = f;
            }
        }
    }
}

}  // namespace

#define LAUNCH_OK (hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP)

int k_gn_prepare(const double *g, const double *h, const double *rn2, int64_t V, int scalar_mode,
                 double mu_rel, double *dir, double *sc, int *accepted, hipStream_t s)
{
    gn_prepare_k<<<1, BLK, 0, s>>>(g, h, rn2, V, scalar_mode, mu_rel, dir, sc, accepted);
    return LAUNCH_OK;
}

int k_armijo_check(const double *part_r, int64_t nparts, const double *alphas, int q, double c1,
                   double *sc, int *accepted, hipStream_t s)
{
    armijo_check_k<<<1, BLK, 0, s>>>(part_r, nparts, alphas, q, c1, sc, accepted);
    return LAUNCH_OK;
}

int k_gn_apply(double *theta, const double *dir, int64_t V, const double *sc,
               const int *accepted, int *status, hipStream_t s)
{
    gn_apply_k<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(theta, dir, V, sc, accepted, status);
    return LAUNCH_OK;
}

int k_scatter_gram(const double *col, int ell, double *G, int ldg, double *rb, hipStream_t s)
{
    scatter_gram_k<<<1, 128, 0, s>>>(col, ell, G, ldg, rb);
    return LAUNCH_OK;
}

int k_symmetrize(double *G, int ldg, int ell, hipStream_t s)
{
    symmetrize_k<<<(unsigned)((ell * ell + 255) / 256), 256, 0, s>>>(G, ldg, ell);
    return LAUNCH_OK;
}

int k_copy_f64(const double *src, double *dst, int64_t n, hipStream_t s)
{
    copy_f64_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, dst, n);
    return LAUNCH_OK;
}

int k_grid_residual(const double *G, int ldg, const double *rb, const double *bnorm2, int ell,
                    double *res2, hipStream_t s)
{
    if (ell < 1 || ell > 56) return NLRMM_ESHAPE;
    grid_residual_k<<<1, 64, 0, s>>>(G, ldg, rb, bnorm2, ell, res2);
    return LAUNCH_OK;
}

int k_grid_pick(const double *res2, int ncand, const double *shifts, double *theta, int64_t V,
                int *best, hipStream_t s)
{
    grid_pick_k<<<1, 256, 0, s>>>(res2, ncand, shifts, theta, V, best);
    return LAUNCH_OK;
}

int k_cg_coef(double *c, int mode, hipStream_t s)
{
    cg_coef_k<<<1, 64, 0, s>>>(c, mode);
    return LAUNCH_OK;
}

int k_offset_gn(const double *d1, const double *d2, const double *lamp, double *out,
                hipStream_t s)
{
    offset_gn_k<<<1, 64, 0, s>>>(d1, d2, lamp, out);
    return LAUNCH_OK;
}

int k_fill_f64(double *dst, int64_t n, double value, hipStream_t s)
{
    fill_f64_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dst, n, value);
    return LAUNCH_OK;
}

int k_offset_dir(const double *gh, double mu_rel, int64_t V, double *dir, double *sc,
                 hipStream_t s)
{
    offset_dir_k<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(gh, mu_rel, V, dir, sc);
    return LAUNCH_OK;
}

int k_lin_image(const float *u, const float *up, int64_t n, const double *alphas, int q,
                const double *dir, const int *accepted, float *out, hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    lin_image_k<<<(unsigned)blocks, 256, 0, s>>>(u, up, n, alphas, q, dir, accepted, out);
    return LAUNCH_OK;
}

int k_sens_objective(const double *rn2, int64_t V, const double *reg, const double *lamp,
                     const double *alphas, int q, double c1, double *sc, int *accepted,
                     hipStream_t s)
{
    sens_objective_k<<<1, BLK, 0, s>>>(rn2, V, reg, lamp, alphas, q, c1, sc, accepted);
    return LAUNCH_OK;
}

int k_fill_f32(float *dst, int64_t n, float value, hipStream_t s)
{
    if (n <= 0) return NLRMM_OK;
    fill_f32_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dst, n, value);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_fill_i32(int *dst, int64_t n, int value, hipStream_t s)
{
    fill_i32_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(dst, n, value);
    return LAUNCH_OK;
}

int k_scale_into(const float *src, const double *norm2, int64_t n, float *dst, double *norm_out,
                 int *status, hipStream_t s)
{
    scale_into_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, norm2, n, dst, norm_out, status);
    return LAUNCH_OK;
}

}  // namespace nlrmm
