// Variable-projection angle update (Section 4.2, eq. "GN_system"; supplementary Alg.
// "update_varpro") in the recycled subspace span(V), V with k columns.
//
// At angles theta:  A_hat = A(theta) V,  M = A_hat^T A_hat + lam B^T B  (B = P Psi V),
//   y = M^-1 A_hat^T b,  r = A_hat y - b,  f = 1/2 ||r||^2 + lam/2 ||B y||^2.
// With E_c = dA/dtheta v_c (view v's block E_{c,v}) and e_v = sum_c y_c E_{c,v}:
//   g_v = <e_v, r_v>                        (envelope: the y-derivative terms cancel)
//   Y[:, v] = -M^-1 (E_v^T r_v + A_hat_v^T e_v)
//   J = diag(||e_v||^2) + C Y + (C Y)^T + Y^T M Y + mu I,  C[v, :] = e_v^T A_hat_v.
// J is diagonal plus rank 2k: J = Lam + Z G Z^T with Z = [C, Y^T] and
// G = [[0, I], [I, M]], so d = -J^-1 g follows from the Woodbury identity with a 2k x 2k
// solve (G^-1 = [[-M, I], [I, 0]]).  Armijo trials re-project V at theta + alpha d and
// recompute y from the k x k Grams; a device flag skips the remaining trials.
#include "internal.h"
#include "krylov.h"

#include <math.h>

namespace nlrmm {
namespace {

constexpr int BLK = 256;
constexpr int KV = 16;   // max columns of the VarPro basis

__device__ double bsum(double v, double *sbuf)
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

// out[c][v] = sum_j X[c][v*nb + j] * e[v*nb + j]  (one block per view)
__global__ __launch_bounds__(BLK) void view_dots_k(const float *__restrict__ X, int64_t ldx, int k,
                                                   const float *__restrict__ e, int nb, int64_t V,
                                                   double *__restrict__ out)
{
    __shared__ double sbuf[BLK / 64];
    const int64_t v = blockIdx.x;
    for (int c = 0; c < k; ++c) {
        double s = 0.0;
        for (int j = threadIdx.x; j < nb; j += BLK)
            s += (double)X[(int64_t)c * ldx + v * nb + j] * (double)e[v * nb + j];
        s = bsum(s, sbuf);
        if (threadIdx.x == 0) out[(int64_t)c * V + v] = s;
    }
}

// In-place Cholesky of a k x k SPD matrix (single thread, k <= KV); returns 0 if not SPD.
__device__ int chol_small(double *A, int k)
{
    for (int j = 0; j < k; ++j) {
        double d = A[j * KV + j];
        for (int m = 0; m < j; ++m) d -= A[j * KV + m] * A[j * KV + m];
        if (!(d > 0.0)) return 0;
        d = sqrt(d);
        A[j * KV + j] = d;
        for (int i = j + 1; i < k; ++i) {
            double s = A[i * KV + j];
            for (int m = 0; m < j; ++m) s -= A[i * KV + m] * A[j * KV + m];
            A[i * KV + j] = s / d;
        }
    }
    return 1;
}

__device__ void chol_solve_small(const double *L, int k, double *x)
{
    for (int i = 0; i < k; ++i) {
        double s = x[i];
        for (int m = 0; m < i; ++m) s -= L[i * KV + m] * x[m];
        x[i] = s / L[i * KV + i];
    }
    for (int i = k - 1; i >= 0; --i) {
        double s = x[i];
        for (int m = i + 1; m < k; ++m) s -= L[m * KV + i] * x[m];
        x[i] = s / L[i * KV + i];
    }
}

// Reduced solve from the Grams: M = GA + lam GP, y = M^-1 ab,
// f = 1/2 (y^T GA y - 2 y^T ab + ||b||^2) + lam/2 y^T GP y.
// sc layout: [0] f0 (written when `first`), [1] g^T d, [2] accepted alpha, [3] mu,
// [4] f at the accepted alpha; y written to yout when `first`.  When `trial` >= 0 the
// result is an Armijo trial with alpha = alphas[trial].
__global__ void varpro_reduced_k(const double *__restrict__ GA, int ldg,
                                 const double *__restrict__ GP, const double *__restrict__ ab,
                                 const double *__restrict__ lamp, const double *__restrict__ bn2,
                                 int k, double *__restrict__ yout, double *__restrict__ Mout,
                                 double *__restrict__ sc, const double *__restrict__ alphas,
                                 int trial, double c1, int *accepted, int *status)
{
    if (threadIdx.x != 0) return;
    if (trial >= 0 && *accepted) return;
    const double lam = lamp[0];
    double M[KV * KV], L[KV * KV], y[KV];
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            M[i * KV + j] = GA[i * ldg + j] + lam * GP[i * ldg + j];
            L[i * KV + j] = M[i * KV + j];
        }
    for (int i = 0; i < k; ++i) y[i] = ab[i];
    if (!chol_small(L, k)) {
        atomicOr(status, NLRMM_ST_NONFINITE);
        if (trial < 0) {
            *accepted = 1;   // nothing to do: keep theta
            sc[2] = 0.0;
        }
        return;
    }
    chol_solve_small(L, k, y);
    double yAy = 0.0, yab = 0.0, yPy = 0.0;
    for (int i = 0; i < k; ++i) {
        yab += y[i] * ab[i];
        for (int j = 0; j < k; ++j) {
            yAy += y[i] * GA[i * ldg + j] * y[j];
            yPy += y[i] * GP[i * ldg + j] * y[j];
        }
    }
    const double f = 0.5 * (yAy - 2.0 * yab + bn2[0]) + 0.5 * lam * yPy;
    if (trial < 0) {
        sc[0] = f;
        for (int i = 0; i < k; ++i) yout[i] = y[i];
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) Mout[i * KV + j] = M[i * KV + j];
        *accepted = 0;
    } else {
        const double a = alphas[trial];
        if (f <= sc[0] + c1 * a * sc[1]) {
            *accepted = 1;
            sc[2] = a;
            sc[4] = f;
        }
    }
}

// Gauss-Newton direction by Woodbury.  Inputs per view: gd[v] = <e_v, r_v>,
// en2[v] = ||e_v||^2, ETr[c][v] = <E_{c,v}, r_v>, Ate[c][v] = <A_hat_{c,v}, e_v>.
__global__ __launch_bounds__(BLK) void varpro_dir_k(const double *__restrict__ Mg, int k,
                                                    const double *__restrict__ gd,
                                                    const double *__restrict__ en2,
                                                    const double *__restrict__ ETr,
                                                    const double *__restrict__ Ate, int64_t V,
                                                    double mu_rel, double *__restrict__ Yw,
                                                    double *__restrict__ dir,
                                                    double *__restrict__ sc, int *status)
{
    __shared__ double sL[KV * KV];
    __shared__ double sM[KV * KV];
    __shared__ double sbuf[BLK / 64];
    __shared__ double sS[2 * KV][2 * KV + 1];
    __shared__ double st[2 * KV];
    __shared__ double smu;
    const int tid = threadIdx.x;
    const int k2 = 2 * k;
    if (tid == 0) {
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                sM[i * KV + j] = Mg[i * KV + j];
                sL[i * KV + j] = Mg[i * KV + j];
            }
        if (!chol_small(sL, k)) atomicOr(status, NLRMM_ST_NONFINITE);
    }
    __syncthreads();
    // Y[:, v] = -M^-1 (ETr[:, v] + Ate[:, v]); diag(J)_v
    double dsum = 0.0;
    for (int64_t v = tid; v < V; v += BLK) {
        double x[KV];
        for (int c = 0; c < k; ++c) x[c] = ETr[c * V + v] + Ate[c * V + v];
        chol_solve_small(sL, k, x);
        double cy = 0.0, ymy = 0.0;
        for (int c = 0; c < k; ++c) {
            const double yc = -x[c];
            Yw[c * V + v] = yc;
            cy += Ate[c * V + v] * yc;
        }
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) ymy += Yw[i * V + v] * sM[i * KV + j] * Yw[j * V + v];
        dsum += en2[v] + 2.0 * cy + ymy;
    }
    dsum = bsum(dsum, sbuf);
    if (tid == 0) smu = mu_rel * dsum / (double)V;
    __syncthreads();
    const double mu = smu;
    // S = G^-1 + Z^T Lam^-1 Z and t = Z^T Lam^-1 g, Z[v] = [Ate[:, v], Y[:, v]]
    for (int a = 0; a < k2; ++a) {
        for (int b2 = a; b2 < k2; ++b2) {
            double s = 0.0;
            for (int64_t v = tid; v < V; v += BLK) {
                const double za = a < k ? Ate[a * V + v] : Yw[(a - k) * V + v];
                const double zb = b2 < k ? Ate[b2 * V + v] : Yw[(b2 - k) * V + v];
                s += za * zb / (en2[v] + mu);
            }
            s = bsum(s, sbuf);
            if (tid == 0) {
                double gi = 0.0;   // G^-1 = [[-M, I], [I, 0]]
                if (a < k && b2 < k) gi = -sM[a * KV + b2];
                else if (a < k && b2 >= k && b2 - k == a) gi = 1.0;
                sS[a][b2] = s + gi;
                sS[b2][a] = s + gi;
            }
        }
        double t = 0.0;
        for (int64_t v = tid; v < V; v += BLK) {
            const double za = a < k ? Ate[a * V + v] : Yw[(a - k) * V + v];
            t += za * gd[v] / (en2[v] + mu);
        }
        t = bsum(t, sbuf);
        if (tid == 0) st[a] = t;
    }
    __syncthreads();
    if (tid == 0) {
        // Gaussian elimination with partial pivoting: S s = t (S symmetric, indefinite)
        for (int c = 0; c < k2; ++c) {
            int p = c;
            for (int r = c + 1; r < k2; ++r)
                if (fabs(sS[r][c]) > fabs(sS[p][c])) p = r;
            if (p != c) {
                for (int j = 0; j < k2; ++j) {
                    const double tmp = sS[c][j];
                    sS[c][j] = sS[p][j];
                    sS[p][j] = tmp;
                }
                const double tmp = st[c];
                st[c] = st[p];
                st[p] = tmp;
            }
            const double piv = sS[c][c];
            if (piv == 0.0) {
                atomicOr(status, NLRMM_ST_NONFINITE);
                continue;
            }
            for (int r = c + 1; r < k2; ++r) {
                const double f = sS[r][c] / piv;
                for (int j = c; j < k2; ++j) sS[r][j] -= f * sS[c][j];
                st[r] -= f * st[c];
            }
        }
        for (int c = k2 - 1; c >= 0; --c) {
            double s = st[c];
            for (int j = c + 1; j < k2; ++j) s -= sS[c][j] * st[j];
            st[c] = sS[c][c] != 0.0 ? s / sS[c][c] : 0.0;
        }
    }
    __syncthreads();
    // d = -Lam^-1 (g - Z s)
    double gdd = 0.0;
    for (int64_t v = tid; v < V; v += BLK) {
        double zs = 0.0;
        for (int a = 0; a < k2; ++a) {
            const double za = a < k ? Ate[a * V + v] : Yw[(a - k) * V + v];
            zs += za * st[a];
        }
        const double d = -(gd[v] - zs) / (en2[v] + mu);
        dir[v] = d;
        gdd += gd[v] * d;
    }
    gdd = bsum(gdd, sbuf);
    if (tid == 0) {
        sc[1] = gdd;
        sc[3] = mu;
    }
}

}  // namespace

#define LAUNCH_OK (hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP)

int k_view_dots(const float *X, int64_t ldx, int k, const float *e, int nb, int64_t V, double *out,
                hipStream_t s)
{
    view_dots_k<<<(unsigned)V, BLK, 0, s>>>(X, ldx, k, e, nb, V, out);
    return LAUNCH_OK;
}

int k_varpro_reduced(const double *GA, int ldg, const double *GP, const double *ab,
                     const double *lamp, const double *bn2, int k, double *yout, double *Mout,
                     double *sc, const double *alphas, int trial, double c1, int *accepted,
                     int *status, hipStream_t s)
{
    if (k < 1 || k > KV) return NLRMM_ESHAPE;
    varpro_reduced_k<<<1, 64, 0, s>>>(GA, ldg, GP, ab, lamp, bn2, k, yout, Mout, sc, alphas, trial,
                                      c1, accepted, status);
    return LAUNCH_OK;
}

int k_varpro_dir(const double *M, int k, const double *gd, const double *en2, const double *ETr,
                 const double *Ate, int64_t V, double mu_rel, double *Yw, double *dir, double *sc,
                 int *status, hipStream_t s)
{
    if (k < 1 || k > KV) return NLRMM_ESHAPE;
    varpro_dir_k<<<1, BLK, 0, s>>>(M, k, gd, en2, ETr, Ate, V, mu_rel, Yw, dir, sc, status);
    return LAUNCH_OK;
}

}  // namespace nlrmm
