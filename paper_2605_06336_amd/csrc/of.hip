// Optical-flow temporal regulariser on gfx950 (Section 7, "Optical Flow Regularization",
// eqs. "of_forward" and "Theta_OF"; the OF branch of Alg. "dyn_nl_rmmgks").
//
// Velocity estimation (SOLVE-OF): for every frame pair t the velocity s = (s_x, s_y) from
// u(t) to u(t+1) minimising || Y s + u_t ||^2 + gamma || L s ||^2 + ridge || s ||^2, with
// Y = [diag(d_x u(t)), diag(d_y u(t))] (central differences, one-sided at the borders),
// u_t = u(t+1) - u(t) and L the forward differences of each component (none across the
// border): the l2/l2 (Horn-Schunck) form of eq. "of_forward", its gamma fixed and a small ridge
// keeping the normal equations definite where the image is flat.  Solved by `iters`
// conjugate-gradient steps on the normal equations from s = 0, every pair in the same launches
// (FP32 vectors, FP64 inner products; the per-pair scalars re-summed from block partials by
// each consumer in a fixed order, so no launch writes a scalar another block reads).
//
// Motion rows' gradient term: r += lam * M_hat^T (w * M_hat u) with M_hat the forward rows
// u(t) - M(s) u(t+1) and the reverse rows u(t+1) - M(-s) u(t) (tv.h).  The transpose of a
// bilinear warp scatters each row's weighted value to the four corners of its cell; the
// scatter accumulates in 64-bit fixed point (2^-36 units, integer atomics), so its result
// does not depend on the order of the atomics.
#include "internal.h"
#include "krylov.h"
#include "tv.h"

#include <math.h>

namespace nlrmm {
namespace {

constexpr int OF_BLK = 256;
constexpr int OF_EPT = 16;                      // vector elements per thread
constexpr int OF_EPB = OF_BLK * OF_EPT;         // per block
constexpr double OF_FIX = 68719476736.0;        // 2^36

int of_blocks(int64_t npix) { return (int)((2 * npix + OF_EPB - 1) / OF_EPB); }

__device__ __forceinline__ double of_wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of a pair's block partials, by the first wave in a fixed order; broadcast via LDS.
__device__ __forceinline__ double of_pair_sum(const double *__restrict__ part, int nblk)
{
    __shared__ double s_sum;
    if (threadIdx.x < 64) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 64) v += part[b];
        v = of_wave_sum(v);
        if (threadIdx.x == 0) s_sum = v;
    }
    __syncthreads();
    const double r = s_sum;
    __syncthreads();
    return r;
}

// Block sum of per-thread FP64 values, written to out[blockIdx.x] (fixed order).
__device__ __forceinline__ void of_block_partial(double v, double *__restrict__ out)
{
    __shared__ double s_w[OF_BLK / 64];
    v = of_wave_sum(v);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < OF_BLK / 64; ++i) t += s_w[i];
        out[blockIdx.x] = t;
    }
}

struct OfCG {
    int nx, ny, P, nblk;
    int64_t npix;
    float gamma, ridge;
    const float *u;
    float *x, *r, *p, *q, *gx, *gy;
    double *pq, *rr0, *rr1;   // [P][nblk] partials
};

// Central differences of frame u (one-sided at the borders) at pixel (k, l).
__device__ __forceinline__ void of_grad(const float *__restrict__ u, int nx, int ny, int k,
                                        int l, float &gx, float &gy)
{
    const int64_t i = (int64_t)l * nx + k;
    gx = k == 0 ? u[i + 1] - u[i] : (k == nx - 1 ? u[i] - u[i - 1] : 0.5f * (u[i + 1] - u[i - 1]));
    gy = l == 0 ? u[i + nx] - u[i]
                : (l == ny - 1 ? u[i] - u[i - nx] : 0.5f * (u[i + nx] - u[i - nx]));
}

// s = 0, r = p = -Y^T u_t, the image gradients; partials of r.r.
__global__ __launch_bounds__(OF_BLK) void of_prep_k(OfCG a)
{
    const int t = blockIdx.y;
    const int64_t n2 = 2 * a.npix;
    const float *u0 = a.u + (int64_t)t * a.npix, *u1 = u0 + a.npix;
    const int64_t vo = (int64_t)t * n2, po = (int64_t)t * a.npix;
    double acc = 0.0;
    for (int j = 0; j < OF_EPT; ++j) {
        const int64_t e = (int64_t)blockIdx.x * OF_EPB + j * OF_BLK + threadIdx.x;
        if (e >= n2) break;
        const int c = e >= a.npix;
        const int64_t pix = e - c * a.npix;
        const int l = (int)(pix / a.nx), k = (int)(pix - (int64_t)l * a.nx);
        float gx, gy;
        of_grad(u0, a.nx, a.ny, k, l, gx, gy);
        const float ut = u1[pix] - u0[pix];
        const float rhs = -(c ? gy : gx) * ut;
        a.x[vo + e] = 0.0f;
        a.r[vo + e] = rhs;
        a.p[vo + e] = rhs;
        if (!c) {
            a.gx[po + pix] = gx;
            a.gy[po + pix] = gy;
        }
        acc = fma((double)rhs, (double)rhs, acc);
    }
    of_block_partial(acc, a.rr0 + (int64_t)t * a.nblk);
}

// q = (Y^T Y + gamma L^T L + ridge I) p; partials of p.q.
__global__ __launch_bounds__(OF_BLK) void of_matvec_k(OfCG a)
{
    const int t = blockIdx.y;
    const int64_t n2 = 2 * a.npix;
    const int64_t vo = (int64_t)t * n2, po = (int64_t)t * a.npix;
    const float *pv = a.p + vo;
    double acc = 0.0;
    for (int j = 0; j < OF_EPT; ++j) {
        const int64_t e = (int64_t)blockIdx.x * OF_EPB + j * OF_BLK + threadIdx.x;
        if (e >= n2) break;
        const int c = e >= a.npix;
        const int64_t pix = e - c * a.npix;
        const int l = (int)(pix / a.nx), k = (int)(pix - (int64_t)l * a.nx);
        const float gx = a.gx[po + pix], gy = a.gy[po + pix];
        const float dot = fmaf(gx, pv[pix], gy * pv[a.npix + pix]);
        const float *pc = pv + c * a.npix;
        const float pe = pc[pix];
        float lap = 0.0f;   // (L^T L p_c) at the pixel: differences with existing neighbours
        if (k > 0) lap += pe - pc[pix - 1];
        if (k < a.nx - 1) lap += pe - pc[pix + 1];
        if (l > 0) lap += pe - pc[pix - a.nx];
        if (l < a.ny - 1) lap += pe - pc[pix + a.nx];
        const float qe = fmaf((c ? gy : gx), dot, fmaf(a.gamma, lap, a.ridge * pe));
        a.q[vo + e] = qe;
        acc = fma((double)pe, (double)qe, acc);
    }
    of_block_partial(acc, a.pq + (int64_t)t * a.nblk);
}

// alpha = r.r / p.q; s += alpha p; r -= alpha q; partials of the new r.r into rr_out.
__global__ __launch_bounds__(OF_BLK) void of_update_k(OfCG a, const double *__restrict__ rr_in,
                                                      double *__restrict__ rr_out)
{
    const int t = blockIdx.y;
    const double rr = of_pair_sum(rr_in + (int64_t)t * a.nblk, a.nblk);
    const double pq = of_pair_sum(a.pq + (int64_t)t * a.nblk, a.nblk);
    const float alpha = pq > 0.0 ? (float)(rr / pq) : 0.0f;
    const int64_t n2 = 2 * a.npix, vo = (int64_t)t * n2;
    double acc = 0.0;
    for (int j = 0; j < OF_EPT; ++j) {
        const int64_t e = (int64_t)blockIdx.x * OF_EPB + j * OF_BLK + threadIdx.x;
        if (e >= n2) break;
        a.x[vo + e] = fmaf(alpha, a.p[vo + e], a.x[vo + e]);
        const float re = fmaf(-alpha, a.q[vo + e], a.r[vo + e]);
        a.r[vo + e] = re;
        acc = fma((double)re, (double)re, acc);
    }
    of_block_partial(acc, rr_out + (int64_t)t * a.nblk);
}

// beta = r.r (new) / r.r (old); p = r + beta p.
__global__ __launch_bounds__(OF_BLK) void of_dir_k(OfCG a, const double *__restrict__ rr_old,
                                                   const double *__restrict__ rr_new)
{
    const int t = blockIdx.y;
    const double ro = of_pair_sum(rr_old + (int64_t)t * a.nblk, a.nblk);
    const double rn = of_pair_sum(rr_new + (int64_t)t * a.nblk, a.nblk);
    const float beta = ro > 0.0 ? (float)(rn / ro) : 0.0f;
    const int64_t n2 = 2 * a.npix, vo = (int64_t)t * n2;
    for (int j = 0; j < OF_EPT; ++j) {
        const int64_t e = (int64_t)blockIdx.x * OF_EPB + j * OF_BLK + threadIdx.x;
        if (e >= n2) break;
        a.p[vo + e] = fmaf(beta, a.p[vo + e], a.r[vo + e]);
    }
}

__global__ void of_fill_i64_k(long long *__restrict__ a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

__device__ __forceinline__ void of_fix_add(long long *a, float v)
{
    const long long q = llrint((double)v * OF_FIX);
    atomicAdd(reinterpret_cast<unsigned long long *>(a), (unsigned long long)q);
}

// One lane per (pair, pixel): the forward and reverse rows of the pixel, weighted, scattered
// to their diagonal pixel and to the four corners of their cells.
__global__ void of_scatter_k(const float *__restrict__ u, const float *__restrict__ w,
                             const float *__restrict__ flow, int nx, int ny, int F,
                             int64_t t_off, float e2, long long *__restrict__ acc)
{
    const int64_t npix = (int64_t)nx * ny;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * (F - 1)) return;
    const int64_t t = i / npix, p = i - t * npix;
    const int l = (int)(p / nx), k = (int)(p - (int64_t)l * nx);
    const float *sx = flow + 2 * t * npix, *sy = sx + npix;
    const float *u0 = u + t * npix, *u1 = u0 + npix;
    long long *a0 = acc + t * npix, *a1 = a0 + npix;
    {   // forward row u(t) - M(s) u(t+1)
        const OfCell c = of_cell(sx[p], sy[p], k, l, nx, ny);
        const float d = u0[p] - of_sample(u1, c, nx);
        const float z = (w ? w[t_off + t * npix + p] : tv_weight(d, e2)) * d;
        of_fix_add(a0 + p, z);
        of_fix_add(a1 + c.base, -c.w00 * z);
        of_fix_add(a1 + c.base + 1, -c.w10 * z);
        of_fix_add(a1 + c.base + nx, -c.w01 * z);
        of_fix_add(a1 + c.base + nx + 1, -c.w11 * z);
    }
    {   // reverse row u(t+1) - M(-s) u(t)
        const OfCell c = of_cell(-sx[p], -sy[p], k, l, nx, ny);
        const float d = u1[p] - of_sample(u0, c, nx);
        const float z = (w ? w[t_off + (F - 1 + t) * npix + p] : tv_weight(d, e2)) * d;
        of_fix_add(a1 + p, z);
        of_fix_add(a0 + c.base, -c.w00 * z);
        of_fix_add(a0 + c.base + 1, -c.w10 * z);
        of_fix_add(a0 + c.base + nx, -c.w01 * z);
        of_fix_add(a0 + c.base + nx + 1, -c.w11 * z);
    }
}

__global__ void of_finish_k(const long long *__restrict__ acc, const double *__restrict__ lamp,
                            float *__restrict__ r, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    r[i] += (float)lamp[0] * (float)((double)acc[i] * (1.0 / OF_FIX));
}

}  // namespace

size_t of_work_floats(int nx, int ny, int F)
{
    const int64_t npix = (int64_t)nx * ny;
    return F > 1 ? (size_t)(8 * (int64_t)(F - 1) * npix) : 0;
}

size_t of_part_doubles(int nx, int ny, int F)
{
    return F > 1 ? (size_t)3 * (size_t)(F - 1) * (size_t)of_blocks((int64_t)nx * ny) : 0;
}

int k_of_estimate(const float *u, int nx, int ny, int F, float gamma, float ridge, int iters,
                  float *flow, float *work, double *part, hipStream_t s)
{
    if (F < 2) return NLRMM_OK;
    if (nx < 2 || ny < 2 || iters < 0 || (F - 1) > 65535) return NLRMM_ESHAPE;
    OfCG a;
    a.nx = nx;
    a.ny = ny;
    a.P = F - 1;
    a.npix = (int64_t)nx * ny;
    a.nblk = of_blocks(a.npix);
    a.gamma = gamma;
    a.ridge = ridge;
    a.u = u;
    a.x = flow;
    const int64_t vec = 2 * (int64_t)a.P * a.npix;
    a.r = work;
    a.p = work + vec;
    a.q = work + 2 * vec;
    a.gx = work + 3 * vec;
    a.gy = a.gx + (int64_t)a.P * a.npix;
    const int64_t np = (int64_t)a.P * a.nblk;
    a.pq = part;
    a.rr0 = part + np;
    a.rr1 = part + 2 * np;
    const dim3 grid((unsigned)a.nblk, (unsigned)a.P);
    of_prep_k<<<grid, OF_BLK, 0, s>>>(a);
    for (int it = 0; it < iters; ++it) {
        double *rin = (it & 1) ? a.rr1 : a.rr0, *rout = (it & 1) ? a.rr0 : a.rr1;
        of_matvec_k<<<grid, OF_BLK, 0, s>>>(a);
        of_update_k<<<grid, OF_BLK, 0, s>>>(a, rin, rout);
        if (it + 1 < iters) of_dir_k<<<grid, OF_BLK, 0, s>>>(a, rin, rout);
    }
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_of_grad_add(const float *u, const float *w, const float *flow, int nx, int ny, int F,
                  const double *lamp, float *r, long long *acc, hipStream_t s, float eps)
{
    if (F < 2) return NLRMM_OK;
    if (nx < 2 || ny < 2 || flow == nullptr) return NLRMM_EINVAL;
    const int64_t npix = (int64_t)nx * ny;
    const int64_t n = npix * F;
    const int64_t per_frame = (int64_t)ny * (nx - 1) + (int64_t)(ny - 1) * nx;
    of_fill_i64_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(acc, n);
    const int64_t rows = npix * (F - 1);
    of_scatter_k<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(u, w, flow, nx, ny, F,
                                                              (int64_t)F * per_frame, eps * eps,
                                                              acc);
    of_finish_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(acc, lamp, r, n);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

}  // namespace nlrmm
