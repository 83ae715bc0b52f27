// Anisotropic TV operator Psi = [D_x; D_y] per frame (forward differences, (n-1) per line,
// unscaled) plus, for dynamic problems, the frame difference D_t (Section 2 regulariser and
// the dynamic ANISO-TV operator of Section 6.4): index layout of Psi u and the gradient
// term (Psi^T (w * Psi u))_pixel shared by the Krylov kernels and the backprojection
// epilogue.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nlrmm {

struct TVGeo {
    int nx, ny, F, temporal;
    int64_t per_frame;   // ny (nx-1) + (ny-1) nx
    int64_t dy_off;      // ny (nx-1)
    int64_t t_off;       // F * per_frame
};

__device__ __forceinline__ TVGeo tvgeo(int nx, int ny, int F, int temporal)
{
    TVGeo g;
    g.nx = nx;
    g.ny = ny;
    g.F = F;
    g.temporal = temporal && F > 1;
    g.dy_off = (int64_t)ny * (nx - 1);
    g.per_frame = g.dy_off + (int64_t)(ny - 1) * nx;
    g.t_off = (int64_t)F * g.per_frame;
    return g;
}

// MM weight of one difference d of Psi u: ((d)^2 + eps^2)^(-1/2) (Section 3.1), FP32.
__device__ __forceinline__ float tv_weight(float d, float e2) { return 1.0f / sqrtf(d * d + e2); }

// (Psi^T (w * Psi u))_i for pixel i of the stacked frames; with w == nullptr the weights
// are formed from u itself (tv_weight with e2 = eps^2), equal to the stored ones.
__device__ __forceinline__ float tv_grad_at(const float *__restrict__ u,
                                            const float *__restrict__ w, const TVGeo &g,
                                            int64_t i, float e2 = 0.0f)
{
    const int64_t npix = (int64_t)g.nx * g.ny;
    const int nx = g.nx, ny = g.ny;
    const int64_t f = i / npix, p = i - f * npix;
    const int l = (int)(p / nx), k = (int)(p - (int64_t)l * nx);
    const float uc = u[i];
    float acc = 0.0f;
    if (w == nullptr) {
        float d;
        if (k < nx - 1) {
            d = u[i + 1] - uc;
            acc -= tv_weight(d, e2) * d;
        }
        if (k > 0) {
            d = uc - u[i - 1];
            acc += tv_weight(d, e2) * d;
        }
        if (l < ny - 1) {
            d = u[i + nx] - uc;
            acc -= tv_weight(d, e2) * d;
        }
        if (l > 0) {
            d = uc - u[i - nx];
            acc += tv_weight(d, e2) * d;
        }
        if (g.temporal) {
            if (f < g.F - 1) {
                d = u[i + npix] - uc;
                acc -= tv_weight(d, e2) * d;
            }
            if (f > 0) {
                d = uc - u[i - npix];
                acc += tv_weight(d, e2) * d;
            }
        }
        return acc;
    }
    const float *wf = w + f * g.per_frame;
    if (k < nx - 1) acc -= wf[(int64_t)l * (nx - 1) + k] * (u[i + 1] - uc);
    if (k > 0) acc += wf[(int64_t)l * (nx - 1) + k - 1] * (uc - u[i - 1]);
    if (l < ny - 1) acc -= wf[g.dy_off + (int64_t)l * nx + k] * (u[i + nx] - uc);
    if (l > 0) acc += wf[g.dy_off + (int64_t)(l - 1) * nx + k] * (uc - u[i - nx]);
    if (g.temporal) {
        if (f < g.F - 1) acc -= w[g.t_off + f * npix + p] * (u[i + npix] - uc);
        if (f > 0) acc += w[g.t_off + (f - 1) * npix + p] * (uc - u[i - npix]);
    }
    return acc;
}

}  // namespace nlrmm
