// Anisotropic TV operator Psi = [D_x; D_y] per frame (forward differences, (n-1) per line,
// unscaled) plus, for dynamic problems, temporal rows (Section 2 regulariser and the dynamic
// operators of Section 7): mode 1, the frame difference D_t of ANISO-TV (operator D1); mode 2,
// the optical-flow motion rows of Theta (eq. "Theta_OF"): for every frame pair t the forward
// consistency u(t) - M(s(t)) u(t+1), then for every pair the reverse consistency
// u(t+1) - M(-s(t)) u(t), M(s) the bilinear warp sampling at (k + s_x, l + s_y) clamped to the
// grid.  Index layout of Psi u and the gradient term (Psi^T (w * Psi u))_pixel shared by the
// Krylov kernels and the backprojection epilogue (the motion rows' transpose is a scatter,
// added by its own kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nlrmm {

constexpr int TEMPORAL_NONE = 0, TEMPORAL_DIFF = 1, TEMPORAL_OF = 2;

struct TVGeo {
    int nx, ny, F, temporal;   // temporal: TEMPORAL_* (NONE when F == 1)
    int64_t per_frame;   // ny (nx-1) + (ny-1) nx
    int64_t dy_off;      // ny (nx-1)
    int64_t t_off;       // F * per_frame
    const float *flow;   // TEMPORAL_OF: velocities [F-1][2][ny][nx] (s_x then s_y per pair)
};

__device__ __forceinline__ TVGeo tvgeo(int nx, int ny, int F, int temporal,
                                       const float *flow = nullptr)
{
    TVGeo g;
    g.nx = nx;
    g.ny = ny;
    g.F = F;
    g.temporal = F > 1 ? temporal : TEMPORAL_NONE;
    g.dy_off = (int64_t)ny * (nx - 1);
    g.per_frame = g.dy_off + (int64_t)(ny - 1) * nx;
    g.t_off = (int64_t)F * g.per_frame;
    g.flow = flow;
    return g;
}

// Bilinear cell of the warp sample at (k + sx, l + sy), clamped to [0, nx-1] x [0, ny-1]:
// the corner (k0, l0) = the floor, kept at most (nx-2, ny-2) (nx, ny >= 2), and the four
// corner weights.  A NaN velocity samples the clamped corner (fmaxf / fminf return the number).
struct OfCell {
    int64_t base;   // l0 * nx + k0 within the frame
    float w00, w10, w01, w11;
};

__device__ __forceinline__ OfCell of_cell(float sx, float sy, int k, int l, int nx, int ny)
{
    const float px = fminf(fmaxf((float)k + sx, 0.0f), (float)(nx - 1));
    const float py = fminf(fmaxf((float)l + sy, 0.0f), (float)(ny - 1));
    const int k0 = min((int)floorf(px), nx - 2), l0 = min((int)floorf(py), ny - 2);
    const float fx = px - (float)k0, fy = py - (float)l0;
    OfCell c;
    c.base = (int64_t)l0 * nx + k0;
    c.w00 = (1.0f - fx) * (1.0f - fy);
    c.w10 = fx * (1.0f - fy);
    c.w01 = (1.0f - fx) * fy;
    c.w11 = fx * fy;
    return c;
}

// The warped frame v (one frame's pixels) at a cell.
__device__ __forceinline__ float of_sample(const float *__restrict__ v, const OfCell &c, int nx)
{
    const float *q = v + c.base;
    return fmaf(c.w11, q[nx + 1], fmaf(c.w01, q[nx], fmaf(c.w10, q[1], c.w00 * q[0])));
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
        if (g.temporal == TEMPORAL_DIFF) {
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
    // the loads are unconditional, at indices that always exist (a missing neighbour reads
    // the pixel itself, a missing weight the frame's first entry), and the missing terms are
    // dropped afterwards: a load under a per-lane branch is waited for before the branch
    // closes, one memory latency per term
    const float *wf = w + f * g.per_frame;
    const bool xp = k < nx - 1, xm = k > 0, yp = l < ny - 1, ym = l > 0;
    const float uxp = u[i + (xp ? 1 : 0)], uxm = u[i - (xm ? 1 : 0)];
    const float uyp = u[i + (yp ? nx : 0)], uym = u[i - (ym ? nx : 0)];
    const float wxp = wf[xp ? (int64_t)l * (nx - 1) + k : 0];
    const float wxm = wf[xm ? (int64_t)l * (nx - 1) + k - 1 : 0];
    const float wyp = wf[yp ? g.dy_off + (int64_t)l * nx + k : 0];
    const float wym = wf[ym ? g.dy_off + (int64_t)(l - 1) * nx + k : 0];
    if (xp) acc -= wxp * (uxp - uc);
    if (xm) acc += wxm * (uc - uxm);
    if (yp) acc -= wyp * (uyp - uc);
    if (ym) acc += wym * (uc - uym);
    if (g.temporal == TEMPORAL_DIFF) {
        const bool tp = f < g.F - 1, tm = f > 0;
        const float utp = u[i + (tp ? npix : 0)], utm = u[i - (tm ? npix : 0)];
        const float wtp = w[tp ? g.t_off + f * npix + p : 0];
        const float wtm = w[tm ? g.t_off + (f - 1) * npix + p : 0];
        if (tp) acc -= wtp * (utp - uc);
        if (tm) acc += wtm * (uc - utm);
    }
    return acc;
}

}  // namespace nlrmm
