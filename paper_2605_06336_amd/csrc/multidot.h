// Block-partial inner products over FP32 vectors with FP64 accumulation, shared by the
// Krylov kernels and the backprojection's split-sum launch (which can form the first
// reorthogonalisation products of the residual it writes).  Blocks of MD_BLK threads.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace nlrmm {
namespace md {

constexpr int MD_MAX = 72;    // inner products per launch
constexpr int MD_BLK = 256;   // threads per block

// sum over b = first, first + step, ... < count of p[b * stride], in that order, with U loads
// in flight at a time (a loop that waits for each load pays one memory latency per term).
// The loads are unconditional, their index clamped to the last term: a load under a branch
// is waited for before the branch closes.  Terms past count add +0.0, which changes no sum.
template <int U = 8>
__device__ __forceinline__ double strided_sum(const double *__restrict__ p, int64_t stride,
                                              int count, int first, int step)
{
    double s = 0.0;
    for (int b0 = first; b0 < count; b0 += U * step) {
        double v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = p[(int64_t)min(b0 + k * step, count - 1) * stride];
#pragma unroll
        for (int k = 0; k < U; ++k) s += b0 + k * step < count ? v[k] : 0.0;
    }
    return s;
}

// Inner products <X_i, y> (i < nv) and <z, y> (i == nv when z is given), FP64 accumulation:
// per-block partials part[block][i].  Each block reduces its share of the elements for
// groups of 16 outputs through LDS (16 threads per output, then a 16-lane butterfly).  Every
// thread of the block must call it; sacc: 16 x MD_BLK doubles of LDS; ends with a barrier.  With one element per
// thread the loads of CH outputs are issued together (all of them in multidot_k; fewer inside
// the Gram launch, whose own work needs few registers).
template <int CH>
__device__ __forceinline__ void multidot_body(const float *__restrict__ X, int64_t ldx, int nv,
                                              const float *__restrict__ y,
                                              const float *__restrict__ z, int64_t n,
                                              double *__restrict__ part, double (*sacc)[MD_BLK],
                                              int64_t bid, int64_t nbk)
{
    constexpr int GRP = 16;            // outputs reduced per LDS round
    const int tid = threadIdx.x;
    const int nout = nv + (z != nullptr ? 1 : 0);
    auto block_reduce = [&](int i0, const double (&acc)[GRP]) __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < GRP; ++a) sacc[a][tid] = acc[a];
        __syncthreads();
        constexpr int TPO = MD_BLK / GRP;            // threads per output of the group
        const int a = tid / TPO, l = tid % TPO;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < MD_BLK / TPO; ++k) s += sacc[a][l + TPO * k];
        for (int off = TPO / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, TPO);
        if (l == 0 && i0 + a < nout) part[bid * nout + i0 + a] = s;
        __syncthreads();
    };
    if (nbk * MD_BLK >= n) {
        // at most one element per thread: issue the loads of CH outputs first, then reduce
        // them by groups (the FP64 product of two floats is exact)
        static_assert(CH % GRP == 0 || CH == MD_MAX, "chunks of whole groups");
        const int64_t e = bid * MD_BLK + tid;
        const bool in = e < n;
        const float ye = in ? y[e] : 0.0f;
        for (int c0 = 0; c0 < nout; c0 += CH) {
            float xv[CH];
#pragma unroll
            for (int ii = 0; ii < CH; ++ii) {
                const int i = c0 + ii;
                float v = 0.0f;
                if (i < nv) v = in ? X[(int64_t)i * ldx + e] : 0.0f;
                else if (i == nv && z != nullptr) v = in ? z[e] : 0.0f;
                xv[ii] = v;
            }
#pragma unroll
            for (int g0 = 0; g0 < CH; g0 += GRP) {
                if (c0 + g0 < nout) {
                    double acc[GRP];
#pragma unroll
                    for (int a = 0; a < GRP; ++a)
                        acc[a] = g0 + a < CH ? (double)xv[g0 + a] * (double)ye : 0.0;
                    block_reduce(c0 + g0, acc);
                }
            }
        }
        return;
    }
    // several elements per thread: 16-byte loads when every column is 16-byte aligned and
    // n is a multiple of 4 (four times the bytes in flight per load)
    const bool vec4 = (ldx % 4) == 0 && (n % 4) == 0 &&
                      (reinterpret_cast<uintptr_t>(X) % 16) == 0 &&
                      (reinterpret_cast<uintptr_t>(y) % 16) == 0 &&
                      (z == nullptr || (reinterpret_cast<uintptr_t>(z) % 16) == 0);
    for (int i0 = 0; i0 < nout; i0 += GRP) {
        double acc[GRP];
#pragma unroll
        for (int a = 0; a < GRP; ++a) acc[a] = 0.0;
        if (vec4) {
            const int64_t n4 = n / 4, ld4 = ldx / 4;
            const float4 *X4 = reinterpret_cast<const float4 *>(X);
            const float4 *y4 = reinterpret_cast<const float4 *>(y);
            const float4 *z4 = reinterpret_cast<const float4 *>(z);
            for (int64_t e = bid * MD_BLK + tid; e < n4; e += nbk * MD_BLK) {
                const float4 yv = y4[e];
#pragma unroll
                for (int a = 0; a < GRP; ++a) {
                    const int i = i0 + a;
                    float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (i < nv) xv = X4[(int64_t)i * ld4 + e];
                    else if (i == nv && z != nullptr) xv = z4[e];
                    double t = acc[a];
                    t = fma((double)xv.x, (double)yv.x, t);
                    t = fma((double)xv.y, (double)yv.y, t);
                    t = fma((double)xv.z, (double)yv.z, t);
                    acc[a] = fma((double)xv.w, (double)yv.w, t);
                }
            }
        } else {
            for (int64_t e = bid * MD_BLK + tid; e < n; e += nbk * MD_BLK) {
                const double ye = (double)y[e];
#pragma unroll
                for (int a = 0; a < GRP; ++a) {
                    const int i = i0 + a;
                    if (i < nv) acc[a] = fma((double)X[(int64_t)i * ldx + e], ye, acc[a]);
                    else if (i == nv && z != nullptr) acc[a] = fma((double)z[e], ye, acc[a]);
                }
            }
        }
        block_reduce(i0, acc);
    }
}



}  // namespace md
}  // namespace nlrmm
