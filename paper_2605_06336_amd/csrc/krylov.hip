// Krylov-side kernels of MM-GKS / RMM-GKS on gfx950 (Section 3 and supplementary
// Algorithms "mmgks", "enlarge", "compress"):
//   * anisotropic TV regulariser Psi (Section 2.2), MM weights w = ((Psi u)^2 + eps^2)^(-1/2)
//     (Section 3.1) and the regulariser part lam Psi^T (w * Psi u) of the GKS residual;
//   * FP64-accumulated Gram matrices and multi-dot products over FP32 basis blocks;
//   * basis GEMV / block updates (u = V z, r -= V h, V <- V T);
//   * a single-workgroup FP64 solver of the projected problem with lambda chosen by the
//     discrepancy principle, and the eigen-decomposition used by the recycling compression.
// Everything that decides (lambda, breakdown, compression size) is decided on the device.
#include "internal.h"
#include "krylov.h"
#include "multidot.h"
#include "solve_reg_launch.h"
#include "tv.h"
#include "wave.h"

#include <math.h>

#include <type_traits>

namespace nlrmm {
namespace {

constexpr int BLK = 256;
static_assert(BLK == md::MD_BLK, "one block shape for the shared multidot body");
constexpr int SOLVE_MAX = 56;
using wave::dpp_mov;
using wave::lane_bcast;
using wave::wave_sum;
using wave::wave_sum_dpp;
using md::MD_MAX;
using md::multidot_body;

constexpr int SOLVE_NT = 256;   // threads of the single-workgroup projected solves   // largest projected problem: two 56x57 FP64 matrices in LDS



// block-wide sum of a double (all threads receive the result)
__device__ double block_sum(double v, double *sbuf)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sbuf[wv] = v;
    __syncthreads();
    double t = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += sbuf[i];
    return t;
}

// ---------------------------------------------------------------------------
// regulariser
// ---------------------------------------------------------------------------
// w = ((Psi u)^2 + eps^2)^(-1/2), one thread per pixel writing its forward differences.
__global__ void psi_weights_k(const float *__restrict__ u, int nx, int ny, int F, int temporal,
                              float eps, float *__restrict__ w, const float *__restrict__ flow)
{
    const TVGeo g = tvgeo(nx, ny, F, temporal, flow);
    const int64_t npix = (int64_t)nx * ny;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * F) return;
    const int64_t f = i / npix, p = i - f * npix;
    const int l = (int)(p / nx), k = (int)(p - (int64_t)l * nx);
    const float uc = u[i];
    const float e2 = eps * eps;
    if (k < nx - 1) w[f * g.per_frame + (int64_t)l * (nx - 1) + k] = tv_weight(u[i + 1] - uc, e2);
    if (l < ny - 1)
        w[f * g.per_frame + g.dy_off + (int64_t)l * nx + k] = tv_weight(u[i + nx] - uc, e2);
    if (g.temporal == TEMPORAL_DIFF && f < F - 1)
        w[g.t_off + f * npix + p] = tv_weight(u[i + npix] - uc, e2);
    if (g.temporal == TEMPORAL_OF && f < F - 1) {
        const float *sx = flow + 2 * f * npix, *sy = sx + npix;
        const OfCell cf = of_cell(sx[p], sy[p], k, l, nx, ny);
        const OfCell cr = of_cell(-sx[p], -sy[p], k, l, nx, ny);
        w[g.t_off + f * npix + p] = tv_weight(uc - of_sample(u + (f + 1) * npix, cf, nx), e2);
        w[g.t_off + (F - 1 + f) * npix + p] =
            tv_weight(u[i + npix] - of_sample(u + f * npix, cr, nx), e2);
    }
}

// r += lam * Psi^T (w * Psi u)  (the regulariser part of the normal-equation residual).
__global__ void tv_grad_add_k(const float *__restrict__ u, const float *__restrict__ w, int nx,
                              int ny, int F, int temporal, const double *__restrict__ lamp,
                              float *__restrict__ r, float e2)
{
    const float lam = (float)lamp[0];
    const TVGeo g = tvgeo(nx, ny, F, temporal);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nx * ny * F) return;
    r[i] += lam * tv_grad_at(u, w, g, i, e2);
}

// Psi u written out (used by tests and by the VarPro regulariser block).
__global__ void psi_apply_k(const float *__restrict__ u, int nx, int ny, int F, int temporal,
                            float *__restrict__ s, const float *__restrict__ flow)
{
    const TVGeo g = tvgeo(nx, ny, F, temporal, flow);
    const int64_t npix = (int64_t)nx * ny;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * F) return;
    const int64_t f = i / npix, p = i - f * npix;
    const int l = (int)(p / nx), k = (int)(p - (int64_t)l * nx);
    const float uc = u[i];
    if (k < nx - 1) s[f * g.per_frame + (int64_t)l * (nx - 1) + k] = u[i + 1] - uc;
    if (l < ny - 1) s[f * g.per_frame + g.dy_off + (int64_t)l * nx + k] = u[i + nx] - uc;
    if (g.temporal == TEMPORAL_DIFF && f < F - 1) s[g.t_off + f * npix + p] = u[i + npix] - uc;
    if (g.temporal == TEMPORAL_OF && f < F - 1) {
        const float *sx = flow + 2 * f * npix, *sy = sx + npix;
        const OfCell cf = of_cell(sx[p], sy[p], k, l, nx, ny);
        const OfCell cr = of_cell(-sx[p], -sy[p], k, l, nx, ny);
        s[g.t_off + f * npix + p] = uc - of_sample(u + (f + 1) * npix, cf, nx);
        s[g.t_off + (F - 1 + f) * npix + p] = u[i + npix] - of_sample(u + f * npix, cr, nx);
    }
}

// Weighted regulariser Gram G[i][j] = sum_e w_e (Psi v_i)_e (Psi v_j)_e for the first ell
// columns of V (column stride ldv), Psi v computed on the fly from V.  Each block handles
// a strided set of 16-pixel chunks: the chunk's weighted difference rows (<= 48 x ell)
// are staged in LDS as FP64 and every thread accumulates a 4x4 tile of G in FP64.
constexpr int GP_PIX = 16;
constexpr int GP_ROWS = GP_PIX * 4;   // at most four rows per pixel (dx, dy, two motion rows)
constexpr int GMAX = 64;

// The j-th difference row (kind 0 dx, 1 dy, 2 dt or forward motion, 3 reverse motion) of
// pixel i for column vc, unweighted, 0 where the row does not exist.
__device__ __forceinline__ double psi_row(const float *__restrict__ vc, const TVGeo &g, int64_t i,
                                          int kind)
{
    const int64_t npix = (int64_t)g.nx * g.ny;
    const int64_t f = i / npix, p = i - f * npix;
    const int l = (int)(p / g.nx), k = (int)(p - (int64_t)l * g.nx);
    if (kind == 0) return k < g.nx - 1 ? (double)vc[i + 1] - (double)vc[i] : 0.0;
    if (kind == 1) return l < g.ny - 1 ? (double)vc[i + g.nx] - (double)vc[i] : 0.0;
    if (f >= g.F - 1) return 0.0;
    if (g.temporal == TEMPORAL_DIFF) return kind == 2 ? (double)vc[i + npix] - (double)vc[i] : 0.0;
    const float *sx = g.flow + 2 * f * npix, *sy = sx + npix;
    if (kind == 2) {
        const OfCell c = of_cell(sx[p], sy[p], k, l, g.nx, g.ny);
        return (double)vc[i] - (double)of_sample(vc + (f + 1) * npix, c, g.nx);
    }
    const OfCell c = of_cell(-sx[p], -sy[p], k, l, g.nx, g.ny);
    return (double)vc[i + npix] - (double)of_sample(vc + f * npix, c, g.nx);
}

// Index of the weight of that row in w.
__device__ __forceinline__ int64_t psi_row_weight(const TVGeo &g, int64_t i, int kind)
{
    const int64_t npix = (int64_t)g.nx * g.ny;
    const int64_t f = i / npix, p = i - f * npix;
    const int l = (int)(p / g.nx), k = (int)(p - (int64_t)l * g.nx);
    if (kind == 0) return f * g.per_frame + (int64_t)l * (g.nx - 1) + k;
    if (kind == 1) return f * g.per_frame + g.dy_off + (int64_t)l * g.nx + k;
    if (kind == 2) return g.t_off + f * npix + p;
    return g.t_off + (g.F - 1 + f) * npix + p;
}

__global__ __launch_bounds__(BLK) void gram_psi_k(const float *__restrict__ V, int64_t ldv, int ell,
                                                  const float *__restrict__ w, int nx, int ny,
                                                  int F, int temporal, double *__restrict__ part,
                                                  const float *__restrict__ flow)
{
    __shared__ double sB[GP_ROWS][GMAX + 1];
    const TVGeo g = tvgeo(nx, ny, F, temporal, flow);
    const int KIND = g.temporal == TEMPORAL_OF ? 4 : (g.temporal == TEMPORAL_DIFF ? 3 : 2);
    const int rows = GP_PIX * KIND;
    const int64_t npix = (int64_t)nx * ny;
    const int64_t ntot = npix * F;
    const int tid = threadIdx.x;
    const int ti = tid / 16, tj = tid % 16;    // 4x4 output tile (4 ti .. 4 ti + 3, 4 tj ..)
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    const int64_t nchunks = (ntot + GP_PIX - 1) / GP_PIX;
    const bool active = 4 * ti < ell && 4 * tj < ell;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        // stage rows: row r = KIND * pixel + kind
        for (int t = tid; t < rows * ell; t += BLK) {
            const int c = t / rows, r = t - c * rows;
            const int pc = r / KIND, kind = r - pc * KIND;
            const int64_t i = ch * GP_PIX + pc;
            double val = 0.0;
            if (i < ntot) {
                const double d = psi_row(V + (int64_t)c * ldv, g, i, kind);
                if (d != 0.0) val = sqrt((double)w[psi_row_weight(g, i, kind)]) * d;
            }
            sB[r][c] = val;
        }
        __syncthreads();
        if (active) {
            for (int r = 0; r < rows; ++r) {
                double ra[4], cb[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int ii = 4 * ti + a, jj = 4 * tj + a;
                    ra[a] = ii < ell ? sB[r][ii] : 0.0;
                    cb[a] = jj < ell ? sB[r][jj] : 0.0;
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = fma(ra[a], cb[b], acc[a][b]);
            }
        }
        __syncthreads();
    }
    double *out = part + (int64_t)blockIdx.x * ell * ell;
    if (active) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int ii = 4 * ti + a, jj = 4 * tj + b;
                if (ii < ell && jj < ell) out[ii * ell + jj] = acc[a][b];
            }
    }
}

// MFMA variant of the weighted regulariser Gram (B^T B with B = sqrt(w) * Psi V, B of
// up to 192 rows per 64-pixel chunk and <= 64 columns).  The chunk's rows are staged in
// LDS as FP32; each of the four waves owns one 32x32 tile of the (padded) 64x64 result and
// runs v_mfma_f32_32x32x2f32 (FP32 operands) or v_mfma_f32_32x32x8bf16_1k (BF16 operands,
// round-to-nearest-even) with FP32 accumulation over the chunk, flushed into FP64
// accumulators after every chunk.  Output layout of the 32x32 MFMA: element (i, j) lives in
// lane j + 32 ((i/4) mod 2), register (i mod 4) + 4 (i / 8).
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
constexpr int MP = 64;            // pixels per chunk (48 with the two motion rows)
constexpr int MRMAX = 3 * MP;     // rows per chunk (dx, dy and dt, or dx, dy and two motion rows)
constexpr int MLDR = MRMAX + 1;   // LDS column stride (floats, odd: conflict-free columns)
constexpr int MLDH = MRMAX + 4;   // BF16 column stride (shorts; 8-byte units odd)

__device__ __forceinline__ short bf16_rne(float f)
{
    unsigned u = __float_as_uint(f);
    const unsigned lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (short)(u >> 16);
}

// G_Psi = (sqrt(w) Psi V)^T (sqrt(w) Psi V) on the matrix cores.  A chunk of MP pixels gives
// KIND * MP rows (the weighted differences of every column, all dx rows of the chunk, then all
// dy rows, ...) staged column-major in LDS; each
// wave multiplies one 32 x 32 tile of the (at most 64 x 64) Gram over the chunk's rows with
// FP32 accumulation, flushed to FP64 per chunk.  Only tiles on or above the diagonal are
// formed: for ell <= 32 the four waves split the rows of the single tile, otherwise waves
// 0..2 take the tiles (0,0), (0,1), (1,1).  Per-block partials go to part[block][ell][ell]
// (both triangles).
template <bool BF16, bool MOTION>
__global__ __launch_bounds__(BLK, 3) void gram_psi_mfma_k(const float *__restrict__ V, int64_t ldv,
                                                       int ell, const float *__restrict__ w,
                                                       int nx, int ny, int F, int temporal,
                                                       double *__restrict__ part,
                                                       const float *__restrict__ u, float e2,
                                                       const float *__restrict__ flow,
                                                       float *__restrict__ wout,
                                                       GramColJob col)
{
    // the chunk's weighted differences, column-major: FP32, or BF16 rounded once at staging
    // (four consecutive rows of a column are then one 8-byte MFMA operand)
    using Elem = typename std::conditional<BF16, short, float>::type;
    constexpr int LD = BF16 ? MLDH : MLDR;
    // A pending data-Gram column is taken by the FP32 instances only: its registers would
    // halve the occupancy of the BF16 ones (whose LDS tile allows six waves per SIMD).
    constexpr bool COLJOB = !BF16;
    // staging area, also the reduction buffer of a pending data-Gram column (16 x BLK doubles)
    constexpr size_t SB_BYTES = sizeof(Elem) * 64 * LD;
    constexpr size_t CB = COLJOB ? 16 * BLK * sizeof(double) : 0;
    constexpr size_t RAW = SB_BYTES > CB ? SB_BYTES : CB;
    __shared__ __align__(16) unsigned char sraw[RAW];
    Elem(*sB)[LD] = reinterpret_cast<Elem(*)[LD]>(sraw);
    // a pending data-Gram column is taken by the launch's last col.cblk blocks (its inner
    // products need no part of this Gram, so they run beside the Gram's blocks)
    int64_t gbid = blockIdx.x, gnb = gridDim.x;
    if constexpr (COLJOB) {
        if (col.X != nullptr) {
            gnb -= col.cblk;
            if (gbid >= gnb) {
                multidot_body<32>(col.X, col.ldx, col.ell + 1, col.xnew, col.b, col.n, col.part,
                                  reinterpret_cast<double(*)[BLK]>(sraw), gbid - gnb, col.cblk);
                return;
            }
        }
    }
    const TVGeo g = tvgeo(nx, ny, F, temporal, flow);
    // MOTION: the launch has the optical-flow rows (temporal mode 2 with several frames)
    constexpr bool motion = MOTION;
    const int KIND = motion ? 4 : (g.temporal == TEMPORAL_DIFF ? 3 : 2);
    constexpr int mp = motion ? 48 : MP;   // pixels per chunk: KIND * mp <= MRMAX rows
    const int MR = KIND * mp;
    const int64_t npix = (int64_t)nx * ny;
    const int64_t ntot = npix * F;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int pc = lane, cg = wv;          // staging: pixel of the chunk, column group
    // padded columns stay zero
    for (int t = tid; t < 64 * LD; t += BLK) {
        const int c = t / LD;
        if (c >= ell) sB[c][t - c * LD] = Elem(0);
    }
    // this wave's tile and row slice
    const bool single = ell <= 32;
    const int ti = single ? 0 : (wv == 2 ? 1 : 0);
    const int tj = single ? 0 : (wv == 0 ? 0 : 1);
    const bool busy = single || wv < 3;
    const int nsl = single ? 4 : 1, sl = single ? wv : 0;
    double accd[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) accd[r] = 0.0;
    const int64_t nchunks = (ntot + mp - 1) / mp;
    for (int64_t ch = gbid; ch < nchunks; ch += gnb) {
        const int64_t i = ch * mp + pc;
        const bool stage = pc < mp;            // lanes beyond the chunk stage nothing
        float w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f;
        int64_t ox = -1, oy = -1, ot = -1;   // neighbour offsets of the existing differences
        OfCell cf{0, 0.f, 0.f, 0.f, 0.f}, cr{0, 0.f, 0.f, 0.f, 0.f};   // motion rows' cells
        int64_t fo = 0, ro = 0;              // their frames' first pixels (f + 1 and f)
        // Every load of the staging is unconditional, at an index that always exists (lanes
        // that stage nothing read element 0, a missing neighbour reads the pixel itself, a
        // missing weight entry reads entry 0), and the values are selected afterwards: a load
        // under a per-lane branch is waited for before the branch closes, which would put
        // one memory latency per column on the chain.
        const bool live = stage && i < ntot;
        const int64_t ib = live ? i : 0;
        const int64_t f = ib / npix, p = ib - f * npix;
        const int l = (int)(p / nx), k = (int)(p - (int64_t)l * nx);
        const bool hx = live && k < nx - 1, hy = live && l < ny - 1;
        const bool ht = live && g.temporal == TEMPORAL_DIFF && f < F - 1;
        const int64_t atx = hx ? f * g.per_frame + (int64_t)l * (nx - 1) + k : 0;
        const int64_t aty = hy ? f * g.per_frame + g.dy_off + (int64_t)l * nx + k : 0;
        const int64_t att = ht ? g.t_off + f * npix + p : 0;
        // weights stored in w, or formed from u (the same values) and then, when wout is
        // given, stored there by wave 0 (each weight belongs to one pixel of one chunk)
        float uc = 0.0f, wx, wy, wt;
        if (u != nullptr) {
            uc = u[ib];
            const float ux = u[ib + (hx ? 1 : 0)], uy = u[ib + (hy ? nx : 0)];
            const float ut = u[ib + (ht ? npix : 0)];
            wx = tv_weight(ux - uc, e2);
            wy = tv_weight(uy - uc, e2);
            wt = tv_weight(ut - uc, e2);
        } else {
            wx = w[atx];
            wy = w[aty];
            wt = w[att];
        }
        const bool put = wout != nullptr && u != nullptr && wv == 0;
        if (hx) {
            if (put) wout[atx] = wx;
            w0 = sqrtf(wx);
            ox = 1;
        }
        if (hy) {
            if (put) wout[aty] = wy;
            w1 = sqrtf(wy);
            oy = nx;
        }
        if (ht) {
            if (put) wout[att] = wt;
            w2 = sqrtf(wt);
            ot = npix;
        }
        if (live) {
            if (motion && f < F - 1) {
                const float *sx = flow + 2 * f * npix, *sy = sx + npix;
                cf = of_cell(sx[p], sy[p], k, l, nx, ny);
                cr = of_cell(-sx[p], -sy[p], k, l, nx, ny);
                fo = (f + 1) * npix;
                ro = f * npix;
                ot = npix;
                const int64_t at2 = g.t_off + f * npix + p, at3 = g.t_off + (F - 1 + f) * npix + p;
                const float wr2 =
                    u != nullptr ? tv_weight(uc - of_sample(u + fo, cf, nx), e2) : w[at2];
                const float wr3 =
                    u != nullptr ? tv_weight(u[i + npix] - of_sample(u + ro, cr, nx), e2) : w[at3];
                if (put) {
                    wout[at2] = wr2;
                    wout[at3] = wr3;
                }
                w2 = sqrtf(wr2);
                w3 = sqrtf(wr3);
            }
        }
        // four columns per step, all their loads issued before any use
        // UC columns per wave per round, their loads issued together (eight in the FP32
        // instances, whose occupancy the LDS tile fixes; four in the BF16 ones)
        constexpr int UC = BF16 ? 4 : 8;
        for (int c0 = cg; c0 < ell; c0 += UC * (BLK / 64)) {
            float x0[UC], x1[UC], x2[UC], x3[UC], m0[UC], m1[UC];
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                const int c = c0 + u * (BLK / 64);
                const bool ok = live && c < ell;
                const float *vc = V + (int64_t)(ok ? c : 0) * ldv;
                if constexpr (!BF16) {
                    const int64_t ic = ok ? i : 0;
                    const float a0 = vc[ic];
                    const float a1 = vc[ic + (ok && ox > 0 ? ox : 0)];
                    const float a2 = vc[ic + (ok && oy > 0 ? oy : 0)];
                    const float a3 = vc[ic + (ok && ot > 0 ? ot : 0)];
                    x0[u] = ok ? a0 : 0.0f;
                    x1[u] = (ok && ox > 0) ? a1 : x0[u];
                    x2[u] = (ok && oy > 0) ? a2 : x0[u];
                    x3[u] = (ok && ot > 0) ? a3 : x0[u];
                } else {
                    // (the BF16 instances keep the guarded form: the unconditional one needs
                    // registers that would cost them a wave per SIMD)
                    x0[u] = ok ? vc[i] : 0.0f;
                    x1[u] = (ok && ox > 0) ? vc[i + ox] : x0[u];
                    x2[u] = (ok && oy > 0) ? vc[i + oy] : x0[u];
                    x3[u] = (ok && ot > 0) ? vc[i + ot] : x0[u];
                }
                // motion rows: the column's frames f + 1 and f warped at the pixel's cells
                m0[u] = (ok && motion && ot > 0) ? of_sample(vc + fo, cf, nx) : x0[u];
                m1[u] = (ok && motion && ot > 0) ? of_sample(vc + ro, cr, nx) : x3[u];
            }
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                const int c = c0 + u * (BLK / 64);
                if (stage && c < ell) {
                    // kind-major rows (row = kind * mp + pixel): consecutive lanes write
                    // consecutive LDS words
                    Elem *col = &sB[c][pc];
                    const float d0 = w0 * (x1[u] - x0[u]), d1 = w1 * (x2[u] - x0[u]);
                    const float d2 = motion ? w2 * (x0[u] - m0[u]) : w2 * (x3[u] - x0[u]);
                    const float d3 = w3 * (x3[u] - m1[u]);
                    if constexpr (BF16) {
                        col[0] = bf16_rne(d0);
                        col[mp] = bf16_rne(d1);
                        if (KIND >= 3) col[2 * mp] = bf16_rne(d2);
                        if (motion) col[3 * mp] = bf16_rne(d3);
                    } else {
                        col[0] = d0;
                        col[mp] = d1;
                        if (KIND >= 3) col[2 * mp] = d2;
                        if (motion) col[3 * mp] = d3;
                    }
                }
            }
        }
        __syncthreads();
        if (busy) {
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
            const int ca = 32 * ti + (lane & 31), cb = 32 * tj + (lane & 31);
            const int kbeg = (MR * sl) / nsl, kend = (MR * (sl + 1)) / nsl;
            if constexpr (BF16) {
                // row slices are multiples of 8 (MR in {128, 192}, split in 1 or 4 parts)
                for (int k0 = kbeg; k0 < kend; k0 += 8) {
                    const int row = k0 + 4 * (lane >> 5);
                    const s16x4 av = *reinterpret_cast<const s16x4 *>(&sB[ca][row]);
                    const s16x4 bv = *reinterpret_cast<const s16x4 *>(&sB[cb][row]);
                    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
                }
            } else {
                for (int k0 = kbeg; k0 < kend; k0 += 2) {
                    const int row = k0 + (lane >> 5);
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sB[ca][row], sB[cb][row], acc, 0,
                                                               0, 0);
                }
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) accd[r] += (double)acc[r];
        }
        __syncthreads();
    }
    double *out = part + gbid * ell * ell;
    if (single) {
        // the four row slices of tile (0,0) meet in LDS (the staging area is free after the
        // last chunk's barrier), summed in slice order
        static_assert(RAW >= 3 * 16 * 64 * sizeof(double), "staging too small");
        double *sacc = reinterpret_cast<double *>(sraw);   // [3][16][64]
        if (wv > 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) sacc[((wv - 1) * 16 + r) * 64 + lane] = accd[r];
        }
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const double v = ((accd[r] + sacc[r * 64 + lane]) + sacc[(16 + r) * 64 + lane]) +
                                 sacc[(32 + r) * 64 + lane];
                const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int j = lane & 31;
                if (i < ell && j < ell) out[i * ell + j] = v;
            }
        }
    } else if (busy) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 32 * ti + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int j = 32 * tj + (lane & 31);
            if (i < ell && j < ell) {
                out[i * ell + j] = accd[r];
                if (ti != tj) out[j * ell + i] = accd[r];
            }
        }
    }
}

// Sum nblk partial ell x ell matrices into G (leading dimension ldg): one wave per entry,
// fixed summation order.  Blocks beyond ell * ell reduce a pending data-Gram column (outputs
// of the multidot run inside the Gram launch, reduce_vec_k's order and values): the new row
// and column col.ell of col.G and col.rb[col.ell].
__global__ __launch_bounds__(64) void reduce_gram_k(const double *__restrict__ part, int nblk,
                                                    int ell, double *__restrict__ G, int ldg,
                                                    GramColJob col)
{
    const int t = blockIdx.x;
    if (t >= ell * ell) {
        const int i = t - ell * ell, nout = col.ell + 2;
        double s = md::strided_sum(col.part + i, nout, col.cblk, threadIdx.x, 64);
        s = wave_sum(s);
        if (threadIdx.x == 0) {
            if (i <= col.ell) {
                col.G[i * col.ldg + col.ell] = s;
                col.G[col.ell * col.ldg + i] = s;
            } else {
                col.rb[col.ell] = s;
            }
        }
        return;
    }
    double s = md::strided_sum(part + t, (int64_t)ell * ell, nblk, threadIdx.x, 64);
    s = wave_sum(s);
    if (threadIdx.x == 0) {
        const int i = t / ell, j = t - i * ell;
        G[i * ldg + j] = s;
    }
}

// ---------------------------------------------------------------------------
// multi-dot / GEMV over basis blocks (FP32 storage, FP64 accumulation)
// ---------------------------------------------------------------------------
// part[blk][i] = sum over this block's entries of X_i[e] * y[e], i < nv; X_i = X + i*ldx.
// An extra row (i = nv) accumulates y[e] * z[e] when z != null.

__global__ __launch_bounds__(BLK) void multidot_k(const float *__restrict__ X, int64_t ldx, int nv,
                                                  const float *__restrict__ y,
                                                  const float *__restrict__ z, int64_t n,
                                                  double *__restrict__ part, const int *skip)
{
    if (skip != nullptr && *skip != 0) return;
    __shared__ double sacc[16][BLK];
    multidot_body<MD_MAX>(X, ldx, nv, y, z, n, part, sacc, blockIdx.x, gridDim.x);
}

// out[i * ostride] = sum_b part[b][i]: one wave per output, lane-strided partial sums
// and a fixed butterfly, so the result is independent of scheduling.
__global__ __launch_bounds__(64) void reduce_vec_k(const double *__restrict__ part, int nblk,
                                                   int nout, double *__restrict__ out,
                                                   int ostride, const int *skip,
                                                   double *__restrict__ G, int ldg,
                                                   double *__restrict__ rb)
{
    if (skip != nullptr && *skip != 0) return;
    const int i = blockIdx.x;
    double s = md::strided_sum(part + i, nout, nblk, threadIdx.x, 64);
    s = wave_sum(s);
    if (threadIdx.x != 0) return;
    if (G == nullptr) {
        out[(int64_t)i * ostride] = s;
    } else {
        // new row / column ell = nout - 2 of a symmetric Gram, last output into rb[ell]
        const int ell = nout - 2;
        if (i <= ell) {
            G[i * ldg + ell] = s;
            G[ell * ldg + i] = s;
        } else {
            rb[ell] = s;
        }
    }
}

// A multidot's block partials summed inside a consumer block, so that they need no launch of
// their own.  Stage 1: acc[L][i] = part[L][i] + part[L + 64][i] + ... (all (L, i) pairs
// spread over the block's threads, consecutive threads on consecutive partials, every load of
// a thread in flight at once).  Stage 2: thread i adds the 64 accumulators of output i in a
// fixed order (eight interleaved sums, then their tree), reading consecutive LDS words across
// the threads.  Deterministic: the order depends only on nblk and nout.  sbuf holds
// MD_MAX * 64 doubles, sh receives the nout sums; ends with a barrier.
constexpr int RR_MAXBLK = 512;   // producer blocks a consumer re-reduces (<= 8 per lane)

// K: partials per accumulator (nblk <= 64 K); U pairs per thread per round, 36 loads in flight
template <int K>
__device__ void rereduce_k(const double *__restrict__ part, int nblk, int nout, double *sbuf,
                           double *sh)
{
    constexpr int U = 36 / K;
    const int tid = threadIdx.x;
    const int npair = nout * 64;
    for (int q0 = 0; q0 < npair; q0 += BLK * U) {
        double v[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // unconditional loads at clamped indices (a load under a branch is waited for
            // before the branch closes, which would serialise them); the sums below skip the
            // clamped ones
            const int q = min(q0 + u * BLK + tid, npair - 1);
            const int L = q / nout, i = q - L * nout;
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[u][k] = part[(int64_t)min(L + 64 * k, nblk - 1) * nout + i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * BLK + tid;
            if (q < npair) {
                const int L = q / nout;
                double a = 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (L + 64 * k < nblk) a += v[u][k];
                sbuf[q] = a;   // pair-major: sbuf[L * nout + i]
            }
        }
    }
    __syncthreads();
    if (tid < nout) {
        double a8[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) a8[r] = sbuf[r * nout + tid];
#pragma unroll
        for (int L = 8; L < 64; ++L) a8[L & 7] += sbuf[L * nout + tid];
        sh[tid] = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
    }
    __syncthreads();
}

__device__ void rereduce(const double *__restrict__ part, int nblk, int nout, double *sbuf,
                         double *sh)
{
    if (nblk <= 256)
        rereduce_k<4>(part, nblk, nout, sbuf, sh);
    else
        rereduce_k<8>(part, nblk, nout, sbuf, sh);
}

// First correction of CGS2 fused with the second pass's products (Alg. "enlarge":
// reorthogonalisation of the new direction).  h = X^T r and ||r||^2 are summed from the
// partials of the multidot that precedes (pin, nin blocks, nv + 1 outputs; block 0 stores
// them in hout), r <- r - X h as gemv_k computes it, then the partials of X^T r as
// multidot_k(X, r) forms them with the same grid (pout[block][i], i < nv).  Every
// element of r is rewritten and read back by the same thread, so no grid-wide order is
// needed.
__global__ __launch_bounds__(BLK) void gemv_multidot_k(const float *__restrict__ X, int64_t ldx,
                                                       int nv, float *r, int64_t n,
                                                       const double *__restrict__ pin, int nin,
                                                       double *__restrict__ pout,
                                                       double *__restrict__ hout)
{
    constexpr int GRP = 16;
    __shared__ double sbuf[MD_MAX * 64];
    __shared__ double sh[MD_MAX];
    const int tid = threadIdx.x;
    rereduce(pin, nin, nv + 1, sbuf, sh);
    if (blockIdx.x == 0 && tid <= nv) hout[tid] = sh[tid];
    double(*sacc)[BLK] = reinterpret_cast<double(*)[BLK]>(sbuf);   // GRP x BLK, free now
    auto block_reduce = [&](int i0, const double (&acc)[GRP]) __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < GRP; ++a) sacc[a][tid] = acc[a];
        __syncthreads();
        constexpr int TPO = BLK / GRP;
        const int a = tid / TPO, l = tid % TPO;
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < BLK / TPO; ++k) t += sacc[a][l + TPO * k];
        for (int off = TPO / 2; off > 0; off >>= 1) t += __shfl_xor(t, off, TPO);
        if (l == 0 && i0 + a < nv) pout[(int64_t)blockIdx.x * nv + i0 + a] = t;
        __syncthreads();
    };
    if ((int64_t)gridDim.x * BLK >= n) {
        const int64_t e = (int64_t)blockIdx.x * BLK + tid;
        const bool in = e < n;
        // the columns' loads issued together: unconditional, at a clamped column and element
        // (a load under a per-lane branch is waited for before the branch closes), the
        // clamped ones zeroed after
        const int64_t ec = in ? e : 0;
        float xv[MD_MAX];
#pragma unroll
        for (int i = 0; i < MD_MAX; ++i) xv[i] = X[(int64_t)min(i, nv - 1) * ldx + ec];
#pragma unroll
        for (int i = 0; i < MD_MAX; ++i) xv[i] = (i < nv && in) ? xv[i] : 0.0f;
        double sg = 0.0;
#pragma unroll
        for (int i = 0; i < MD_MAX; ++i)
            if (i < nv) sg = fma((double)xv[i], sh[i], sg);
        float ye = 0.0f;
        if (in) {
            ye = (float)(-1.0 * sg + 1.0 * (double)r[e]);
            r[e] = ye;
        }
#pragma unroll
        for (int i0 = 0; i0 < MD_MAX; i0 += GRP) {
            if (i0 < nv) {
                double acc[GRP];
#pragma unroll
                for (int a = 0; a < GRP; ++a) acc[a] = (double)xv[i0 + a] * (double)ye;
                block_reduce(i0, acc);
            }
        }
        return;
    }
    // several elements per thread: the correction first, over exactly the elements (and with
    // the layout) that multidot_k gives this thread, then multidot_k's loops on the result
    const bool vec4 = (ldx % 4) == 0 && (n % 4) == 0 &&
                      (reinterpret_cast<uintptr_t>(X) % 16) == 0 &&
                      (reinterpret_cast<uintptr_t>(r) % 16) == 0;
    const int64_t per = vec4 ? 4 : 1, ne = vec4 ? n / 4 : n;
    for (int64_t q = (int64_t)blockIdx.x * BLK + tid; q < ne; q += (int64_t)gridDim.x * BLK) {
        for (int64_t e = q * per; e < q * per + per; ++e) {
            double sg = 0.0;
            for (int i = 0; i < nv; ++i) sg = fma((double)X[(int64_t)i * ldx + e], sh[i], sg);
            r[e] = (float)(-1.0 * sg + 1.0 * (double)r[e]);
        }
    }
    for (int i0 = 0; i0 < nv; i0 += GRP) {
        double acc[GRP];
#pragma unroll
        for (int a = 0; a < GRP; ++a) acc[a] = 0.0;
        if (vec4) {
            const int64_t ld4 = ldx / 4;
            const float4 *X4 = reinterpret_cast<const float4 *>(X);
            const float4 *y4 = reinterpret_cast<const float4 *>(r);
            for (int64_t e = (int64_t)blockIdx.x * BLK + tid; e < ne;
                 e += (int64_t)gridDim.x * BLK) {
                const float4 yv = y4[e];
#pragma unroll
                for (int a = 0; a < GRP; ++a) {
                    const int i = i0 + a;
                    float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (i < nv) xv = X4[(int64_t)i * ld4 + e];
                    double t = acc[a];
                    t = fma((double)xv.x, (double)yv.x, t);
                    t = fma((double)xv.y, (double)yv.y, t);
                    t = fma((double)xv.z, (double)yv.z, t);
                    acc[a] = fma((double)xv.w, (double)yv.w, t);
                }
            }
        } else {
            for (int64_t e = (int64_t)blockIdx.x * BLK + tid; e < n;
                 e += (int64_t)gridDim.x * BLK) {
                const double ye = (double)r[e];
#pragma unroll
                for (int a = 0; a < GRP; ++a) {
                    const int i = i0 + a;
                    if (i < nv) acc[a] = fma((double)X[(int64_t)i * ldx + e], ye, acc[a]);
                }
            }
        }
        block_reduce(i0, acc);
    }
}

// Second correction of CGS2 with its norm: h2 summed from the partials of
// gemv_multidot_k (block 0 stores it in hout), then gemv_norm_k's work.
__global__ __launch_bounds__(BLK) void gemv_norm_red_k(const float *__restrict__ X, int64_t ldx,
                                                       int nv, float *r, int64_t n,
                                                       const double *__restrict__ pin, int nin,
                                                       double *__restrict__ hout,
                                                       double *__restrict__ part)
{
    __shared__ double sbuf[MD_MAX * 64];
    __shared__ double sh[MD_MAX];
    __shared__ double sw[BLK / 64];
    rereduce(pin, nin, nv, sbuf, sh);
    if (blockIdx.x == 0 && (int)threadIdx.x < nv) hout[threadIdx.x] = sh[threadIdx.x];
    double q = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BLK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLK) {
        double sg = 0.0;
        for (int i = 0; i < nv; ++i) sg = fma((double)X[(int64_t)i * ldx + e], sh[i], sg);
        const float o = (float)(-1.0 * sg + 1.0 * (double)r[e]);
        r[e] = o;
        q = fma((double)o, (double)o, q);
    }
    q = wave_sum(q);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < BLK / 64; ++w) t += sw[w];
        part[blockIdx.x] = t;
    }
}

// The data Gram from scratch: every inner product of the columns of [X, b] (nc <= 10 columns
// of X in slots 0 .. nc-1, b in slot 10, zeros between) in one launch.  Pairs (i, j), i <= j,
// in a fixed order, so every register index is static; FP64 sums of the exact products,
// block partials part[block][pair] reduced through LDS in groups of 16 as multidot_k reduces
// its outputs (the same values as one multidot per column).
constexpr int PG_SLOTS = 11;
constexpr int PG_PAIRS = PG_SLOTS * (PG_SLOTS + 1) / 2;   // 66

__host__ __device__ constexpr int pg_first(int p)
{
    int i = 0;
    while (p >= PG_SLOTS - i) {
        p -= PG_SLOTS - i;
        ++i;
    }
    return i;
}
__host__ __device__ constexpr int pg_second(int p)
{
    int i = 0;
    while (p >= PG_SLOTS - i) {
        p -= PG_SLOTS - i;
        ++i;
    }
    return i + p;
}

__global__ __launch_bounds__(BLK) void gram_cols_k(const float *__restrict__ X, int64_t ldx,
                                                   int nc, const float *__restrict__ b,
                                                   int64_t n, double *__restrict__ part)
{
    constexpr int GRP = 16;
    __shared__ double sacc[GRP][BLK];
    const int tid = threadIdx.x;
#pragma unroll
    for (int g0 = 0; g0 < PG_PAIRS; g0 += GRP) {
        double acc[GRP];
#pragma unroll
        for (int a = 0; a < GRP; ++a) acc[a] = 0.0;
        for (int64_t e = (int64_t)blockIdx.x * BLK + tid; e < n; e += (int64_t)gridDim.x * BLK) {
            float v[PG_SLOTS];
#pragma unroll
            for (int k = 0; k < PG_SLOTS - 1; ++k) v[k] = k < nc ? X[(int64_t)k * ldx + e] : 0.0f;
            v[PG_SLOTS - 1] = b[e];
#pragma unroll
            for (int a = 0; a < GRP; ++a) {
                const int pidx = g0 + a;
                if (pidx < PG_PAIRS)
                    acc[a] = fma((double)v[pg_first(pidx)], (double)v[pg_second(pidx)], acc[a]);
            }
        }
#pragma unroll
        for (int a = 0; a < GRP; ++a) sacc[a][tid] = acc[a];
        __syncthreads();
        constexpr int TPO = BLK / GRP;
        const int a = tid / TPO, l = tid % TPO;
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < BLK / TPO; ++k) t += sacc[a][l + TPO * k];
        for (int off = TPO / 2; off > 0; off >>= 1) t += __shfl_xor(t, off, TPO);
        if (l == 0 && g0 + a < PG_PAIRS) part[(int64_t)blockIdx.x * PG_PAIRS + g0 + a] = t;
        __syncthreads();
    }
}

// One wave per pair: its nblk partials summed as reduce_vec_k sums them, written as G[i][j]
// and G[j][i] (i, j < nc), rb[i] (the pair of column i with b) or bn2 (b with itself).
__global__ __launch_bounds__(64) void gram_cols_reduce_k(const double *__restrict__ part,
                                                         int nblk, int nc,
                                                         double *__restrict__ G, int ldg,
                                                         double *__restrict__ rb,
                                                         double *__restrict__ bn2)
{
    const int p = blockIdx.x;
    const int i = pg_first(p), j = pg_second(p);
    const bool bi = i == PG_SLOTS - 1, bj = j == PG_SLOTS - 1;
    if ((!bi && i >= nc) || (!bj && j >= nc)) return;
    double s = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 64) s += part[(int64_t)k * PG_PAIRS + p];
    s = wave_sum(s);
    if (threadIdx.x != 0) return;
    if (!bi && !bj) {
        G[i * ldg + j] = s;
        G[j * ldg + i] = s;
    } else if (!bi) {
        rb[i] = s;
    } else {
        bn2[0] = s;
    }
}

// out[e] = alpha * a[e] + beta * sum_i X_i[e] c_i   (a may be null or equal to out; c FP64
// on the device)
__global__ __launch_bounds__(BLK) void gemv_k(const float *__restrict__ X, int64_t ldx, int nv,
                                              const double *__restrict__ c, double beta,
                                              const float *a, double alpha, int64_t n,
                                              float *out)
{
    __shared__ double sc[MD_MAX];
    for (int i = threadIdx.x; i < nv; i += BLK) sc[i] = c[i];
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * BLK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLK) {
        double s = 0.0;
        for (int i = 0; i < nv; ++i) s = fma((double)X[(int64_t)i * ldx + e], sc[i], s);
        double r = beta * s;
        if (a) r += alpha * (double)a[e];
        out[e] = (float)r;
    }
}

// Two independent gemv_k jobs in one launch (blocks [0, g0) do the first).
struct GemvJob {
    const float *X;
    int64_t ldx;
    int nv;
    const double *c;
    double beta;
    const float *a;
    double alpha;
    int64_t n;
    float *out;
};

__global__ __launch_bounds__(BLK) void gemv2_k(GemvJob j0, GemvJob j1, unsigned g0)
{
    const bool first = blockIdx.x < g0;
    const GemvJob &j = first ? j0 : j1;
    const int64_t blk = first ? blockIdx.x : blockIdx.x - g0;
    const int64_t nblk = first ? g0 : gridDim.x - g0;
    // the coefficients read where they are (one address for the whole block): no LDS staging
    // and no barrier ahead of the first column loads
    const double *__restrict__ sc = j.c;
    for (int64_t e = blk * BLK + threadIdx.x; e < j.n; e += nblk * BLK) {
        double s = 0.0;
#pragma unroll 8
        for (int i = 0; i < j.nv; ++i) s = fma((double)j.X[(int64_t)i * j.ldx + e], sc[i], s);
        double r = j.beta * s;
        if (j.a) r += j.alpha * (double)j.a[e];
        j.out[e] = (float)r;
    }
}

// out = r - X c (as gemv_k with beta = -1, alpha = 1, a = r), plus per-block partial sums of
// out^2 (FP64) in part[block].
__global__ __launch_bounds__(BLK) void gemv_norm_k(const float *__restrict__ X, int64_t ldx, int nv,
                                                   const double *__restrict__ c,
                                                   const float *r, int64_t n, float *out,
                                                   double *__restrict__ part)
{
    __shared__ double sc[MD_MAX];
    __shared__ double sw[BLK / 64];
    for (int i = threadIdx.x; i < nv; i += BLK) sc[i] = c[i];
    __syncthreads();
    double q = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BLK + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * BLK) {
        double s = 0.0;
        for (int i = 0; i < nv; ++i) s = fma((double)X[(int64_t)i * ldx + e], sc[i], s);
        const float o = (float)(-1.0 * s + 1.0 * (double)r[e]);
        out[e] = o;
        q = fma((double)o, (double)o, q);
    }
    q = wave_sum(q);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < BLK / 64; ++w) t += sw[w];
        part[blockIdx.x] = t;
    }
}

// scal[1] = sum_b part[b] (same fixed order in every block), then as normalize_into_k:
// vout = r / sqrt(scal[1]) with the breakdown test against sqrt(scal[0]).
__global__ __launch_bounds__(BLK) void normalize_red_k(const float *__restrict__ r,
                                                       const double *__restrict__ part, int nblk,
                                                       double *__restrict__ scal, double tol,
                                                       int64_t n, float *__restrict__ vout,
                                                       int *__restrict__ status)
{
    __shared__ double stot;
    if (threadIdx.x < 64) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 64) t += part[b];
        t = wave_sum(t);
        if (threadIdx.x == 0) stot = t;
    }
    __syncthreads();
    const double tot = stot;
    const double raw = sqrt(fmax(scal[0], 0.0));
    const double perp = sqrt(fmax(tot, 0.0));
    const double inv = perp > 0.0 ? 1.0 / perp : 0.0;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) {
        scal[1] = tot;
        if (!(perp > tol * raw)) atomicOr(status, NLRMM_ST_BREAKDOWN);
        if (!isfinite(perp)) atomicOr(status, NLRMM_ST_NONFINITE);
    }
    if (e < n) vout[e] = (float)((double)r[e] * inv);
}

// r -= V h with h = part-reduced coefficients already in `h` (FP64).
// (gemv_k with alpha = 1, beta = -1, a = r, out = r covers this.)

// V_new[:, j] = sum_i V[:, i] T[i][j] for j < kout, written to Y (column stride ldy).
__global__ __launch_bounds__(BLK) void block_update_k(const float *__restrict__ X, int64_t ldx,
                                                      int nin, const double *__restrict__ T,
                                                      int ldt, int kout, int64_t n,
                                                      float *__restrict__ Y, int64_t ldy)
{
    __shared__ double sT[MD_MAX * 16];
    const int tid = threadIdx.x;
    for (int i = tid; i < nin * kout; i += BLK) {
        const int r = i / kout, c = i - r * kout;
        sT[i] = T[r * ldt + c];
    }
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * BLK + tid; e < n; e += (int64_t)gridDim.x * BLK) {
        double acc[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = 0.0;
        for (int i = 0; i < nin; ++i) {
            const double xv = (double)X[(int64_t)i * ldx + e];
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c < kout) acc[c] = fma(xv, sT[i * kout + c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c < kout) Y[(int64_t)c * ldy + e] = (float)acc[c];
    }
}

// Y[c][e] = sum_i X[i][e] T[i][c] (c < kout <= 16) with BF16 operands on the matrix cores
// and FP32 accumulation (the basis GEMM V [W, c] of the mixed-precision path).  One wave
// per 32 pixels: D = A B with A[c][i] = T[i][c] (32 x 8 per step, rows c >= kout zero) and
// B[i][e] = X[i][e] (8 x 32), v_mfma_f32_32x32x8bf16_1k; lane l then holds pixel l % 32 of
// outputs c = 8 (r / 4) + 4 (l / 32) + r % 4, r < 16, so the stores are coalesced.
__global__ __launch_bounds__(BLK) void block_update_bf16_k(const float *__restrict__ X,
                                                           int64_t ldx, int nin,
                                                           const double *__restrict__ T, int ldt,
                                                           int kout, int64_t n,
                                                           float *__restrict__ Y, int64_t ldy)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t e0 = ((int64_t)blockIdx.x * (BLK / 64) + wv) * 32;
    if (e0 >= n) return;   // whole wave
    const int m = lane & 31, kq = 4 * (lane >> 5);
    const int64_t e = e0 + m;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    for (int i0 = 0; i0 < nin; i0 += 8) {
        s16x4 av, bv;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + kq + q;
            const float t = (i < nin && m < kout) ? (float)T[i * ldt + m] : 0.0f;
            const float x = (i < nin && e < n) ? X[(int64_t)i * ldx + e] : 0.0f;
            av[q] = bf16_rne(t);
            bv[q] = bf16_rne(x);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
    if (e < n) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int c = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (c < kout) Y[(int64_t)c * ldy + e] = acc[r];
        }
    }
}

__global__ void copy_cols_k(const float *__restrict__ src, int64_t lds, float *__restrict__ dst,
                            int64_t ldd, int ncols, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * ncols) return;
    const int64_t c = t / n, e = t - c * n;
    dst[c * ldd + e] = src[c * lds + e];
}

// v = r / ||r|| into column `col` of V; breakdown when ||r_perp|| <= tol ||r_raw||.
// scal[0] = ||r_raw||^2, scal[1] = ||r_perp||^2 (device).  On breakdown the column is
// still written (normalised) and the status bit is set.
__global__ void normalize_into_k(const float *__restrict__ r, const double *__restrict__ scal,
                                 double tol, int64_t n, float *__restrict__ vout,
                                 int *__restrict__ status, double *__restrict__ norm_out)
{
    const double raw = sqrt(fmax(scal[0], 0.0));
    const double perp = sqrt(fmax(scal[1], 0.0));
    const double inv = perp > 0.0 ? 1.0 / perp : 0.0;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) {
        if (!(perp > tol * raw)) atomicOr(status, NLRMM_ST_BREAKDOWN);
        if (!isfinite(perp)) atomicOr(status, NLRMM_ST_NONFINITE);
        if (norm_out) *norm_out = perp;
    }
    if (e < n) vout[e] = (float)((double)r[e] * inv);
}

// ---------------------------------------------------------------------------
// single-workgroup FP64 dense linear algebra (ell <= 64), all operands in LDS
// ---------------------------------------------------------------------------
// In-place lower Cholesky of the n x n matrix A (row stride ld).  Returns via *bad a
// non-zero value when a pivot was not positive (the pivot is then replaced by a tiny one).
__device__ void chol_lower(double *A, int n, int ld, int *bad)
{
    const int tid = threadIdx.x;
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            double p = A[j * ld + j];
            if (!(p > 0.0)) {
                *bad = 1;
                p = 1e-300;
            }
            A[j * ld + j] = sqrt(p);
        }
        __syncthreads();
        const double piv = A[j * ld + j];
        for (int i = j + 1 + tid; i < n; i += blockDim.x) A[i * ld + j] /= piv;
        __syncthreads();
        const int m = n - j - 1;
        for (int t = tid; t < m * m; t += blockDim.x) {
            const int i = j + 1 + t / m, k = j + 1 + t % m;
            if (k <= i) A[i * ld + k] -= A[i * ld + j] * A[k * ld + j];
        }
        __syncthreads();
    }
}

// Solve L X = B in place (B: n x nrhs, row stride ldb), L lower (row stride ld).
__device__ void trsm_lower(const double *L, int ld, double *B, int ldb, int n, int nrhs)
{
    const int tid = threadIdx.x;
    for (int j = 0; j < n; ++j) {
        for (int c = tid; c < nrhs; c += blockDim.x) B[j * ldb + c] /= L[j * ld + j];
        __syncthreads();
        const int m = n - j - 1;
        for (int t = tid; t < m * nrhs; t += blockDim.x) {
            const int i = j + 1 + t / nrhs, c = t % nrhs;
            B[i * ldb + c] -= L[i * ld + j] * B[j * ldb + c];
        }
        __syncthreads();
    }
}

// Solve L^T x = y in place (vector), L lower.
__device__ void trsv_lower_T(const double *L, int ld, double *x, int n)
{
    const int tid = threadIdx.x;
    for (int j = n - 1; j >= 0; --j) {
        if (tid == 0) x[j] /= L[j * ld + j];
        __syncthreads();
        for (int i = tid; i < j; i += blockDim.x) x[i] -= L[j * ld + i] * x[j];
        __syncthreads();
    }
}

// Cyclic parallel Jacobi eigen-decomposition of the symmetric n x n matrix A (row stride
// ld, overwritten; eigenvalues end on its diagonal) with eigenvectors accumulated in the
// columns of U.  Round-robin pairing: n/2 disjoint rotations per round.
__device__ void jacobi_eig(double *A, double *U, int n, int ld, double *sc, int *spair)
{
    const int tid = threadIdx.x;
    for (int t = tid; t < n * n; t += blockDim.x) {
        const int i = t / n, j = t % n;
        U[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (n < 2) return;
    const int np = (n + 1) & ~1;   // even number of players (a phantom when n is odd)
    const int npair = np / 2;
    double *cs = sc;               // [npair] cos
    double *sn = sc + 32;          // [npair] sin
    __shared__ int srot;
    __shared__ double sdmax;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) {
            srot = 0;
            double dm = 0.0;
            for (int i = 0; i < n; ++i) dm = fmax(dm, fabs(A[i * ld + i]));
            sdmax = dm;
        }
        __syncthreads();
        const double floor_abs = 1e-14 * sdmax;   // below the rounding noise of A
        for (int r = 0; r < np - 1; ++r) {
            if (tid < npair) {
                int p, q;
                if (tid == 0) {
                    p = r;
                    q = np - 1;
                } else {
                    p = (r + tid) % (np - 1);
                    q = (r - tid + np - 1) % (np - 1);
                }
                if (p > q) {
                    const int t2 = p;
                    p = q;
                    q = t2;
                }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[p * ld + q];
                    const double app = A[p * ld + p], aqq = A[q * ld + q];
                    if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                        srot = 1;
                    } else {
                        q = -1;
                    }
                } else {
                    q = -1;
                }
                cs[tid] = c;
                sn[tid] = s;
                spair[2 * tid] = p;
                spair[2 * tid + 1] = q;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int t = tid; t < npair * n; t += blockDim.x) {
                const int k = t / n, j = t % n;
                const int p = spair[2 * k], q = spair[2 * k + 1];
                if (q < 0) continue;
                const double c = cs[k], s = sn[k];
                const double ap = A[p * ld + j], aq = A[q * ld + j];
                A[p * ld + j] = c * ap - s * aq;
                A[q * ld + j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, U <- U J
            for (int t = tid; t < npair * n; t += blockDim.x) {
                const int k = t / n, i = t % n;
                const int p = spair[2 * k], q = spair[2 * k + 1];
                if (q < 0) continue;
                const double c = cs[k], s = sn[k];
                const double ap = A[i * ld + p], aq = A[i * ld + q];
                A[i * ld + p] = c * ap - s * aq;
                A[i * ld + q] = s * ap + c * aq;
                const double up = U[i * ld + p], uq = U[i * ld + q];
                U[i * ld + p] = c * up - s * uq;
                U[i * ld + q] = s * up + c * uq;
            }
            __syncthreads();
        }
        if (srot == 0) break;
        __syncthreads();
    }
}

// Projected MM-GKS solve (eq. "reduced_problem") from the Grams:
//   GA = (AV)^T AV, GP = (P Psi V)^T (P Psi V), rb = (AV)^T b, scal = {||b||^2, target}.
// With GA = L L^T and L^-1 GP L^-T = U diag(gam) U^T, c = L^-1 rb, beta = U^T c:
//   ||AV z(lam) - b||^2 = sum_i (lam gam_i beta_i / (1 + lam gam_i))^2 + ||b||^2 - ||c||^2,
//   z(lam) = L^-T U diag(1 / (1 + lam gam)) beta.
// lam by the discrepancy principle (residual = target) with a log-bracket
// [1e-10, 1e10] * tr(GA)/tr(GP) and clamping to its ends, or lam = lam_fix >= 0.
// Outputs: z[0..ell), out[0] = lam, out[1] = ||AVz - b||^2 (model), status bits.
__global__ __launch_bounds__(SOLVE_NT) void gks_solve_k(const double *__restrict__ GA,
                                                   const double *__restrict__ GP, int ldg,
                                                   const double *__restrict__ rb,
                                                   const double *__restrict__ scal, int ell,
                                                   double lam_fix, double *__restrict__ z,
                                                   double *__restrict__ out,
                                                   int *__restrict__ status)
{
    // LDS: two n x (n+1) matrices (L then U; K then L again) and four vectors.
    extern __shared__ double sm[];
    const int n = ell, ld = ell + 1;
    double *A = sm;                 // L, later U
    double *K = A + n * ld;         // K, later L again
    double *c = K + n * ld;         // n
    double *be = c + n;             // n
    double *ga = be + n;            // n
    double *yv = ga + n;            // n
    double *sc = yv + n;            // 128 scratch
    __shared__ int spair[64];
    __shared__ int sbad;
    __shared__ int sfirst;
    const int tid = threadIdx.x;
    if (tid == 0) sbad = 0;
    for (int t = tid; t < n * n; t += SOLVE_NT) {
        const int i = t / n, j = t % n;
        A[i * ld + j] = GA[i * ldg + j];
        K[i * ld + j] = GP[i * ldg + j];
    }
    for (int i = tid; i < n; i += SOLVE_NT) c[i] = rb[i];
    __syncthreads();
    double trA = 0.0, trP = 0.0;
    for (int i = 0; i < n; ++i) {
        trA += A[i * ld + i];
        trP += K[i * ld + i];
    }
    chol_lower(A, n, ld, &sbad);
    trsm_lower(A, ld, c, 1, n, 1);          // c = L^-1 rb
    trsm_lower(A, ld, K, ld, n, n);         // X = L^-1 GP
    for (int t = tid; t < n * n; t += SOLVE_NT) {
        const int i = t / n, j = t % n;
        if (i < j) {
            const double a = K[i * ld + j];
            K[i * ld + j] = K[j * ld + i];
            K[j * ld + i] = a;
        }
    }
    __syncthreads();
    trsm_lower(A, ld, K, ld, n, n);         // K = L^-1 X^T = L^-1 GP L^-T
    for (int t = tid; t < n * n; t += SOLVE_NT) {
        const int i = t / n, j = t % n;
        if (i < j) {
            const double a = 0.5 * (K[i * ld + j] + K[j * ld + i]);
            K[i * ld + j] = a;
            K[j * ld + i] = a;
        }
    }
    __syncthreads();
    jacobi_eig(K, A, n, ld, sc, spair);     // A <- U (L is rebuilt below)
    for (int i = tid; i < n; i += SOLVE_NT) {
        ga[i] = fmax(K[i * ld + i], 0.0);
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += A[k * ld + i] * c[k];
        be[i] = s;
    }
    __syncthreads();
    double cn2 = 0.0;
    for (int i = 0; i < n; ++i) cn2 += c[i] * c[i];
    const double out2 = fmax(scal[0] - cn2, 0.0);
    const double t2 = scal[1] * scal[1];
    auto phi = [&](double lam) {
        double s = out2;
        for (int i = 0; i < n; ++i) {
            const double q = lam * ga[i];
            const double f = q * be[i] / (1.0 + q);
            s += f * f;
        }
        return s;
    };
    double lam;
    int flag = 0;
    if (lam_fix >= 0.0) {
        lam = lam_fix;
    } else {
        const double scale = trA / fmax(trP, 1e-300);
        double lo = log(1e-10 * scale), hi = log(1e10 * scale);
        if (phi(exp(lo)) >= t2) {
            lam = exp(lo);
            flag = NLRMM_ST_DP_LOW;
        } else if (phi(exp(hi)) <= t2) {
            lam = exp(hi);
            flag = NLRMM_ST_DP_HIGH;
        } else {
            // NT-way parallel bracketing: each round shrinks the bracket by NT + 1
            for (int round = 0; round < 12; ++round) {
                const double x = lo + (hi - lo) * (double)(tid + 1) / (double)(SOLVE_NT + 1);
                const int above = phi(exp(x)) >= t2;
                if (tid == 0) sfirst = SOLVE_NT;
                __syncthreads();
                if (above) atomicMin(&sfirst, tid);
                __syncthreads();
                const int k = sfirst;
                const double nlo = (k == 0) ? lo : lo + (hi - lo) * (double)k / (double)(SOLVE_NT + 1);
                const double nhi = (k == SOLVE_NT) ? hi : lo + (hi - lo) * (double)(k + 1) / (double)(SOLVE_NT + 1);
                __syncthreads();
                lo = nlo;
                hi = nhi;
                if (hi - lo <= 4e-16 * fmax(1.0, fabs(lo))) break;
            }
            lam = exp(0.5 * (lo + hi));
        }
    }
    // y = U diag(1/(1 + lam gam)) beta, then z = L^-T y with L refactored into K's storage
    for (int i = tid; i < n; i += SOLVE_NT) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += A[i * ld + k] * (be[k] / (1.0 + lam * ga[k]));
        yv[i] = s;
    }
    __syncthreads();
    for (int t = tid; t < n * n; t += SOLVE_NT) {
        const int i = t / n, j = t % n;
        K[i * ld + j] = GA[i * ldg + j];
    }
    __syncthreads();
    chol_lower(K, n, ld, &sbad);
    trsv_lower_T(K, ld, yv, n);
    for (int i = tid; i < n; i += SOLVE_NT) z[i] = yv[i];
    if (tid == 0) {
        out[0] = lam;
        out[1] = phi(lam);
        int st = flag;
        if (sbad) st |= NLRMM_ST_NONFINITE;
        if (!isfinite(lam) || !isfinite(out[1])) st |= NLRMM_ST_NONFINITE;
        if (st) atomicOr(status, st);
    }
}

// Projected MM-GKS solve, single-wave tridiagonal form (same mathematics as gks_solve_k).
// With GA = L L^T (augmented Cholesky of [[GA, rb], [rb^T, ||b||^2]] also gives c = L^-1 rb
// and out2 = ||b||^2 - ||c||^2) and K = L^-1 GP L^-T, a reflector H0 maps c to s ||c|| e1
// and Householder tridiagonalisation of H0 K H0 (which leaves e1 fixed) gives T = Q^T K Q.
// With y = (I + lam T)^-1 e1 one has ||AV z(lam) - b||^2 = out2 + ||c||^2 ||e1 - y||^2, and
// the pivots of the bottom-up elimination of I + lam T,
//   D_{n-1} = 1 + lam d_{n-1},  D_i = 1 + lam d_i - lam^2 e_i^2 / D_{i+1},
// give y_0 = 1 / D_0 and y_i = -(lam e_{i-1} / D_i) y_{i-1}, so ||e1 - y||^2 is a sum of
// nonnegative terms accumulated in the same O(ell) sweep (no eigenvectors).  Each lane
// evaluates one lam; a 65-way bracket search runs on the log-bracket of the discrepancy
// principle.  z = L^-T Q (I + lam T)^-1 (s ||c|| e1).
constexpr int TRI_NT = 64;

__device__ __forceinline__ double wsum64(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(TRI_NT) void gks_solve_tri_k(const double *__restrict__ GA,
                                                         const double *__restrict__ GP, int ldg,
                                                         const double *__restrict__ rb,
                                                         const double *__restrict__ scal, int ell,
                                                         double lam_fix, double *__restrict__ z,
                                                         double *__restrict__ out,
                                                         int *__restrict__ status)
{
    extern __shared__ double sm[];
    const int n = ell, n1 = ell + 1;
    const int lda = n1 + 1, ldk = n + 1;
    double *A = sm;                   // n1 x lda: augmented matrix -> Cholesky factor
    double *K = A + n1 * lda;         // n x ldk: K, then reflectors stored below the diagonal
    double *vv = K + n * ldk;         // n: current reflector
    double *ww = vv + n;              // n
    double *tau = ww + n;             // n: tau_j of reflector j (j = 0 is H0, j >= 1 tridiag)
    double *dd = tau + n;             // n: diagonal of T
    double *ee = dd + n;              // n: sub-diagonal of T
    double *yv = ee + n;              // n
    double *h0 = yv + n;              // n: reflector H0
    __shared__ int sbad;
    __shared__ int sfirst;
    const int tid = threadIdx.x;
    if (tid == 0) sbad = 0;
    for (int t = tid; t < n * n; t += TRI_NT) {
        const int i = t / n, j = t - (t / n) * n;
        A[i * lda + j] = GA[i * ldg + j];
        K[i * ldk + j] = GP[i * ldg + j];
    }
    for (int i = tid; i < n; i += TRI_NT) {
        A[i * lda + n] = rb[i];
        A[n * lda + i] = rb[i];
    }
    if (tid == 0) A[n * lda + n] = scal[0];
    __syncthreads();
    double trA = 0.0, trP = 0.0;
    for (int i = 0; i < n; ++i) {
        trA += A[i * lda + i];
        trP += K[i * ldk + i];
    }
    // 1. augmented Cholesky (right-looking, lower); the last pivot is left unrooted (= out2)
    for (int j = 0; j < n1; ++j) {
        if (tid == 0 && j < n) {
            double p = A[j * lda + j];
            if (!(p > 0.0)) {
                sbad = 1;
                p = 1e-300;
            }
            A[j * lda + j] = sqrt(p);
        }
        __syncthreads();
        if (j == n) break;
        const double piv = A[j * lda + j];
        for (int i = j + 1 + tid; i < n1; i += TRI_NT) A[i * lda + j] /= piv;
        __syncthreads();
        const int m = n1 - j - 1;
        for (int t = tid; t < m * m; t += TRI_NT) {
            const int i = j + 1 + t / m, k = j + 1 + t % m;
            if (k <= i) A[i * lda + k] -= A[i * lda + j] * A[k * lda + j];
        }
        __syncthreads();
    }
    double cn2 = 0.0;
    for (int k = 0; k < n; ++k) cn2 += A[n * lda + k] * A[n * lda + k];
    const double out2 = fmax(scal[0] - cn2, 0.0);
    const double cn = sqrt(cn2);
    // 2. K = L^-1 GP L^-T (column sweeps, one column per lane)
    for (int pass = 0; pass < 2; ++pass) {
        for (int k = 0; k < n; ++k) {
            const double lkk = A[k * lda + k];
            for (int c = tid; c < n; c += TRI_NT) K[k * ldk + c] /= lkk;
            __syncthreads();
            for (int c = tid; c < n; c += TRI_NT) {
                const double xk = K[k * ldk + c];
                for (int i = k + 1; i < n; ++i) K[i * ldk + c] -= A[i * lda + k] * xk;
            }
            __syncthreads();
        }
        for (int t = tid; t < n * n; t += TRI_NT) {
            const int i = t / n, j = t - (t / n) * n;
            if (i < j) {
                const double a = K[i * ldk + j];
                K[i * ldk + j] = K[j * ldk + i];
                K[j * ldk + i] = a;
            }
        }
        __syncthreads();
    }
    for (int t = tid; t < n * n; t += TRI_NT) {
        const int i = t / n, j = t - (t / n) * n;
        if (i < j) {
            const double a = 0.5 * (K[i * ldk + j] + K[j * ldk + i]);
            K[i * ldk + j] = a;
            K[j * ldk + i] = a;
        }
    }
    __syncthreads();
    // 3. H0 = I - tau0 v v^T with H0 c = s ||c|| e1 (s = -sign(c0)); K <- H0 K H0
    double sgn = 1.0;
    {
        const double c0 = A[n * lda + 0];
        sgn = (c0 >= 0.0) ? -1.0 : 1.0;
        for (int i = tid; i < n; i += TRI_NT) h0[i] = A[n * lda + i] - (i == 0 ? sgn * cn : 0.0);
        __syncthreads();
        double vtv = 0.0;
        for (int i = 0; i < n; ++i) vtv += h0[i] * h0[i];
        const double t0 = vtv > 0.0 ? 2.0 / vtv : 0.0;
        if (tid == 0) tau[0] = t0;
        // p = t0 K v, mu = t0/2 p^T v, w = p - mu v, K -= v w^T + w v^T
        double pi = 0.0;
        if (tid < n) {
            for (int k = 0; k < n; ++k) pi += K[tid * ldk + k] * h0[k];
            pi *= t0;
        }
        const double mu = 0.5 * t0 * wsum64(tid < n ? pi * h0[tid] : 0.0);
        if (tid < n) ww[tid] = pi - mu * h0[tid];
        __syncthreads();
        if (tid < n) {
            const double vi = h0[tid], wi = ww[tid];
            for (int k = 0; k < n; ++k) K[tid * ldk + k] -= vi * ww[k] + wi * h0[k];
        }
        __syncthreads();
    }
    // 4. Householder tridiagonalisation (reflector j acts on indices j+1 .. n-1)
    for (int j = 0; j + 2 < n; ++j) {
        const double xi = (tid > j && tid < n) ? K[tid * ldk + j] : 0.0;
        const double s2 = wsum64(xi * xi);
        const double x0 = K[(j + 1) * ldk + j];
        const double tail = s2 - x0 * x0;
        double tj = 0.0, alpha = x0;
        if (tail > 0.0) {
            const double sigma = sqrt(s2);
            alpha = (x0 >= 0.0) ? -sigma : sigma;
            const double v0 = x0 - alpha;
            tj = 2.0 / (tail + v0 * v0);
            if (tid > j && tid < n) vv[tid] = (tid == j + 1) ? v0 : xi;
        }
        if (tid == 0) {
            dd[j] = K[j * ldk + j];
            ee[j] = alpha;
            tau[j + 1] = tj;
        }
        __syncthreads();
        if (tj != 0.0) {
            double pi = 0.0;
            if (tid > j && tid < n) {
                for (int k = j + 1; k < n; ++k) pi += K[tid * ldk + k] * vv[k];
                pi *= tj;
            }
            const double mu = 0.5 * tj * wsum64((tid > j && tid < n) ? pi * vv[tid] : 0.0);
            if (tid > j && tid < n) ww[tid] = pi - mu * vv[tid];
            __syncthreads();
            if (tid > j && tid < n) {
                const double vi = vv[tid], wi = ww[tid];
                for (int k = j + 1; k < n; ++k) K[tid * ldk + k] -= vi * ww[k] + wi * vv[k];
            }
            __syncthreads();
        }
        // keep the reflector in column j below the sub-diagonal position (v_{j+1} included)
        if (tid > j && tid < n) K[tid * ldk + j] = (tj != 0.0) ? vv[tid] : 0.0;
        __syncthreads();
    }
    if (tid == 0) {
        if (n >= 2) {
            dd[n - 2] = K[(n - 2) * ldk + (n - 2)];
            ee[n - 2] = K[(n - 1) * ldk + (n - 2)];
            if (n >= 3) tau[n - 1] = 0.0;
        }
        dd[n - 1] = K[(n - 1) * ldk + (n - 1)];
        ee[n - 1] = 0.0;
    }
    __syncthreads();
    // 5. discrepancy principle on the tridiagonal form
    auto phi = [&](double lam) {
        // backward sweep: D_i pivots, E_i = D_i - 1, R_1 = sum_{i>=1} (y_i / y_0)^2
        double D = 1.0 + lam * dd[n - 1], E = lam * dd[n - 1], R = 0.0;
        for (int i = n - 2; i >= 0; --i) {
            const double b = lam * ee[i];
            const double b2 = b * b;
            R = b2 / (D * D) * (1.0 + R);
            E = lam * dd[i] - b2 / D;
            D = 1.0 + E;
        }
        return out2 + cn2 * (E * E + R) / (D * D);
    };
    const double t2 = scal[1] * scal[1];
    double lam;
    int flag = 0;
    if (lam_fix >= 0.0) {
        lam = lam_fix;
    } else {
        const double scale = trA / fmax(trP, 1e-300);
        double lo = log(1e-10 * scale), hi = log(1e10 * scale);
        const double plo = phi(exp(lo)), phh = phi(exp(hi));
        if (plo >= t2) {
            lam = exp(lo);
            flag = NLRMM_ST_DP_LOW;
        } else if (phh <= t2) {
            lam = exp(hi);
            flag = NLRMM_ST_DP_HIGH;
        } else {
            for (int round = 0; round < 12; ++round) {
                const double x = lo + (hi - lo) * (double)(tid + 1) / (double)(TRI_NT + 1);
                const int above = phi(exp(x)) >= t2;
                if (tid == 0) sfirst = TRI_NT;
                __syncthreads();
                if (above) atomicMin(&sfirst, tid);
                __syncthreads();
                const int k = sfirst;
                const double nlo = (k == 0) ? lo : lo + (hi - lo) * (double)k / (double)(TRI_NT + 1);
                const double nhi = (k == TRI_NT) ? hi : lo + (hi - lo) * (double)(k + 1) / (double)(TRI_NT + 1);
                __syncthreads();
                lo = nlo;
                hi = nhi;
                if (hi - lo <= 4e-16 * fmax(1.0, fabs(lo))) break;
            }
            lam = exp(0.5 * (lo + hi));
        }
    }
    // 6. y = (I + lam T)^-1 (s ||c|| e1) by a tridiagonal LDL^T solve (one lane)
    if (tid == 0) {
        // forward elimination, pivots kept in ww
        ww[0] = 1.0 + lam * dd[0];
        yv[0] = sgn * cn;
        for (int i = 1; i < n; ++i) {
            const double l = lam * ee[i - 1] / ww[i - 1];
            ww[i] = 1.0 + lam * dd[i] - l * lam * ee[i - 1];
            yv[i] = -l * yv[i - 1];
        }
        yv[n - 1] /= ww[n - 1];
        for (int i = n - 2; i >= 0; --i) yv[i] = (yv[i] - lam * ee[i] * yv[i + 1]) / ww[i];
    }
    __syncthreads();
    // apply the tridiagonalisation reflectors in reverse order, then H0
    for (int j = n - 3; j >= 0; --j) {
        const double tj = tau[j + 1];
        if (tj == 0.0) continue;
        const double vi = (tid > j && tid < n) ? K[tid * ldk + j] : 0.0;
        const double dot = wsum64(vi * ((tid > j && tid < n) ? yv[tid] : 0.0));
        __syncthreads();
        if (tid > j && tid < n) yv[tid] -= tj * dot * vi;
        __syncthreads();
    }
    {
        const double vi = tid < n ? h0[tid] : 0.0;
        const double dot = wsum64(vi * (tid < n ? yv[tid] : 0.0));
        __syncthreads();
        if (tid < n) yv[tid] -= tau[0] * dot * vi;
        __syncthreads();
    }
    // 7. z = L^-T y
    for (int j = n - 1; j >= 0; --j) {
        if (tid == 0) yv[j] /= A[j * lda + j];
        __syncthreads();
        for (int i = tid; i < j; i += TRI_NT) yv[i] -= A[j * lda + i] * yv[j];
        __syncthreads();
    }
    for (int i = tid; i < n; i += TRI_NT) z[i] = yv[i];
    if (tid == 0) {
        out[0] = lam;
        out[1] = phi(lam);
        int st = flag;
        if (sbad) st |= NLRMM_ST_NONFINITE;
        if (!isfinite(lam) || !isfinite(out[1])) st |= NLRMM_ST_NONFINITE;
        if (st) atomicOr(status, st);
    }
}


// Compression (Alg. "compress"): S = GA + lam GP = H^T H with H = [RA; sqrt(lam) RP];
// W = eigenvectors of the kmin-1 largest eigenvalues of S (= dominant right singular
// vectors of H), sign rule: largest-magnitude entry positive.  c = z - W W^T z; if
// ||c|| > 1e-12 ||z|| the transform is T = [W, c/||c||] and z' = [W^T z; ||c||], else
// T = W, z' = W^T z and the status bit is set.  Writes T (ell x kmin, row stride ldt),
// z' (zout) and knew (out_k[0]).
__global__ __launch_bounds__(SOLVE_NT) void compress_eig_k(const double *__restrict__ GA,
                                                      const double *__restrict__ GP, int ldg,
                                                      const double *__restrict__ lamp, int ell,
                                                      int kmin, const double *__restrict__ zin,
                                                      double *__restrict__ T, int ldt,
                                                      double *__restrict__ zout,
                                                      int *__restrict__ out_k,
                                                      int *__restrict__ status)
{
    extern __shared__ double sm[];
    const int n = ell, ld = ell + 1;
    double *S = sm;
    double *U = S + n * ld;
    double *sc = U + n * ld;     // 128
    double *zz = sc + 128;       // n
    double *wz = zz + n;         // kmin
    double *cc = wz + kmin;      // n
    __shared__ int spair[64];
    __shared__ int order[64];
    const int tid = threadIdx.x;
    const double lam = lamp[0];
    for (int t = tid; t < n * n; t += SOLVE_NT) {
        const int i = t / n, j = t % n;
        S[i * ld + j] = GA[i * ldg + j] + lam * GP[i * ldg + j];
    }
    for (int i = tid; i < n; i += SOLVE_NT) zz[i] = zin[i];
    __syncthreads();
    for (int t = tid; t < n * n; t += SOLVE_NT) {
        const int i = t / n, j = t % n;
        if (i < j) {
            const double a = 0.5 * (S[i * ld + j] + S[j * ld + i]);
            S[i * ld + j] = a;
            S[j * ld + i] = a;
        }
    }
    __syncthreads();
    jacobi_eig(S, U, n, ld, sc, spair);
    // order eigenvalues descending (rank sort; ties by index)
    for (int i = tid; i < n; i += SOLVE_NT) {
        const double ei = S[i * ld + i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double ej = S[j * ld + j];
            if (ej > ei || (ej == ei && j < i)) ++rank;
        }
        order[rank] = i;
    }
    __syncthreads();
    const int kw = kmin - 1;
    // sign rule and W^T z
    for (int a = tid; a < kw; a += SOLVE_NT) {
        const int col = order[a];
        int jm = 0;
        double vm = -1.0;
        for (int i = 0; i < n; ++i) {
            const double v = fabs(U[i * ld + col]);
            if (v > vm) {
                vm = v;
                jm = i;
            }
        }
        const double sg = U[jm * ld + col] < 0.0 ? -1.0 : 1.0;
        double s = 0.0;
        for (int i = 0; i < n; ++i) {
            const double v = sg * U[i * ld + col];
            T[i * ldt + a] = v;
            s += v * zz[i];
        }
        wz[a] = s;
    }
    __syncthreads();
    // c = z - W (W^T z)
    for (int i = tid; i < n; i += SOLVE_NT) {
        double s = zz[i];
        for (int a = 0; a < kw; ++a) s -= T[i * ldt + a] * wz[a];
        cc[i] = s;
    }
    __syncthreads();
    double cn = 0.0, zn = 0.0;
    for (int i = 0; i < n; ++i) {
        cn += cc[i] * cc[i];
        zn += zz[i] * zz[i];
    }
    cn = sqrt(cn);
    zn = sqrt(zn);
    const bool keep = cn > 1e-12 * zn;
    if (keep) {
        for (int i = tid; i < n; i += SOLVE_NT) T[i * ldt + kw] = cc[i] / cn;
    } else {
        for (int i = tid; i < n; i += SOLVE_NT) T[i * ldt + kw] = 0.0;
    }
    for (int a = tid; a < kw; a += SOLVE_NT) zout[a] = wz[a];
    if (tid == 0) {
        if (keep) zout[kw] = cn;
        out_k[0] = keep ? kmin : kw;
        if (!keep) atomicOr(status, NLRMM_ST_COMPRESS_SKIP);
    }
}

// G' = T^T G T (ell -> k), applied to a Gram after compression; rb' = T^T rb.
__global__ __launch_bounds__(BLK) void gram_transform_k(double *__restrict__ G, int ldg,
                                                        double *__restrict__ rb, int ell,
                                                        const double *__restrict__ T, int ldt,
                                                        const int *__restrict__ kp)
{
    extern __shared__ double sm[];
    const int k = kp[0];
    double *GT = sm;            // ell x k : G T
    double *rr = GT + ell * 16; // k
    const int tid = threadIdx.x;
    for (int t = tid; t < ell * k; t += BLK) {
        const int i = t / k, j = t % k;
        double s = 0.0;
        for (int m = 0; m < ell; ++m) s += G[i * ldg + m] * T[m * ldt + j];
        GT[i * 16 + j] = s;
    }
    for (int j = tid; j < k; j += BLK) {
        double s = 0.0;
        for (int m = 0; m < ell; ++m) s += T[m * ldt + j] * rb[m];
        rr[j] = s;
    }
    __syncthreads();
    for (int t = tid; t < k * k; t += BLK) {
        const int i = t / k, j = t % k;
        double s = 0.0;
        for (int m = 0; m < ell; ++m) s += T[m * ldt + i] * GT[m * 16 + j];
        G[i * ldg + j] = s;   // rows/cols beyond k are stale and never read
    }
    __syncthreads();
    for (int j = tid; j < k; j += BLK) rb[j] = rr[j];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned grid_for(int64_t n, int per = BLK, int64_t cap = 4096)
{
    int64_t g = (n + per - 1) / per;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

int k_psi_weights(const float *u, int nx, int ny, int F, int temporal, float eps, float *w,
                  hipStream_t s, const float *flow)
{
    if (temporal == TEMPORAL_OF && F > 1 && (flow == nullptr || nx < 2 || ny < 2))
        return NLRMM_EINVAL;
    const int64_t n = (int64_t)nx * ny * F;
    psi_weights_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(u, nx, ny, F, temporal, eps, w,
                                                             flow);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_psi_apply(const float *u, int nx, int ny, int F, int temporal, float *out, hipStream_t s,
                const float *flow)
{
    if (temporal == TEMPORAL_OF && F > 1 && (flow == nullptr || nx < 2 || ny < 2))
        return NLRMM_EINVAL;
    const int64_t n = (int64_t)nx * ny * F;
    psi_apply_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(u, nx, ny, F, temporal, out, flow);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_tv_grad_add(const float *u, const float *w, int nx, int ny, int F, int temporal,
                  const double *lamp, float *r, hipStream_t s, float eps)
{
    const int64_t n = (int64_t)nx * ny * F;
    tv_grad_add_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(u, w, nx, ny, F, temporal, lamp, r,
                                                             eps * eps);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_gram_psi(const float *V, int64_t ldv, int ell, const float *w, int nx, int ny, int F,
               int temporal, double *part, int nblk, double *G, int ldg, hipStream_t s, int mode,
               const float *u, float eps, const float *flow, float *wout, const GramColJob *col)
{
    if (ell > GMAX) return NLRMM_ESHAPE;
    if (w == nullptr && u == nullptr) return NLRMM_EINVAL;
    if (temporal == TEMPORAL_OF && F > 1 && (flow == nullptr || nx < 2 || ny < 2))
        return NLRMM_EINVAL;
    const float e2 = eps * eps;
    const bool motion = temporal == TEMPORAL_OF && F > 1;
    GramColJob cj{};   // X == nullptr: no column inside this launch
    if (col != nullptr && col->X != nullptr) {
        // blocks of its own, four elements per thread (one 16-byte load per column), so that
        // they and the Gram's blocks are resident together on 256x256 images
        int64_t cb = (col->n + 4 * BLK - 1) / (4 * BLK);
        cb = cb < col->md_blocks ? cb : col->md_blocks;
        if (mode == 1 && col->ell + 2 <= MD_MAX && cb * (col->ell + 2) <= col->part_cap) {
            cj = *col;
            cj.cblk = (int)cb;
        } else {
            const int rc = k_multidot_gram_col(col->X, col->ldx, col->ell, col->xnew, col->b,
                                               col->n, col->part, col->md_blocks, col->G,
                                               col->ldg, col->rb, s);
            if (rc) return rc;
        }
    }
    if (mode == 0) {
        // the FP64 kernel takes stored weights
        if (w == nullptr) {
            if (wout == nullptr) return NLRMM_EINVAL;
            const int rc = k_psi_weights(u, nx, ny, F, temporal, eps, wout, s, flow);
            if (rc) return rc;
            w = wout;
        }
        gram_psi_k<<<(unsigned)nblk, BLK, 0, s>>>(V, ldv, ell, w, nx, ny, F, temporal, part,
                                                  flow);
    } else {
        const float *ww = w ? nullptr : u;
        float *wo = w ? nullptr : wout;
        if (mode == 1 && motion)
            gram_psi_mfma_k<false, true><<<(unsigned)(nblk + cj.cblk), BLK, 0, s>>>(
                V, ldv, ell, w, nx, ny, F, temporal, part, ww, e2, flow, wo, cj);
        else if (mode == 1)
            gram_psi_mfma_k<false, false><<<(unsigned)(nblk + cj.cblk), BLK, 0, s>>>(
                V, ldv, ell, w, nx, ny, F, temporal, part, ww, e2, flow, wo, cj);
        else if (mode == 2 && motion)
            gram_psi_mfma_k<true, true><<<(unsigned)nblk, BLK, 0, s>>>(
                V, ldv, ell, w, nx, ny, F, temporal, part, ww, e2, flow, wo, cj);
        else
            gram_psi_mfma_k<true, false><<<(unsigned)nblk, BLK, 0, s>>>(
                V, ldv, ell, w, nx, ny, F, temporal, part, ww, e2, flow, wo, cj);
    }
    const unsigned rblocks = (unsigned)(ell * ell + (cj.X != nullptr ? cj.ell + 2 : 0));
    reduce_gram_k<<<rblocks, 64, 0, s>>>(part, nblk, ell, G, ldg, cj);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_multidot(const float *X, int64_t ldx, int nv, const float *y, const float *z, int64_t n,
               double *part, int nblk, double *out, int ostride, hipStream_t s, const int *skip)
{
    const int nout = nv + (z ? 1 : 0);
    if (nout > MD_MAX || nblk < 1) return NLRMM_ESHAPE;
    // one element per thread at most, at most the partials' capacity
    int64_t g = (n + BLK - 1) / BLK;
    if (g > nblk) g = nblk;
    if (g < 1) g = 1;
    multidot_k<<<(unsigned)g, BLK, 0, s>>>(X, ldx, nv, y, z, n, part, skip);
    reduce_vec_k<<<(unsigned)nout, 64, 0, s>>>(part, (int)g, nout, out, ostride, skip, nullptr, 0,
                                               nullptr);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_multidot_gram_col(const float *X, int64_t ldx, int ell, const float *xnew, const float *b,
                        int64_t n, double *part, int nblk, double *G, int ldg, double *rb,
                        hipStream_t s)
{
    const int nout = ell + 2;
    if (nout > MD_MAX || nblk < 1) return NLRMM_ESHAPE;
    int64_t g = (n + BLK - 1) / BLK;
    if (g > nblk) g = nblk;
    if (g < 1) g = 1;
    multidot_k<<<(unsigned)g, BLK, 0, s>>>(X, ldx, ell + 1, xnew, b, n, part, nullptr);
    reduce_vec_k<<<(unsigned)nout, 64, 0, s>>>(part, (int)g, nout, nullptr, 0, nullptr, G, ldg,
                                               rb);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_cgs2(const float *X, int64_t ldx, int nv, float *r, int64_t n, double *part1,
           double *part2, int nblk, double *h1, double *h2, double tol, float *vout,
           int *status, hipStream_t s, int p1_blocks, int *norm_blocks)
{
    if (nv + 1 > MD_MAX || nblk < 1) return NLRMM_ESHAPE;
    int64_t g = (n + BLK - 1) / BLK;
    if (g > nblk) g = nblk;
    if (g < 1) g = 1;
    const unsigned g3 = grid_for(n);   // blocks of the norm partials (<= 4096 <= 72 nblk)
    if (p1_blocks > 0) {
        // the first products came with r, from the launch that wrote it (the fused kernels
        // need at least one column: their loads clamp the column index to nv - 1)
        if (p1_blocks != g || g > RR_MAXBLK || nv < 1) return NLRMM_EINVAL;
    } else if (nv < 1 || g > RR_MAXBLK) {
        // a launch per reduction (the same arithmetic except for the order of the block sums)
        int rc;
        if ((rc = k_multidot(X, ldx, nv, r, r, n, part1, nblk, h1, 1, s))) return rc;
        if ((rc = k_gemv(X, ldx, nv, h1, -1.0, r, 1.0, n, r, s))) return rc;
        if ((rc = k_multidot(X, ldx, nv, r, nullptr, n, part1, nblk, h2, 1, s))) return rc;
        gemv_norm_k<<<g3, BLK, 0, s>>>(X, ldx, nv, h2, r, n, r, part1);
        if (norm_blocks) {
            *norm_blocks = (int)g3;
        } else {
            normalize_red_k<<<(unsigned)((n + BLK - 1) / BLK), BLK, 0, s>>>(
                r, part1, (int)g3, h1 + nv, tol, n, vout, status);
        }
        return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
    }
    if (p1_blocks == 0) multidot_k<<<(unsigned)g, BLK, 0, s>>>(X, ldx, nv, r, r, n, part1, nullptr);
    gemv_multidot_k<<<(unsigned)g, BLK, 0, s>>>(X, ldx, nv, r, n, part1, (int)g, part2, h1);
    gemv_norm_red_k<<<g3, BLK, 0, s>>>(X, ldx, nv, r, n, part2, (int)g, h2, part1);
    if (norm_blocks) {
        *norm_blocks = (int)g3;
    } else {
        normalize_red_k<<<(unsigned)((n + BLK - 1) / BLK), BLK, 0, s>>>(r, part1, (int)g3,
                                                                        h1 + nv, tol, n, vout,
                                                                        status);
    }
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_normalize_red(const float *r, const double *part, int nblk, double *scal, double tol,
                    int64_t n, float *vout, int *status, hipStream_t s)
{
    normalize_red_k<<<(unsigned)((n + BLK - 1) / BLK), BLK, 0, s>>>(r, part, nblk, scal, tol, n,
                                                                    vout, status);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_gram_cols(const float *X, int64_t ldx, int nc, const float *b, int64_t n, double *part,
                int nblk, double *G, int ldg, double *rb, double *bn2, hipStream_t s)
{
    if (nc < 1 || nc > PG_SLOTS - 1 || nblk < 1) return NLRMM_ESHAPE;
    if ((size_t)nblk * PG_PAIRS > md_part_doubles(nblk)) return NLRMM_ESHAPE;
    int64_t g = (n + BLK - 1) / BLK;
    if (g > nblk) g = nblk;
    if (g < 1) g = 1;
    gram_cols_k<<<(unsigned)g, BLK, 0, s>>>(X, ldx, nc, b, n, part);
    gram_cols_reduce_k<<<(unsigned)PG_PAIRS, 64, 0, s>>>(part, (int)g, nc, G, ldg, rb, bn2);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_gemv2(const float *X0, int64_t ldx0, int nv0, const double *c0, double beta0,
            const float *a0, double alpha0, int64_t n0, float *out0, const float *X1,
            int64_t ldx1, int nv1, const double *c1, double beta1, const float *a1,
            double alpha1, int64_t n1, float *out1, hipStream_t s)
{
    if (nv0 > MD_MAX || nv1 > MD_MAX) return NLRMM_ESHAPE;
    const unsigned g0 = grid_for(n0), g1 = grid_for(n1);
    gemv2_k<<<g0 + g1, BLK, 0, s>>>(GemvJob{X0, ldx0, nv0, c0, beta0, a0, alpha0, n0, out0},
                                    GemvJob{X1, ldx1, nv1, c1, beta1, a1, alpha1, n1, out1}, g0);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_gemv_norm_normalize(const float *X, int64_t ldx, int nv, const double *c, float *r,
                          int64_t n, double *part, int nblk, double *scal, double tol,
                          float *vout, int *status, hipStream_t s)
{
    if (nv > MD_MAX) return NLRMM_ESHAPE;
    int64_t g = grid_for(n);
    if (g > nblk) g = nblk;
    gemv_norm_k<<<(unsigned)g, BLK, 0, s>>>(X, ldx, nv, c, r, n, r, part);
    normalize_red_k<<<(unsigned)((n + BLK - 1) / BLK), BLK, 0, s>>>(r, part, (int)g, scal, tol, n,
                                                                    vout, status);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_gemv(const float *X, int64_t ldx, int nv, const double *c, double beta, const float *a,
           double alpha, int64_t n, float *out, hipStream_t s)
{
    if (nv > MD_MAX) return NLRMM_ESHAPE;
    gemv_k<<<grid_for(n), BLK, 0, s>>>(X, ldx, nv, c, beta, a, alpha, n, out);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_block_update(const float *X, int64_t ldx, int nin, const double *T, int ldt, int kout,
                   int64_t n, float *Y, int64_t ldy, hipStream_t s, int precision)
{
    if (nin > MD_MAX || kout > 16) return NLRMM_ESHAPE;
    if (precision == 2) {
        const int64_t per = 32 * (BLK / 64);
        block_update_bf16_k<<<(unsigned)((n + per - 1) / per), BLK, 0, s>>>(X, ldx, nin, T, ldt,
                                                                           kout, n, Y, ldy);
        return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
    }
    block_update_k<<<grid_for(n), BLK, 0, s>>>(X, ldx, nin, T, ldt, kout, n, Y, ldy);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_copy_cols(const float *src, int64_t lds, float *dst, int64_t ldd, int ncols, int64_t n,
                hipStream_t s)
{
    const int64_t t = n * ncols;
    copy_cols_k<<<(unsigned)((t + 255) / 256), 256, 0, s>>>(src, lds, dst, ldd, ncols, n);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_normalize_into(const float *r, const double *scal, double tol, int64_t n, float *vout,
                     int *status, double *norm_out, hipStream_t s)
{
    normalize_into_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(r, scal, tol, n, vout, status,
                                                                 norm_out);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_gks_solve(const double *GA, const double *GP, int ldg, const double *rb, const double *scal,
                int ell, double lam_fix, double *z, double *out, int *status, hipStream_t s,
                int method, double *Lst, int linc)
{
    if (ell < 1 || ell > SOLVE_MAX) return NLRMM_ESHAPE;
    if ((Lst != nullptr || linc) && method != 1) return NLRMM_EINVAL;
    if (method == 1) {
        const int nb = (ell + 8) / 8 * 8;   // padded size >= ell + 1
        switch (nb) {
#define NLRMM_REG_CASE(NB)                                                                        \
    case NB:                                                                                      \
        return reg::launch_gks_solve_reg<NB>(GA, GP, ldg, rb, scal, ell, lam_fix, z, out, status, \
                                             s, Lst, linc);
            NLRMM_REG_CASE(8)
            NLRMM_REG_CASE(16)
            NLRMM_REG_CASE(24)
            NLRMM_REG_CASE(32)
            NLRMM_REG_CASE(40)
            NLRMM_REG_CASE(48)
            NLRMM_REG_CASE(56)
#undef NLRMM_REG_CASE
        default: return NLRMM_ESHAPE;
        }
    }
    if (method == 2) {
        const size_t sh = sizeof(double) * ((size_t)(ell + 1) * (ell + 2) + (size_t)ell * (ell + 1) +
                                            7 * (size_t)ell);
        gks_solve_tri_k<<<1, TRI_NT, sh, s>>>(GA, GP, ldg, rb, scal, ell, lam_fix, z, out, status);
        return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
    }
    const size_t sh = sizeof(double) * (2 * (size_t)ell * (ell + 1) + 4 * ell + 128);
    gks_solve_k<<<1, SOLVE_NT, sh, s>>>(GA, GP, ldg, rb, scal, ell, lam_fix, z, out, status);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_compress_eig(const double *GA, const double *GP, int ldg, const double *lam, int ell,
                   int kmin, const double *z, double *T, int ldt, double *zout, int *kout,
                   int *status, hipStream_t s, int method)
{
    if (ell < 1 || ell > SOLVE_MAX || kmin < 2 || kmin > 16 || kmin > ell) return NLRMM_ESHAPE;
    if (method == 1) {
        const int nb = (ell + 8) / 8 * 8;
        switch (nb) {
#define NLRMM_CMP_CASE(NB)                                                                     \
    case NB:                                                                                   \
        return reg::launch_compress_reg<NB>(GA, GP, ldg, lam, ell, kmin, z, T, ldt, zout, kout, \
                                            status, s);
            NLRMM_CMP_CASE(8)
            NLRMM_CMP_CASE(16)
            NLRMM_CMP_CASE(24)
            NLRMM_CMP_CASE(32)
            NLRMM_CMP_CASE(40)
            NLRMM_CMP_CASE(48)
            NLRMM_CMP_CASE(56)
#undef NLRMM_CMP_CASE
        default: return NLRMM_ESHAPE;
        }
    }
    const size_t sh = sizeof(double) * (2 * (size_t)ell * (ell + 1) + 128 + 2 * ell + kmin);
    compress_eig_k<<<1, SOLVE_NT, sh, s>>>(GA, GP, ldg, lam, ell, kmin, z, T, ldt, zout, kout, status);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

int k_gram_transform(double *G, int ldg, double *rb, int ell, const double *T, int ldt,
                     const int *kp, hipStream_t s)
{
    const size_t sh = sizeof(double) * ((size_t)ell * 16 + 16);
    gram_transform_k<<<1, BLK, sh, s>>>(G, ldg, rb, ell, T, ldt, kp);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

}  // namespace nlrmm
