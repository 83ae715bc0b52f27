// Photoacoustic circular-means operator with a global radial shift on gfx950 (Section 6.3,
// "Photoacoustic Tomography with Sensor Radius Uncertainty": circles of radii r_j(p) = r_j + p
// around every sensor).  The paper leaves the operator to its toolbox; this is the library's
// model:
//   * n_a sensors at angles 2 pi a / n_a on the circle of radius rho around the origin;
//   * radii r_j(p) = (j + 1) dr + p, j = 0 .. n_c - 1 (dr = 2 / n_c gives r_j = 2 j / n_c);
//   * between pixel centres the image is its bilinear interpolant, 0 for indices outside the
//     grid; a circle integral is the K-point trapezoid rule,
//       y[a][j] = (2 pi r / K) sum_k I(s_a + r e_k),  e_k = (cos, sin)(2 pi k / K);
//   * its derivative in p: (2 pi / K) sum_k [I + r grad I . e_k], grad I the gradient of the
//     sample cell's bilinear interpolant.
// Sample positions, cells and bilinear weights are FP64 (the derivative's gradient jumps at
// cell boundaries, so a sample must fall in the same cell as in an FP64 evaluation); pixel
// values FP32; sums FP64.
//
// Projection: one wave per (column, sensor, radius), the K samples split over the lanes, the
// lanes' sums added by a fixed butterfly (a negative r = r_j + p is used as it stands: the
// circle of radius |r| traced from the opposite side, with the negative factor 2 pi r / K).
// Transpose (gather, no atomics): 16, 32 or 64 lanes per pixel (whichever first covers the
// sensors), lane s taking sensors s, s + lpp, ...; for each sensor the radii whose |r| is
// within d sqrt(2) of the pixel's distance and, on each, the samples within asin(d sqrt(2)/|r|)
// of the pixel's direction seen from the sensor; a sample adds its
// value times the bilinear weight of the pixel's corner when the pixel is a corner of its
// cell (the same FP64 directions, from LDS up to 2048 samples per circle, and the same FP64
// cell test as the projection); the lanes' sums are joined by a fixed butterfly.
#include "internal.h"

#include <math.h>

namespace nlrmm {
namespace {

constexpr int PAT_BLK = 256;
constexpr int PAT_KMAX = 8192;       // samples per circle
constexpr int PAT_DIR_CHUNK = 1024;  // directions staged in LDS per pass
constexpr int PAT_BWD_KLDS = 2048;   // transpose: all directions in LDS up to this K

struct PatArgs {
    int nx, ny, ncols, na, nc, K;
    double x0, y0, d, rho, dr, p;
    const float *src;
    float *dst;
};

__device__ __forceinline__ double pat_pix(double o, double d, int k)
{
    return __dadd_rn(o, __dmul_rn((double)k + 0.5, d));
}

// Cell of a point: corner indices and fractions (fractional pixel index = (x - x0) / d - 1/2).
struct PatCell {
    int k0, l0;
    double tx, ty;
};

__device__ __forceinline__ PatCell pat_cell(double x, double y, const PatArgs &a)
{
    const double fx = (x - a.x0) / a.d - 0.5, fy = (y - a.y0) / a.d - 0.5;
    const double ffx = floor(fx), ffy = floor(fy);
    PatCell c;
    // far-away points: any index outside the grid contributes 0 (clamped to stay in int range)
    c.k0 = (int)fmin(fmax(ffx, -4.0), (double)a.nx + 4.0);
    c.l0 = (int)fmin(fmax(ffy, -4.0), (double)a.ny + 4.0);
    c.tx = fx - ffx;
    c.ty = fy - ffy;
    return c;
}

__device__ __forceinline__ double pat_val(const float *__restrict__ x, const PatArgs &a, int k,
                                          int l)
{
    return (k >= 0 && k < a.nx && l >= 0 && l < a.ny) ? (double)x[(int64_t)l * a.nx + k] : 0.0;
}

template <bool DERIV>
__global__ __launch_bounds__(PAT_BLK) void pat_fwd_k(PatArgs a)
{
    __shared__ double2 dirs[PAT_DIR_CHUNK];
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * PAT_BLK + threadIdx.x) >> 6;
    const int64_t ncirc = (int64_t)a.ncols * a.na * a.nc;
    const bool valid = wave < ncirc;
    const int64_t cw = valid ? wave : 0;
    const int col = (int)(cw / ((int64_t)a.na * a.nc));
    const int64_t rem = cw - (int64_t)col * a.na * a.nc;
    const int sa = (int)(rem / a.nc), j = (int)(rem - (int64_t)sa * a.nc);
    double ss, sc;
    sincospi(2.0 * sa / a.na, &ss, &sc);
    const double sx = a.rho * sc, sy = a.rho * ss;
    const double r = (j + 1) * a.dr + a.p;
    const float *x = a.src + (int64_t)col * a.nx * a.ny;
    double acc = 0.0;
    for (int k0 = 0; k0 < a.K; k0 += PAT_DIR_CHUNK) {
        const int n = min(PAT_DIR_CHUNK, a.K - k0);
        __syncthreads();
        for (int t = threadIdx.x; t < n; t += PAT_BLK) {
            double sn, cs;
            sincospi(2.0 * (k0 + t) / a.K, &sn, &cs);
            dirs[t] = make_double2(cs, sn);
        }
        __syncthreads();
        for (int t = lane; t < n; t += 64) {
            const double2 e = dirs[t];
            const PatCell c = pat_cell(fma(r, e.x, sx), fma(r, e.y, sy), a);
            const double v00 = pat_val(x, a, c.k0, c.l0), v10 = pat_val(x, a, c.k0 + 1, c.l0);
            const double v01 = pat_val(x, a, c.k0, c.l0 + 1);
            const double v11 = pat_val(x, a, c.k0 + 1, c.l0 + 1);
            const double I = (1 - c.tx) * (1 - c.ty) * v00 + c.tx * (1 - c.ty) * v10 +
                             (1 - c.tx) * c.ty * v01 + c.tx * c.ty * v11;
            if (DERIV) {
                const double gx = ((1 - c.ty) * (v10 - v00) + c.ty * (v11 - v01)) / a.d;
                const double gy = ((1 - c.tx) * (v01 - v00) + c.tx * (v11 - v10)) / a.d;
                acc += I + r * (gx * e.x + gy * e.y);
            } else {
                acc += I;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (valid && lane == 0) {
        const double scale = DERIV ? 2.0 * M_PI / a.K : 2.0 * M_PI * r / a.K;
        a.dst[cw] = (float)(scale * acc);
    }
}

__global__ __launch_bounds__(PAT_BLK) void pat_bwd_k(PatArgs a)
{
    // the K sample directions of every circle, the same FP64 values as the projection's
    __shared__ double2 dirs[PAT_BWD_KLDS];
    const bool staged = a.K <= PAT_BWD_KLDS;
    if (staged) {
        for (int t = threadIdx.x; t < a.K; t += PAT_BLK) {
            double sn, cs;
            sincospi(2.0 * t / a.K, &sn, &cs);
            dirs[t] = make_double2(cs, sn);
        }
    }
    __syncthreads();
    // lpp lanes per pixel (16, 32 or 64: the first that covers the sensors), 64 / lpp pixels
    // per wave
    const int lpp = a.na <= 16 ? 16 : (a.na <= 32 ? 32 : 64);
    const int lane = threadIdx.x & 63, sl = lane & (lpp - 1);
    const int64_t gid = ((int64_t)blockIdx.x * PAT_BLK + threadIdx.x) / lpp;
    const int64_t npix = (int64_t)a.nx * a.ny;
    const bool live = gid < npix * a.ncols;   // no barrier follows: idle lanes just add 0
    const int64_t gl = live ? gid : 0;
    const int col = (int)(gl / npix);
    const int64_t pix = gl - col * npix;
    const int l = (int)(pix / a.nx), k = (int)(pix - (int64_t)l * a.nx);
    const double xc = pat_pix(a.x0, a.d, k), yc = pat_pix(a.y0, a.d, l);
    const float *y = a.src + (int64_t)col * a.na * a.nc;
    const double reach = a.d * M_SQRT2;
    double acc = 0.0;
    for (int sa = sl; live && sa < a.na; sa += lpp) {
        double ss, sc;
        sincospi(2.0 * sa / a.na, &ss, &sc);
        const double sx = a.rho * sc, sy = a.rho * ss;
        const double dx = xc - sx, dy = yc - sy;
        const double dist = sqrt(dx * dx + dy * dy);
        // radii with ||r| - dist| < d sqrt(2): a sample whose cell has this pixel as a corner
        // lies within d sqrt(2) of the pixel centre (a negative radius r = r_j + p traces the
        // circle of radius |r| from the opposite side)
        const double psi = atan2(dy, dx);   // direction of the pixel seen from the sensor
        for (int side = 0; side < 2; ++side) {
            const double sg = side ? -1.0 : 1.0;
            const double rlo = side ? -dist - reach : dist - reach;
            const double rhi = side ? -dist + reach : dist + reach;
            const double jlo_f = ceil((rlo - a.p) / a.dr - 1.0) - 1.0;
            const double jhi_f = floor((rhi - a.p) / a.dr - 1.0) + 1.0;
            const int jlo = (int)fmax(jlo_f, 0.0), jhi = (int)fmin(jhi_f, (double)(a.nc - 1));
            for (int j = jlo; j <= jhi; ++j) {
                const double r = (j + 1) * a.dr + a.p;
                if (!(sg * r > 0.0)) continue;   // each radius on its own side once
                const double ar = fabs(r);
                // samples within the angle the support subtends: a sample within d sqrt(2) of
                // the pixel is at most asin(d sqrt(2) / |r|) from the pixel's direction, seen
                // from the sensor (one sample of margin)
                const double sarg = reach / ar;
                int kb, kn;
                if (sarg >= 1.0) {
                    kb = 0;
                    kn = a.K;
                } else {
                    const double half = asin(sarg) * a.K / (2.0 * M_PI) + 1.0;
                    const double kc = (side ? psi + M_PI : psi) * a.K / (2.0 * M_PI);
                    kb = (int)floor(kc - half);
                    kn = min(a.K, (int)ceil(kc + half) - kb + 1);
                }
                double sv = 0.0;
                for (int t = 0; t < kn; ++t) {
                    int kk = (kb + t) % a.K;
                    if (kk < 0) kk += a.K;
                    double sn, cs;
                    if (staged) {
                        const double2 e = dirs[kk];
                        cs = e.x;
                        sn = e.y;
                    } else {
                        sincospi(2.0 * kk / a.K, &sn, &cs);
                    }
                    const PatCell c = pat_cell(fma(r, cs, sx), fma(r, sn, sy), a);
                    const int dk = k - c.k0, dl = l - c.l0;
                    if (dk < 0 || dk > 1 || dl < 0 || dl > 1) continue;
                    const double wx = dk ? c.tx : 1.0 - c.tx, wy = dl ? c.ty : 1.0 - c.ty;
                    sv += wx * wy;
                }
                acc += sv * (2.0 * M_PI * r / a.K) * (double)y[(int64_t)sa * a.nc + j];
            }
        }
    }
    // the sensors' sums joined in a fixed order
    for (int off = lpp / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (live && sl == 0) a.dst[gid] = (float)acc;
}

}  // namespace

int pat_check(const nlrmm_geom &g, const nlrmm_pat_geom &pg, int ncols, double p)
{
    if (ncols < 1 || pg.n_sensors < 1 || pg.n_radii < 1 || pg.n_samples < 1) return NLRMM_ESHAPE;
    if (pg.n_samples > PAT_KMAX || pg.n_sensors > 65536 || pg.n_radii > 65536)
        return NLRMM_ESHAPE;
    if ((int64_t)ncols * pg.n_sensors * pg.n_radii > ((int64_t)1 << 26)) return NLRMM_ESHAPE;
    if (!isfinite(pg.sensor_radius) || !(pg.sensor_radius >= 0.0) || !isfinite(p) ||
        !(pg.radius_step > 0.0) || !isfinite(pg.radius_step))
        return NLRMM_EINVAL;
    (void)g;
    return NLRMM_OK;
}

int launch_pat(const nlrmm_geom &g, const nlrmm_pat_geom &pg, int ncols, double p, int mode,
               const float *src, float *dst, hipStream_t s)
{
    PatArgs a;
    a.nx = g.nx;
    a.ny = g.ny;
    a.ncols = ncols;
    a.na = pg.n_sensors;
    a.nc = pg.n_radii;
    a.K = pg.n_samples;
    a.x0 = g.x0;
    a.y0 = g.y0;
    a.d = g.d;
    a.rho = pg.sensor_radius;
    a.dr = pg.radius_step;
    a.p = p;
    a.src = src;
    a.dst = dst;
    if (mode == 2) {
        const int64_t n = (int64_t)ncols * g.nx * g.ny;   // lpp lanes per pixel
        const int lpp = pg.n_sensors <= 16 ? 16 : (pg.n_sensors <= 32 ? 32 : 64);
        const int64_t per = PAT_BLK / lpp;
        pat_bwd_k<<<(unsigned)((n + per - 1) / per), PAT_BLK, 0, s>>>(a);
    } else {
        const int64_t lanes = (int64_t)ncols * a.na * a.nc * 64;
        const unsigned blocks = (unsigned)((lanes + PAT_BLK - 1) / PAT_BLK);
        if (mode == 1)
            pat_fwd_k<true><<<blocks, PAT_BLK, 0, s>>>(a);
        else
            pat_fwd_k<false><<<blocks, PAT_BLK, 0, s>>>(a);
    }
    NLRMM_HIP_CHECK(hipGetLastError());
    return NLRMM_OK;
}

}  // namespace nlrmm
