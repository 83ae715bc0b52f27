// Fan-beam strip-area projector family for gfx950: projection, exact transpose, per-view
// angle derivative and its transpose for the CT geometry of Section 6.2 (a point source
// at distance R from the rotation centre; the geometry's own distances are not stated in
// the paper, this is the library's model).
//
// Geometry: view theta has n = (cos, sin), t = (-sin, cos), the source at S = -R t and the
// detector on the line through the centre along n; the ray of detector coordinate s runs
// from S through the point s n.  Near a pixel centre c the rays are taken as parallel along
// the ray through c, direction t(alpha) with alpha = theta - gamma, tan gamma = (c.n) / b,
// b = R + c.t.  That ray meets the detector line at s_c = R (c.n) / b, and a shift w across
// the rays at c moves s by m w with m = R l / b^2, l = |c - S|.  The weight is the parallel
// strip weight of the pixel for direction alpha, centred at s_c and scaled by m:
//   a[v][j][pix] = (m / ds) (Phi_alpha((e_{j+1} - s_c) / m) - Phi_alpha((e_j - s_c) / m)),
// exact to first order in the pixel size and the strip-area model as R grows.  With the
// odd part psi of Phi_alpha / h (the even part cancels between the two edges):
//   a = (m h / ds) (psi(v_{j+1}) - psi(v_j)),  v_e = (e b - R (c.n)) / (b m).
// The angle derivative of F(e) = m Phi_alpha(v_e) is
//   dF = m' Phi_alpha(v) - L(v) (s_c' + v m') - m alpha' L(v) mu(v),
// L the chord length at footprint offset v, mu its midpoint along t(alpha), with
//   s_c' = R (c.t b + (c.n)^2) / b^2,  alpha' = 1 - (c.t b + (c.n)^2) / l^2,
//   m' = R (c.n) (2 l^2 - R b) / (l b^3),
// and d a / d theta = (dF(e_{j+1}) - dF(e_j)) / ds.
//
// Precision: c.n, c.t, b, c - S and the numerators e b - R (c.n) are FP64 (the footprint
// offsets are small differences of detector-sized numbers, and the local direction is read
// off c - S, so that its sine and cosine keep their relative precision near the image axes);
// the magnification, footprint shape and Phi are FP32.  The derivative positions each edge
// inside the footprint in FP64 (its chord length is steep in narrow ramps), forms the chord
// terms in FP32 and combines their differences between a bin's edges.  Sums over pixels or
// views accumulate in FP64.
//
// Projection (bin-driven gather): four lanes per (column, view, group of four bins), each
// walking every fourth line.  The group's rays are walked line by line through the image
// (rows when their central ray is closer to the y axis, columns otherwise); on every line the
// pixels whose footprint can reach the group lie within a short window around the crossings
// of its two outer edge rays (the perspective projection is monotone along a line that the
// rays cross at under 45 degrees); each candidate's local parameters serve the group's five
// edges.  The lanes' sums meet in a fixed butterfly.  No atomics; deterministic.
//
// Transpose (pixel-driven gather): one lane per pixel of an 8x8 tile, four waves per block
// splitting the frame's views; per view a pixel forms its local parameters once, walks the
// edges inside its magnified footprint and gathers the bins; the four partial sums meet in
// LDS in a fixed order.  Same weight function as the projection: the two are transposes up
// to FP32 rounding.
#include "internal.h"

#include <math.h>

namespace nlrmm {
namespace {

constexpr int FAN_FWD_BLK = 256;   // projection lanes per block
constexpr int FAN_TILE = 8;        // transpose: 8x8 pixels per block
constexpr int FAN_WAVES = 4;       // transpose: waves per block splitting the views
constexpr int FAN_VCH = 64;        // transpose: views whose trig is staged per chunk

struct FanArgs {
    int nx, ny, nb, nframes, ncols;
    int64_t nviews;
    double x0, y0, d, s0, ds, R;
    const int64_t *view_off;
    const double *theta;
    const float *src;   // image (projection) or sinogram (transpose)
    float *dst;
};

// Local parameters of one pixel in one view.
struct FanLocal {
    double b, rcn;        // R + c.t and R (c.n): v_e = (e b - rcn) * inv_bm
    float inv_bm;         // 1 / (b m)
    float wo, wi, fk;     // odd part of the footprint of the local ray direction
    float scale;          // m h / ds
};

// Extra terms of the angle derivative.  Where a bin edge falls inside a narrow ramp of the
// footprint (local directions near an image axis: ramp width d |sin alpha|), the chord length
// rises with slope 1 / (|cos alpha| |sin alpha|), so the footprint's half-width, ramp width and
// the edge's offset are positioned in FP64 there.
struct FanDeriv {
    float m, h, mp, scp, ap;        // m, h, m', s_c', alpha'
    float rho, inv_ab, Kr, tq, kp, kappa;   // chord constants of direction alpha
    double wod, rhod, inv_bmd;      // FP64 half-width, ramp width and 1 / (b m)
};

__device__ __forceinline__ double fan_edge(double s0, double ds, int64_t j)
{
    return __dadd_rn(s0, __dmul_rn((double)j, ds));
}
__device__ __forceinline__ double fan_pix(double o, double d, int k)
{
    return __dadd_rn(o, __dmul_rn((double)k + 0.5, d));
}

__device__ __forceinline__ int fan_frame(const int64_t *vo, int F, int64_t v)
{
    if (F <= 1 || vo == nullptr) return 0;
    int lo = 0, hi = F - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vo[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Odd part of Phi / h: c1 the offset clamped to [-wo, wo], q its part beyond the plateau
// [-wi, wi], psi = c1 - q |q| / (2 rho); +-(wi + rho / 2) outside the footprint.
__device__ __forceinline__ float fan_psi(float v, float wo, float wi, float fk)
{
    const float c1 = __builtin_amdgcn_fmed3f(v, -wo, wo);
    const float q = c1 - __builtin_amdgcn_fmed3f(v, -wi, wi);
    return fmaf(-fk, q * fabsf(q), c1);
}

template <bool DERIV>
__device__ __forceinline__ void fan_local(double xc, double yc, double cs, double sn, double R,
                                          float d, float inv_ds, FanLocal &f, FanDeriv &g)
{
    const double cn = fma(xc, cs, yc * sn);
    const double ct = fma(-xc, sn, yc * cs);
    f.b = R + ct;
    f.rcn = R * cn;
    const float bf = (float)f.b, cnf = (float)cn, Rf = (float)R;
    // the local ray direction t(alpha) = (c - S) / l, formed from the FP64 components of
    // c - S = (x - R sin, y + R cos): no cancellation when alpha is near an image axis
    const float uxf = (float)(xc - R * sn), uyf = (float)(yc + R * cs);
    const float l2 = fmaf(uxf, uxf, uyf * uyf);
    const float l = sqrtf(l2);
    const float il = 1.0f / l;
    const float ca = uyf * il;    // cos alpha
    const float sa = -uxf * il;   // sin alpha
    const float aa = fabsf(ca), ab = fabsf(sa);
    const float p = d * aa, r = d * ab;
    const float rho = fminf(p, r);
    f.wo = 0.5f * (p + r);
    f.wi = 0.5f * fabsf(p - r);
    f.fk = rho > 1e-30f ? 0.5f / rho : 0.0f;
    const float h = d / fmaxf(aa, ab);
    const float m = Rf * l / (bf * bf);
    f.inv_bm = bf / (Rf * l);
    f.scale = m * h * inv_ds;
    if (DERIV) {
        const double uxd = xc - R * sn, uyd = yc + R * cs;
        const double ild = 1.0 / sqrt(fma(uxd, uxd, uyd * uyd));
        const double aad = fabs(uyd * ild), abd = fabs(uxd * ild);
        const double dd = (double)d;
        g.wod = 0.5 * dd * (aad + abd);
        g.rhod = dd * fmin(aad, abd);
        g.inv_bmd = f.b * ild / R;
        const float k1 = fmaf((float)ct, bf, cnf * cnf);   // c.t b + (c.n)^2
        g.m = m;
        g.h = h;
        g.scp = Rf * k1 / (bf * bf);
        g.ap = 1.0f - k1 / l2;
        g.mp = Rf * cnf * fmaf(2.0f, l2, -Rf * bf) / (l * bf * bf * bf);
        g.rho = (float)g.rhod;
        const float abp = fmaxf(aa * ab, 1e-30f);
        g.inv_ab = 1.0f / abp;
        g.Kr = (ab * ab - aa * aa) * 0.5f * g.inv_ab;
        g.tq = 0.5f * d * (aa - ab);
        g.kappa = (ca * sa >= 0.0f) ? 1.0f : -1.0f;
        g.kp = aa >= ab ? -g.kappa * ab / aa : g.kappa * aa / ab;
    }
}

// Footprint offset of detector coordinate e.
__device__ __forceinline__ float fan_off(const FanLocal &f, double e)
{
    return (float)fma(e, f.b, -f.rcn) * f.inv_bm;
}

// Terms of the angle derivative of m Phi_alpha(v) at footprint offset v: the odd part psi of
// Phi / h, the chord length L, L v and the chord's first moment L mu along t(alpha).  A bin's
// derivative weight combines the differences of these terms between its two edges,
//   (m' h dpsi - s_c' dL - m' d(L v) - m alpha' d(L mu)) / ds,
// so that no detector-sized product is formed before the difference is taken.
struct FanEdge {
    float ps, L, Lv, Lmu;
};

// Terms at detector coordinate e: the offset and its distance inside the footprint's end
// in FP64, the rest in FP32.
__device__ __forceinline__ FanEdge fan_edge_terms(double e, const FanLocal &f, const FanDeriv &g)
{
    const double vd = fma(e, f.b, -f.rcn) * g.inv_bmd;
    const float v = (float)vd;
    const double dld = g.wod - fabs(vd);
    const float dl = (float)fmax(dld, 0.0);
    const float dr = fminf(dl, g.rho);
    const float sgn = v >= 0.0f ? 1.0f : -1.0f;
    const float mu = (dld >= g.rhod) ? v * g.kp : sgn * g.kappa * fmaf(dr, g.Kr, g.tq);
    FanEdge t;
    t.L = fminf(dl * g.inv_ab, g.h);
    t.Lv = t.L * v;
    t.Lmu = t.L * mu;
    t.ps = fan_psi(v, f.wo, f.wi, f.fk);
    return t;
}

__device__ __forceinline__ float fan_dweight(const FanEdge &e1, const FanEdge &e0,
                                             const FanDeriv &g)
{
    const float t = fmaf(g.mp * g.h, e1.ps - e0.ps, -g.scp * (e1.L - e0.L));
    return fmaf(-g.mp, e1.Lv - e0.Lv, fmaf(-g.m * g.ap, e1.Lmu - e0.Lmu, t));
}

// ---------------------------------------------------------------------------
// projection and its angle derivative: four lanes per (column, view, group of four bins)
// ---------------------------------------------------------------------------
constexpr int FAN_G = 4;   // bins per group: the candidates' local parameters serve all four
constexpr int FAN_Q = 4;   // lanes per group, each walking every fourth line

template <bool DERIV>
__global__ __launch_bounds__(FAN_FWD_BLK) void fan_fwd_k(FanArgs a)
{
    const int64_t gid = (int64_t)blockIdx.x * FAN_FWD_BLK + threadIdx.x;
    const int q = (int)(gid & (FAN_Q - 1));
    const int ngroups = (a.nb + FAN_G - 1) / FAN_G;
    const int64_t per_col = a.nviews * ngroups;
    // lanes past the last group work on group 0 and write nothing: every lane of the wave
    // takes part in the closing shuffles
    const int64_t grp_raw = gid / FAN_Q;
    const bool valid = grp_raw < per_col * a.ncols;
    const int64_t grp = valid ? grp_raw : 0;
    const int col = (int)(grp / per_col);
    const int64_t rem = grp - (int64_t)col * per_col;
    const int64_t v = rem / ngroups;
    const int j0 = (int)(rem - v * ngroups) * FAN_G;
    const int nj = min(FAN_G, a.nb - j0);     // bins of this group on the detector
    const int f = fan_frame(a.view_off, a.nframes, v);
    const float *x = a.src + ((int64_t)col * a.nframes + f) * a.nx * a.ny;
    double sn, cs;
    sincos(a.theta[v], &sn, &cs);
    const double R = a.R;
    const float d = (float)a.d;
    const float inv_ds = (float)(1.0 / a.ds);
    double e[FAN_G + 1];
#pragma unroll
    for (int i = 0; i <= FAN_G; ++i) e[i] = fan_edge(a.s0, a.ds, j0 + i);
    const double ea = e[0], eb = fan_edge(a.s0, a.ds, j0 + nj);
    // ray of detector coordinate s: direction u = s n + R t
    const double em = 0.5 * (ea + eb);
    const double uxm = em * cs - R * sn, uym = fma(em, sn, R * cs);
    const bool rows = fabs(uym) >= fabs(uxm);
    const double uxa = ea * cs - R * sn, uya = fma(ea, sn, R * cs);
    const double uxb = eb * cs - R * sn, uyb = fma(eb, sn, R * cs);
    // along the walked line: the crossing of an edge ray moves by k per unit across lines
    const double ka = rows ? uxa / uya : uya / uxa;
    const double kb = rows ? uxb / uyb : uyb / uxb;
    const double slope = fmax(fabs(ka), fabs(kb));
    // a pixel's footprint spans (d/2)(1 + |slope of its own ray|) along the line; the window
    // adds a tenth of it and a twentieth of a pixel for the curvature of the projection
    const double reach = a.d * (0.6 + 0.6 * slope + 0.05);
    const double Sx = R * sn, Sy = -R * cs;
    const int nlines = rows ? a.ny : a.nx;
    const int nalong = rows ? a.nx : a.ny;
    const double o_line = rows ? a.y0 : a.x0, o_along = rows ? a.x0 : a.y0;
    const double S_line = rows ? Sy : Sx, S_along = rows ? Sx : Sy;
    const double inv_d = 1.0 / a.d;
    FanLocal lc;
    FanDeriv dg;
    double acc[FAN_G];
#pragma unroll
    for (int i = 0; i < FAN_G; ++i) acc[i] = 0.0;
    for (int li = q; li < nlines; li += FAN_Q) {
        const double pl = fan_pix(o_line, a.d, li);
        const double xa = fma(pl - S_line, ka, S_along), xb = fma(pl - S_line, kb, S_along);
        const double lo = fmin(xa, xb) - reach, hi = fmax(xa, xb) + reach;
        // along-line indices with centres in [lo, hi]
        const double tlo = (lo - o_along) * inv_d - 0.5, thi = (hi - o_along) * inv_d - 0.5;
        if (!(thi >= 0.0 && tlo <= (double)(nalong - 1))) continue;   // also NaN
        const int klo = (int)ceil(fmax(tlo, 0.0));
        const int khi = (int)floor(fmin(thi, (double)(nalong - 1)));
        for (int kk = klo; kk <= khi; ++kk) {
            const int kx = rows ? kk : li, ly = rows ? li : kk;
            const float xv = x[(int64_t)ly * a.nx + kx];
            if (xv == 0.0f) continue;
            const double pa = fan_pix(o_along, a.d, kk);
            const double xc = rows ? pa : pl, yc = rows ? pl : pa;
            fan_local<DERIV>(xc, yc, cs, sn, R, d, inv_ds, lc, dg);
            const double xd = (double)xv;
            if (DERIV) {
                FanEdge tp = fan_edge_terms(e[0], lc, dg);
#pragma unroll
                for (int i = 0; i < FAN_G; ++i) {
                    const FanEdge tn = fan_edge_terms(e[i + 1], lc, dg);
                    acc[i] = fma(xd, (double)(fan_dweight(tn, tp, dg) * inv_ds), acc[i]);
                    tp = tn;
                }
            } else {
                float pp = fan_psi(fan_off(lc, e[0]), lc.wo, lc.wi, lc.fk);
#pragma unroll
                for (int i = 0; i < FAN_G; ++i) {
                    const float pn = fan_psi(fan_off(lc, e[i + 1]), lc.wo, lc.wi, lc.fk);
                    acc[i] = fma(xd, (double)(lc.scale * (pn - pp)), acc[i]);
                    pp = pn;
                }
            }
        }
    }
    // the four lanes' partial sums: a butterfly (commutative additions, the same bits in
    // every lane of the group), then lane q writes bin j0 + q
    double out = 0.0;
#pragma unroll
    for (int i = 0; i < FAN_G; ++i) {
        double t = acc[i];
        t += __shfl_xor(t, 1, 64);
        t += __shfl_xor(t, 2, 64);
        if (i == q) out = t;
    }
    if (valid && q < nj) a.dst[((int64_t)col * a.nviews + v) * a.nb + j0 + q] = (float)out;
}

// ---------------------------------------------------------------------------
// transpose and derivative transpose: one lane per pixel, views split over four waves
// ---------------------------------------------------------------------------
template <bool DERIV>
__global__ __launch_bounds__(FAN_TILE * FAN_TILE * FAN_WAVES) void fan_bwd_k(FanArgs a)
{
    __shared__ double trig[2][FAN_VCH];
    __shared__ double red[FAN_WAVES - 1][FAN_TILE * FAN_TILE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_x = (a.nx + FAN_TILE - 1) / FAN_TILE;
    const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
    const int kx = tx * FAN_TILE + (lane & (FAN_TILE - 1));
    const int ly = ty * FAN_TILE + (lane >> 3);
    const int cf = blockIdx.y;                  // column * nframes + frame
    const int f = cf % a.nframes;
    const int col = cf / a.nframes;
    const bool inside = kx < a.nx && ly < a.ny;
    const double xc = fan_pix(a.x0, a.d, min(kx, a.nx - 1));
    const double yc = fan_pix(a.y0, a.d, min(ly, a.ny - 1));
    const int64_t v_begin = (a.nframes > 1) ? a.view_off[f] : 0;
    const int64_t v_end = (a.nframes > 1) ? a.view_off[f + 1] : a.nviews;
    const float *y = a.src + (int64_t)col * a.nviews * a.nb;
    const double R = a.R;
    const float d = (float)a.d;
    const float inv_ds = (float)(1.0 / a.ds);
    const double inv_dsd = 1.0 / a.ds;
    FanLocal lc;
    FanDeriv dg;
    double acc = 0.0;
    for (int64_t c0 = v_begin; c0 < v_end; c0 += FAN_VCH) {
        const int nc = (int)min((int64_t)FAN_VCH, v_end - c0);
        __syncthreads();
        if (threadIdx.x < nc) {
            double sn, cs;
            sincos(a.theta[c0 + threadIdx.x], &sn, &cs);
            trig[0][threadIdx.x] = cs;
            trig[1][threadIdx.x] = sn;
        }
        __syncthreads();
        for (int i = wave; i < nc; i += FAN_WAVES) {
            const double cs = trig[0][i], sn = trig[1][i];
            fan_local<DERIV>(xc, yc, cs, sn, R, d, inv_ds, lc, dg);
            // bins met by the magnified footprint [s_c - m wo, s_c + m wo] (a superset: bins
            // beyond it weigh exactly 0); s_c = rcn / b by an FP32 quotient and one FP64
            // correction step
            const float ib = 1.0f / (float)lc.b;
            double sc = (double)((float)lc.rcn * ib);
            sc = fma(fma(-sc, lc.b, lc.rcn), (double)ib, sc);
            const double tc = (sc - a.s0) * inv_dsd;
            const double half = (double)(lc.wo * ib / lc.inv_bm) * inv_dsd + 1e-3;
            const int jlo = (int)fmin(fmax(floor(tc - half), 0.0), (double)a.nb);
            const int jhi = (int)fmin(fmax(floor(tc + half), -1.0), (double)(a.nb - 1));
            const float *yv = y + (c0 + i) * a.nb;
            float sv = 0.0f;
            if (DERIV) {
                FanEdge ep = fan_edge_terms(fan_edge(a.s0, a.ds, jlo), lc, dg);
                for (int j = jlo; j <= jhi; ++j) {
                    const FanEdge en = fan_edge_terms(fan_edge(a.s0, a.ds, j + 1), lc, dg);
                    sv = fmaf(yv[j], fan_dweight(en, ep, dg), sv);
                    ep = en;
                }
                sv *= inv_ds;
            } else {
                float fprev = fan_psi(fan_off(lc, fan_edge(a.s0, a.ds, jlo)), lc.wo, lc.wi,
                                      lc.fk);
                for (int j = jlo; j <= jhi; ++j) {
                    const float fn = fan_psi(fan_off(lc, fan_edge(a.s0, a.ds, j + 1)), lc.wo,
                                             lc.wi, lc.fk);
                    sv = fmaf(yv[j], fn - fprev, sv);
                    fprev = fn;
                }
                sv *= lc.scale;
            }
            acc += (double)sv;
        }
    }
    // the four waves' partial sums, added in wave order
    if (wave > 0) red[wave - 1][lane] = acc;
    __syncthreads();
    if (wave == 0 && inside) {
        for (int w = 0; w < FAN_WAVES - 1; ++w) acc += red[w][lane];
        a.dst[((int64_t)col * a.nframes + f) * a.nx * a.ny + (int64_t)ly * a.nx + kx] =
            (float)acc;
    }
}

FanArgs fan_args(const nlrmm_geom &g, const nlrmm_batch &b, int ncols, double R,
                 const double *theta, const float *src, float *dst)
{
    FanArgs a;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nb = g.nbins;
    a.nframes = b.nframes;
    a.ncols = ncols;
    a.nviews = b.nviews;
    a.x0 = g.x0;
    a.y0 = g.y0;
    a.d = g.d;
    a.s0 = g.s0;
    a.ds = g.ds;
    a.R = R;
    a.view_off = b.view_off;
    a.theta = theta;
    a.src = src;
    a.dst = dst;
    return a;
}

}  // namespace

double fan_min_distance(const nlrmm_geom &g)
{
    const double xs[2] = {g.x0, g.x0 + g.nx * g.d};
    const double ys[2] = {g.y0, g.y0 + g.ny * g.d};
    double r2 = 0.0;
    for (double xv : xs)
        for (double yv : ys) r2 = fmax(r2, xv * xv + yv * yv);
    return 1.5 * sqrt(r2);
}

int launch_fan(const nlrmm_geom &g, const nlrmm_batch &b, int ncols, double R, int deriv,
               int transpose, const double *theta, const float *src, float *dst, hipStream_t s)
{
    const FanArgs a = fan_args(g, b, ncols, R, theta, src, dst);
    if (!transpose) {
        const int64_t ngroups = (g.nbins + FAN_G - 1) / FAN_G;
        const int64_t n = (int64_t)ncols * b.nviews * ngroups * FAN_Q;
        const unsigned blocks = (unsigned)((n + FAN_FWD_BLK - 1) / FAN_FWD_BLK);
        if (deriv)
            fan_fwd_k<true><<<blocks, FAN_FWD_BLK, 0, s>>>(a);
        else
            fan_fwd_k<false><<<blocks, FAN_FWD_BLK, 0, s>>>(a);
    } else {
        const int tiles = ((g.nx + FAN_TILE - 1) / FAN_TILE) * ((g.ny + FAN_TILE - 1) / FAN_TILE);
        dim3 grid((unsigned)tiles, (unsigned)(ncols * b.nframes));
        if (deriv)
            fan_bwd_k<true><<<grid, FAN_TILE * FAN_TILE * FAN_WAVES, 0, s>>>(a);
        else
            fan_bwd_k<false><<<grid, FAN_TILE * FAN_TILE * FAN_WAVES, 0, s>>>(a);
    }
    NLRMM_HIP_CHECK(hipGetLastError());
    return NLRMM_OK;
}

}  // namespace nlrmm
