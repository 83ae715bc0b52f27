// Strip-area parallel-beam projector family for gfx950: forward projection, exact
// adjoint and per-view angle derivative of the forward operator H(p) (Section 1, eq.
// "nonlinear_forward"; the CT operator of Section 6.2 with per-view angles).
//
// Model: a[v][j][pix] = (Phi(e_{j+1} - c) - Phi(e_j - c)) / ds, where c is the pixel
// centre's detector coordinate, e_j = s0 + j ds the bin edges and Phi(t) the area of the
// pixel square on the side {p.n < c + t} (a piecewise quadratic: ramps of width rho at
// both ends of a plateau of height h).  The angle derivative follows from the moving
// strip boundaries: d a / d theta = (M(e_j) - M(e_{j+1})) / ds with M(e) the first
// moment along t = (-sin, cos) of the chord {p in pixel : p.n = e}.
//
// Forward (edge-driven): one lane per detector EDGE e.  The lane accumulates
//   C(e) = area-weighted image mass on the side p.n < e     (projection)
//   Mo(e) = sum over pixels of x * M(e)                      (derivative)
// over the image lines (rows for views closer to the y axis, columns otherwise); on
// each line at most two pixels straddle the edge, the pixels fully on the left enter
// through a per-line FP64 prefix sum.  Bins follow as y_j = (C(e_{j+1}) - C(e_j)) / ds
// and D_j = (Mo(e_j) - Mo(e_{j+1})) / ds.  Every Phi evaluation is shared by the two
// bins that meet at the edge, so each application evaluates Phi ~2 per edge-line
// instead of ~2 per (ray, pixel) nonzero; the even part of Phi (half the pixel area) is
// carried by the line packs, so only its odd part is evaluated.  No atomics; results are
// deterministic.
//
// Forward lanes of one block are 64 consecutive edges; every wave of the block walks the
// union of the 64 edges' line ranges (one pack load of a wave reads neighbouring entries of
// one line), the block's waves split that union (1..8 waves, tuned per shape), four lines
// per step with their loads in flight together, and their partial sums meet in LDS.
//
// Backward (pixel-driven gather): one lane per pixel pair of a 16x16 tile; for chunks of
// views the tile's detector window is staged in LDS, each pixel locates its footprint
// in bin units relative to the tile centre (FP64), evaluates the odd part of Phi at the
// <= E edges inside it (FP32 offsets) and gathers its <= E+1 bins; the even part enters
// through the footprint's two end bins.  Same weight function as the forward; the two are
// transposes up to FP32 rounding of the offsets.  The derivative's transpose
// gathers the chord moments at the same edges the same way.
#include "internal.h"
#include "multidot.h"
#include "tv.h"
#include "wave.h"

#include <math.h>

#include <type_traits>

namespace nlrmm {
namespace {

constexpr int BLK = 256;          // threads per block: four wave64
constexpr int BINS = 63;          // bins produced per forward block (64 edges, one per lane)
constexpr int FSEG_DEFAULT = 4;   // forward: waves per block sharing each edge's lines
constexpr int TILE = 16;          // backward tile side
constexpr int VCHUNK = 32;        // views staged per backward chunk
constexpr int WMAX = 64;          // max staged bins per view (backward)
constexpr int MAX_LINE = 4096;    // max pixels per image line handled by the packer

struct ViewC {
    double cs, sn, wo;
    float fwo, fwi, frho, f2wi, fh;   // Phi constants
    float fk;                         // 1 / (2 rho) (0 when rho = 0): ramps of Phi / h
    float inv_ab, Kr, tq, kp, kappa;        // chord-moment constants
    int steep;                              // |cos| >= |sin|: lines are image rows
};

__device__ __forceinline__ ViewC make_view(double th, double d)
{
    ViewC q;
    double sn, cs;
    sincos(th, &sn, &cs);
    const double a = fabs(cs), b = fabs(sn);
    const double p = d * a, r = d * b;
    const double wo = 0.5 * (p + r), wi = 0.5 * fabs(p - r), rho = fmin(p, r);
    const double h = d / fmax(a, b);
    q.cs = cs;
    q.sn = sn;
    q.wo = wo;
    q.fwo = (float)wo;
    q.fwi = (float)wi;
    q.frho = (float)rho;
    q.f2wi = (float)(2.0 * wi);
    q.fh = (float)h;
    q.fk = rho > 0.0 ? (float)(0.5 / rho) : 0.0f;
    const double ab = fmax(a * b, 1e-30);
    q.inv_ab = (float)(1.0 / ab);
    q.Kr = (float)((b * b - a * a) / (2.0 * ab));
    q.tq = (float)(0.5 * d * (a - b));
    const double kappa = (cs * sn >= 0.0) ? 1.0 : -1.0;
    q.kappa = (float)kappa;
    q.kp = (float)(a >= b ? -kappa * b / a : kappa * a / b);
    q.steep = a >= b;
    return q;
}

// Cumulative footprint Phi(v): the area of the pixel on the side p.n < c + v, a piecewise
// quadratic in v (a left ramp of width rho, a plateau of height h, a right ramp) whose even
// part is the constant d^2 / 2, half the pixel's area.  The forward and backward kernels
// evaluate its odd part psi_h of offsets formed with different (both FP64-positioned)
// arithmetic, so the two operators are transposes of each other up to FP32 rounding of the
// offsets.
// Phi(v) / h - d^2 / (2 h), the odd part of the cumulative footprint: with c1 the offset
// clamped to the footprint [-wo, wo] and q = c1 - clamp(v, -wi, wi) its part beyond the
// plateau, psi = c1 - q |q| / (2 rho) (fk = 1 / (2 rho), 0 when rho = 0).  On the plateau
// psi = v, on a ramp v -+ (|v| - wi)^2 / (2 rho), outside the footprint +-(wi + rho / 2).
__device__ __forceinline__ float psi_h(float v, float wo, float wi, float fk)
{
    const float c1 = __builtin_amdgcn_fmed3f(v, -wo, wo);
    const float q = c1 - __builtin_amdgcn_fmed3f(v, -wi, wi);
    return fmaf(-fk, q * fabsf(q), c1);
}

// Chord through the pixel at offset v from its centre: length L and the local midpoint
// mu of its t-coordinate.  Plateau: mu = v * kp; ramps: the chord cuts a corner whose
// t-coordinate is sign(v) kappa (d/2)(a - b), and the midpoint moves by Kr per unit of
// distance from that corner.
__device__ __forceinline__ void moment_f(float v, const ViewC &q, float &L, float &mu)
{
    const float av = fabsf(v);
    const float dl = fmaxf(q.fwo - av, 0.0f);
    L = fminf(dl * q.inv_ab, q.fh);
    const float dr = fminf(dl, q.frho);
    const float sg = v >= 0.0f ? 1.0f : -1.0f;
    const float mur = sg * q.kappa * fmaf(dr, q.Kr, q.tq);
    const float mup = v * q.kp;
    mu = (av <= q.fwi) ? mup : mur;
}

__device__ __forceinline__ int frame_of(const int64_t *vo, int F, int64_t v)
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

// e - lc*sl - mc*sm with a fixed rounding sequence (shared by forward and backward).
__device__ __forceinline__ double edge_coord(double s0, double ds, int64_t j)
{
    return __dadd_rn(s0, __dmul_rn((double)j, ds));
}
__device__ __forceinline__ double pix_coord(double o, double d, int k)
{
    return __dadd_rn(o, __dmul_rn((double)k + 0.5, d));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// preparation: per-line packs of rows and columns
// ---------------------------------------------------------------------------
// One block per (image, line), rows (blockIdx.x < ny) and columns (the rest) of the image
// in one launch: entries i = -2..n of the line, stored at i + 2: a = x_i, b = x_{i+1} (zero
// outside the line) and P = the sum of pixels 0..i-1 plus (a + b) / 2 (FP64: the prefix up to
// the middle of the pair, which carries the even part d^2 / 2 of the pair's footprint areas,
// so that the walk needs only the odd part psi_h); tot = the line's sum.  The mirrored
// pack holds the same entries for the reversed line (pixel i of it is pixel n-1-i), so a
// walk against the pixel order reads its prefix directly.
// Normalisation applied while packing (see FwdOptions): src / sqrt(sum of part), written to
// out by the row blocks.
struct NormJob {
    const float *src;
    const double *part;
    int nblk;
    double *scal;
    double tol;
    float *out;
    int *status;
};

__global__ __launch_bounds__(BLK) void pack_lines_k(const float *__restrict__ x, int nx, int ny,
                                                    PackEntry *__restrict__ rowpack,
                                                    PackEntry *__restrict__ colpack,
                                                    PackEntry *__restrict__ rowpack_m,
                                                    PackEntry *__restrict__ colpack_m,
                                                    double *__restrict__ rowtot,
                                                    double *__restrict__ coltot, NormJob nj)
{
    __shared__ float sx[MAX_LINE + 2];
    __shared__ double sP[MAX_LINE + 1];
    __shared__ double swave[BLK / 64];
    __shared__ double sinv;
    const bool is_row = (int)blockIdx.x < ny;
    const int64_t line = is_row ? blockIdx.x : blockIdx.x - ny;
    const int n = is_row ? nx : ny;
    const int nlines = is_row ? ny : nx;
    const int64_t img = blockIdx.y;
    const bool norm = nj.part != nullptr;
    const float *src = (norm ? nj.src : x) + img * (int64_t)nx * ny;
    const int64_t step = is_row ? 1 : nx;
    const float *row = src + (is_row ? line * nx : line);
    PackEntry *pack = is_row ? rowpack : colpack;
    double *tot = is_row ? rowtot : coltot;
    const int tid = threadIdx.x;
    if (norm) {
        // the squared norm as the Krylov normalisation sums it (lane-strided partials, then
        // the butterfly), its breakdown test once
        if (tid < 64) {
            double t = md::strided_sum(nj.part, 1, nj.nblk, tid, 64);
            t = wave_sum(t);
            const double raw = sqrt(fmax(nj.scal[0], 0.0));
            const double perp = sqrt(fmax(t, 0.0));
            if (tid == 0) {
                sinv = perp > 0.0 ? 1.0 / perp : 0.0;
                if (blockIdx.x == 0 && blockIdx.y == 0) {
                    nj.scal[1] = t;
                    if (!(perp > nj.tol * raw)) atomicOr(nj.status, NLRMM_ST_BREAKDOWN);
                    if (!isfinite(perp)) atomicOr(nj.status, NLRMM_ST_NONFINITE);
                }
            }
        }
        __syncthreads();
        const double inv = sinv;
        float *orow = nj.out + img * (int64_t)nx * ny + line * nx;
        for (int i = tid; i < n; i += BLK) {
            const float v = (float)((double)row[i * step] * inv);
            sx[i] = v;
            if (is_row) orow[i] = v;
        }
    } else {
        for (int i = tid; i < n; i += BLK) sx[i] = row[i * step];
    }
    if (tid < 2) sx[n + tid] = 0.0f;
    __syncthreads();
    const int cpt = (n + BLK - 1) / BLK;
    const int i0 = min(tid * cpt, n), i1 = min(i0 + cpt, n);
    double ls = 0.0;
    for (int i = i0; i < i1; ++i) ls += (double)sx[i];
    // block exclusive scan of ls
    const int lane = tid & 63, wv = tid >> 6;
    double incl = ls;
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) swave[wv] = incl;
    __syncthreads();
    double base = 0.0;
    for (int w = 0; w < wv; ++w) base += swave[w];
    double run = base + incl - ls;
    for (int i = i0; i < i1; ++i) {
        sP[i] = run;
        run += (double)sx[i];
    }
    if (tid == BLK - 1) sP[n] = run;   // the last thread's chunk ends the line
    __syncthreads();
    const int64_t lofs = (img * nlines + line) * (int64_t)(n + 3);
    PackEntry *out = pack + lofs;
    PackEntry *outm = (is_row ? rowpack_m : colpack_m) + lofs;
    for (int e = tid; e < n + 3; e += BLK) {
        const int i = e - 2;
        PackEntry pe, pm;
        pe.a = (i >= 0 && i < n) ? sx[i] : 0.0f;
        pe.b = (i + 1 >= 0 && i + 1 < n) ? sx[i + 1] : 0.0f;
        pe.P = ((i > 0) ? sP[i] : 0.0) + 0.5 * ((double)pe.a + (double)pe.b);
        pm.a = (i >= 0 && i < n) ? sx[n - 1 - i] : 0.0f;
        pm.b = (i + 1 >= 0 && i + 1 < n) ? sx[n - 2 - i] : 0.0f;
        pm.P = ((i > 0) ? sP[n] - sP[n - i] : 0.0) + 0.5 * ((double)pm.a + (double)pm.b);
        out[e] = pe;
        outm[e] = pm;
    }
    if (tid == 0) tot[img * nlines + line] = sP[n];
}

// Exclusive prefix of the line totals, pre[img][0..nlines] (blockIdx.y: rows 0, columns 1),
// for images whose lines are too many for the forward kernel to sum the skipped ones itself.
__global__ __launch_bounds__(BLK) void line_prefix_k(const double *__restrict__ rowtot,
                                                     const double *__restrict__ coltot, int nx,
                                                     int ny, double *__restrict__ rowpre,
                                                     double *__restrict__ colpre)
{
    __shared__ double swave[BLK / 64];
    const bool rows = blockIdx.y == 0;
    const int nlines = rows ? ny : nx;
    const int64_t img = blockIdx.x;
    const double *t = (rows ? rowtot : coltot) + img * nlines;
    double *pre = (rows ? rowpre : colpre) + img * (int64_t)(nlines + 1);
    const int tid = threadIdx.x;
    // each thread a contiguous run of lines; an exclusive scan of the run sums over the block
    const int run = (nlines + BLK - 1) / BLK;
    const int i0 = min(tid * run, nlines), i1 = min(i0 + run, nlines);
    double own = 0.0;
    for (int i = i0; i < i1; ++i) own += t[i];
    const int lane = tid & 63, wv = tid >> 6;
    double incl = own;
    for (int off = 1; off < 64; off <<= 1) {
        const double u = __shfl_up(incl, off, 64);
        incl += lane >= off ? u : 0.0;
    }
    if (lane == 63) swave[wv] = incl;
    __syncthreads();
    double acc = incl - own;
    for (int w = 0; w < wv; ++w) acc += swave[w];
    for (int i = i0; i < i1; ++i) {
        pre[i] = acc;
        acc += t[i];
    }
    if (tid == BLK - 1) pre[nlines] = acc;
}

// ---------------------------------------------------------------------------
// forward: projection and angle derivative, edge-driven
// ---------------------------------------------------------------------------
// Work item (view v, chunk q of 63 bins) of forward block b out of T = views x chunks.
// Blocks are dealt to the 8 XCDs in turn (b mod 8), so consecutive blocks sit on different
// L2 caches; the first T - T mod 8 blocks are renumbered so that each XCD takes a contiguous
// run w of items, and runs are ordered by groups of 16 neighbouring views, chunk, view: the
// blocks an XCD holds at once work on the same chunk of nearly the same angles, whose edges
// cross nearly the same pack entries.
constexpr int FWD_XCDS = 8, FWD_VGROUP = 16;
constexpr int FWD_UNROLL = 4;   // pack entries in flight per step of the forward walk
__device__ __forceinline__ void fwd_block_item(int64_t b, int64_t T, int nchunks, int64_t &v,
                                               int &q)
{
    const int64_t body = T - T % FWD_XCDS;
    const int64_t w = b < body ? (b % FWD_XCDS) * (body / FWD_XCDS) + b / FWD_XCDS : b;
    const int64_t V = T / nchunks;
    const int64_t gitems = (int64_t)FWD_VGROUP * nchunks;
    const int64_t g = w / gitems;
    const int64_t gsz = min((int64_t)FWD_VGROUP, V - g * FWD_VGROUP);
    const int64_t rem = w - g * gitems;
    q = (int)(rem / gsz);
    v = g * FWD_VGROUP + rem % gsz;
}

struct FwdArgs {
    const PackEntry *rowpack;   // [img][ny][nx+3]
    const PackEntry *colpack;   // [img][nx][ny+3]
    const PackEntry *rowpack_m; // mirrored lines, same layout
    const PackEntry *colpack_m;
    const double *rowtot;       // line totals [img][ny]
    const double *coltot;       // [img][nx]
    const double *rowpre;       // exclusive prefixes of the totals [img][ny + 1], or null: the
    const double *colpre;       // kernel then sums the skipped lines itself; [img][nx + 1]
    const double *theta;
    const int64_t *view_off;
    int nframes;
    int64_t V;
    int nx, ny, nb;
    double x0, y0, d, s0, ds;
    int ncols;        // columns in this launch (images = ncols * nframes, column-major)
    int col_out0;     // global column index of the first column (outputs)
    int nchunks;      // blocks per view
    float *y;         // [col][V][nb] or null
    float *dy;        // [col][V][nb] or null
    const float *g;   // [V][nb] or null
    double *part;     // [3][col][V][nchunks] (gdot, dnorm2, rnorm2 partials) or null
    int64_t part_cols;  // total columns of the partials array
    const float *bres;      // [V][nb]: residual mode, g := y - b (needs the projection)
    const double *tdir;     // trial angles theta + alpha[0] * tdir (null: theta)
    const double *talpha;
    const int *skip;        // when *skip != 0 the launch does nothing
    int write_resid;        // with bres: store y - b into y
};

template <int MODE, int NC, int FSEG>
__global__ __launch_bounds__(64 * FSEG) void fwd_edges_k(FwdArgs a)
{
    constexpr bool PROJ = (MODE & 1) != 0;
    constexpr bool MOM = (MODE & 2) != 0;
    __shared__ double sC[PROJ ? NC : 1][FSEG][64];
    __shared__ double sM[MOM ? NC : 1][FSEG][64];

    if (a.skip != nullptr && *a.skip != 0) return;   // uniform over the launch
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int seg = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index, uniform
    int64_t v;
    int q;
    fwd_block_item(blockIdx.x, gridDim.x, a.nchunks, v, q);
    const int c0 = blockIdx.y * NC;
    const int nc = min(NC, a.ncols - c0);
    const int f = frame_of(a.view_off, a.nframes, v);
    // The view constants, each edge's line range and the wave union of the ranges are the same
    // for every wave of the block (the waves share the block's 64 edges): wave 0 forms them
    // and hands them to the others through LDS.
    struct Shared {
        ViewC w;
        double inv_step;
        int la[64], lb[64];
        int WA, WB;
    };
    __shared__ Shared sh;
    const bool first = FSEG == 1 || seg == 0;
    ViewC w;
    if (first) {
        const double th = a.tdir != nullptr ? a.theta[v] + a.talpha[0] * a.tdir[v] : a.theta[v];
        w = make_view(th, a.d);
        if (FSEG > 1 && lane == 0) sh.w = w;
    }
    if (FSEG > 1) {
        __syncthreads();
        if (!first) w = sh.w;
    }
    const int64_t j = (int64_t)q * BINS + lane;

    const bool steep = w.steep != 0;
    const int nlines = steep ? a.ny : a.nx;
    const int nminor = steep ? a.nx : a.ny;
    const double line0 = steep ? a.y0 : a.x0;
    const double minor0 = steep ? a.x0 : a.y0;
    const double sl = steep ? w.sn : w.cs;
    const double sm = steep ? w.cs : w.sn;
    const double tl = steep ? w.cs : -w.sn;
    const double tm = steep ? -w.sn : w.cs;
    const bool asc = sm > 0.0;
    const double step = a.d * fabs(sm);
    double inv_step;
    if (first) {
        inv_step = 1.0 / step;
        if (FSEG > 1 && lane == 0) sh.inv_step = inv_step;
    }
    const double cw0 = asc ? (minor0 + 0.5 * a.d) * sm : (minor0 + (nminor - 0.5) * a.d) * sm;
    // descending walks read the mirrored packs, so every walk advances through its pack
    const PackEntry *pack = steep ? (asc ? a.rowpack : a.rowpack_m)
                                  : (asc ? a.colpack : a.colpack_m);
    const double *ltot = steep ? a.rowtot : a.coltot;
    const double *lpre = steep ? a.rowpre : a.colpre;
    const int64_t pstride = (int64_t)nlines * (nminor + 3);
    const int64_t tstride = nlines;
    const int64_t img0 = (int64_t)c0 * a.nframes + f;
    const int64_t cstride = a.nframes;   // images between consecutive columns

    double accP[NC], accF[NC], accM[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) accP[c] = accF[c] = accM[c] = 0.0;

    // The line range an edge touches (lines outside it lie wholly on one side of the edge),
    // then the wave's union of its edges' ranges, split evenly over the block's waves: every
    // lane walks the same lines, so one pack load of the wave reads one line's neighbouring
    // entries.  On a line outside an edge's own range the walk's clamped entry gives exactly
    // 0 or the line's total, the value the line contributes.
    const bool live = j <= a.nb;
    const double e = edge_coord(a.s0, a.ds, j);
    int la = nlines, lb = -1;   // lanes without an edge take no part in the union
    int WA, WB;
    if (first && live) {
        if (sl == 0.0) {
            la = 0;
            lb = nlines - 1;
        } else {
            const double A = e - w.wo - cw0 - (nminor - 1) * step;
            const double B = e + w.wo - cw0;
            // reciprocals instead of divisions: the range is padded by a line either side
            const double isl = 1.0 / sl, id = 1.0 / a.d;
            const double l1 = (A * isl - line0) * id - 0.5;
            const double l2 = (B * isl - line0) * id - 0.5;
            double lo = fmin(l1, l2), hi = fmax(l1, l2);
            lo = fmin(fmax(lo, -4.0), nlines + 4.0);
            hi = fmin(fmax(hi, -4.0), nlines + 4.0);
            la = min(max((int)floor(lo) - 1, 0), nlines);
            lb = min(max((int)ceil(hi) + 1, -1), nlines - 1);
        }
    }
    if (first) {
        WA = la;
        WB = lb;
        for (int off = 32; off > 0; off >>= 1) {
            WA = min(WA, __shfl_xor(WA, off, 64));
            WB = max(WB, __shfl_xor(WB, off, 64));
        }
        if (FSEG > 1) {
            sh.la[lane] = la;
            sh.lb[lane] = lb;
            if (lane == 0) {
                sh.WA = WA;
                sh.WB = WB;
            }
        }
    }
    if (FSEG > 1) {
        __syncthreads();
        if (!first) {
            inv_step = sh.inv_step;
            la = sh.la[lane];
            lb = sh.lb[lane];
            WA = sh.WA;
            WB = sh.WB;
        }
    }
    WA = __builtin_amdgcn_readfirstlane(WA);
    WB = __builtin_amdgcn_readfirstlane(WB);
    {
        // this wave's share of the union
        const int len = WB - WA + 1;
        const int sa = len > 0 ? WA + (len * seg) / FSEG : WA;
        const int sb = len > 0 ? WA + (len * (seg + 1)) / FSEG - 1 : WB;
        // Walk position of the edge on line L, in pixel steps (walk order):
        // q(L) = (e - lc(L) sl - wo - cw0) / step, linear in L.  The first pixel the edge
        // straddles is K0 = floor(q) + 1; with r = q + 2 clamped to [0, n + 1] the pack entry
        // index is K0 + 2 = 1 + trunc(r) and r - trunc(r) its fraction.  The offsets of the
        // edge from the centres of pixels K0 and K0 + 1 are va = wo + (q - K0) step and
        // va - step, FMAs of that fraction.
        const double dq = -a.d * sl * inv_step;
        double r = sa <= sb ? (__dsub_rn(e, __dmul_rn(pix_coord(line0, a.d, sa), sl)) - w.wo -
                               cw0) * inv_step + 2.0
                            : 0.0;
        const float stepf = (float)step;
        const float c0a = (float)(w.wo - step);            // va = c0a + dr * step
        const PackEntry *pline = pack + img0 * pstride + (int64_t)sa * (nminor + 3) + 1;
        // Along-ray coordinate of the centre of pixel k on line L, affine in both indices:
        // t(L, k) = tS + (L - sa) d tl + k d tm, with tS the value at (sa, 0) formed in FP64.
        // The walk's straddled pixel is k = K1 - 1 (ascending) or n - K1 (descending), so per
        // walk direction t = tB + (L - sa) d tl + K1 ks with an FP32 base tB and signed step
        // ks; the coordinates are O(1) on the unit square, so FP32 keeps them to ~1e-7.
        double tS = 0.0;
        float dtlf = 0.0f;
        if (MOM) {
            tS = pix_coord(line0, a.d, sa) * tl + pix_coord(minor0, a.d, 0) * tm;
            dtlf = (float)(a.d * tl);
        }
        auto walk = [&](auto ascending) __attribute__((always_inline)) {
            constexpr bool ASC = decltype(ascending)::value;
            float tBf = 0.0f, ksf = 0.0f;
            if (MOM) {
                const double dtm = a.d * tm;
                tBf = (float)(ASC ? tS - dtm : tS + (double)nminor * dtm);
                ksf = (float)(ASC ? dtm : -dtm);
            }
            // Entry of line L at walk position rl: clamping the position itself is exact
            // (beyond [0, n + 1] the entry's pixels are padding, or the edge lies past the
            // footprint of pixel 0); K1 = K0 + 1 and the fraction dr.
            auto locate = [&](double rl, int &K1, float &dr) __attribute__((always_inline)) {
                const double rc = fmin(fmax(rl, 0.0), (double)(nminor + 1));
                K1 = (int)rc;
                dr = (float)__builtin_amdgcn_fract(rc);
            };
            // x * psi_h (and the chord moments) of the two straddled pixels of a located
            // line into the FP32 sums fF / fM of its pair of lines; the prefix into accP
            auto apply = [&](int L, int K1, float dr, const PackEntry (&E)[NC], float (&fF)[NC],
                             float (&fM)[NC]) __attribute__((always_inline)) {
                float pa = 0.f, pb = 0.f, ma = 0.f, mb = 0.f;
                const float va = fmaf(dr, stepf, c0a);
                const float vb = va - stepf;
                if (PROJ) {
                    pa = psi_h(va, w.fwo, w.fwi, w.fk);
                    pb = psi_h(vb, w.fwo, w.fwi, w.fk);
                }
                if (MOM) {
                    const float tLf = fmaf((float)(L - sa), dtlf, tBf);
                    const float ta = fmaf((float)K1, ksf, tLf);   // straddled pixel a
                    const float tb = ta + ksf;                      // its neighbour b
                    float La, Lb, mua, mub;
                    moment_f(va, w, La, mua);
                    moment_f(vb, w, Lb, mub);
                    ma = La * (ta + mua);
                    mb = Lb * (tb + mub);
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if (c == 0 || c < nc) {
                        if (PROJ) {
                            accP[c] += E[c].P;
                            fF[c] = fmaf(E[c].b, pb, fmaf(E[c].a, pa, fF[c]));
                        }
                        if (MOM) fM[c] = fmaf(E[c].b, mb, fmaf(E[c].a, ma, fM[c]));
                    }
                }
            };
            auto fetch = [&](const PackEntry *pl, int K1, PackEntry (&E)[NC])
                             __attribute__((always_inline)) {
                const PackEntry *pe = pl + (unsigned)K1;
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    if (c == 0 || c < nc) E[c] = pe[c * cstride * pstride];   // nc >= 1
            };
            auto flush = [&](const float (&fF)[NC], const float (&fM)[NC])
                             __attribute__((always_inline)) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if (PROJ) accF[c] += (double)fF[c];
                    if (MOM) accM[c] += (double)fM[c];
                }
            };
            const int lstride = nminor + 3;
            int L = sa;
            // U lines per step, every load issued before any line's arithmetic (the loads
            // wait on L2; several in flight hide that latency); U * NC entries per step
            constexpr int U = FWD_UNROLL / NC > 1 ? FWD_UNROLL / NC : 1;
            for (; L + U - 1 <= sb; L += U) {
                double rr[U];
                int K1[U];
                float dr[U];
                PackEntry E[U][NC];
                rr[0] = r;
#pragma unroll
                for (int u = 1; u < U; ++u) rr[u] = rr[u - 1] + dq;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    locate(rr[u], K1[u], dr[u]);
                    fetch(pline + u * lstride, K1[u], E[u]);
                }
                float fF[NC], fM[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) fF[c] = fM[c] = 0.0f;
#pragma unroll
                for (int u = 0; u < U; ++u) apply(L + u, K1[u], dr[u], E[u], fF, fM);
                flush(fF, fM);
                r = rr[U - 1] + dq;
                pline += U * lstride;
            }
            for (; L <= sb; ++L, r += dq, pline += lstride) {
                int K1a;
                float dra;
                locate(r, K1a, dra);
                PackEntry Ea[NC];
                fetch(pline, K1a, Ea);
                float fF[NC], fM[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) fF[c] = fM[c] = 0.0f;
                apply(L, K1a, dra, Ea, fF, fM);
                flush(fF, fM);
            }
        };
        if (asc) walk(std::true_type{});
        else walk(std::false_type{});
        if (PROJ && seg == 0) {
            // lines outside the union that lie wholly on the lower side of this edge: for
            // sl > 0 the lines below la, for sl < 0 the lines above lb.  A live edge has
            // WA <= la <= lb + 1 <= WB + 1, so these are the lines below WA (sl > 0) or above
            // WB (sl < 0).  With prefixes of the line totals each is a difference of two of
            // them; otherwise the wave sums the totals on its side of the union (lanes strided
            // over the lines, a fixed DPP reduction) and keeps exact sums for the other terms.
            auto range = [&](const double *lt, int l0, int l1) {
                double t = 0.0;
                for (int l = l0; l < l1; ++l) t += lt[l];
                return t;
            };
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (c < nc && sl != 0.0) {
                    if (lpre != nullptr) {
                        const double *pr = lpre + (img0 + c * cstride) * (tstride + 1);
                        if (live) {
                            double add = 0.0;
                            if (sl > 0.0) {
                                add += pr[min(la, WA)];
                                if (la > WB + 1) add += pr[la] - pr[WB + 1];
                            } else {
                                if (lb + 1 < WA) add += pr[WA] - pr[lb + 1];
                                add += pr[nlines] - pr[max(lb + 1, WB + 1)];
                            }
                            accP[c] += add;
                        }
                        continue;
                    }
                    const double *lt = ltot + (img0 + c * cstride) * tstride;
                    const int s0 = sl > 0.0 ? 0 : WB + 1, s1 = sl > 0.0 ? WA : nlines;
                    // a lane's lines with eight loads in flight, in line order
                    double side = md::strided_sum(lt + s0, 1, s1 - s0, lane, 64);
                    side = wave::wave_sum_dpp(side);
                    if (live) {
                        double add = 0.0;
                        if (sl > 0.0) {
                            add += la >= WA ? side : range(lt, 0, la);
                            if (la > WB + 1) add += range(lt, WB + 1, la);
                        } else {
                            if (lb + 1 < WA) add += range(lt, lb + 1, WA);
                            add += lb <= WB ? side : range(lt, lb + 1, nlines);
                        }
                        accP[c] += add;
                    }
                }
            }
        }
    }
    const double hq = (double)w.fh;
#pragma unroll
    for (int c = 0; c < NC; ++c) accF[c] *= hq;
    const double d2 = a.d * a.d;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (PROJ) sC[c][seg][lane] = d2 * accP[c] + accF[c];
        if (MOM) sM[c][seg][lane] = accM[c];
    }
    __syncthreads();
    if (seg != 0) return;
    // wave 0: C(e) of its 64 edges (segments summed in a fixed order), then 63 bins
    double Ce[NC], Me[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        Ce[c] = Me[c] = 0.0;
#pragma unroll
        for (int sg = 0; sg < FSEG; ++sg) {
            if (PROJ) Ce[c] += sC[c][sg][lane];
            if (MOM) Me[c] += sM[c][sg][lane];
        }
    }
    const int64_t jb = (int64_t)q * BINS + lane;
    const bool has_bin = lane < BINS && jb < a.nb;
    const double inv_ds = 1.0 / a.ds;
    const float gv_in = (a.g != nullptr && has_bin) ? a.g[v * a.nb + jb] : 0.0f;
    const float bv = (a.bres != nullptr && has_bin) ? a.bres[v * a.nb + jb] : 0.0f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c >= nc) break;
        const int64_t col = a.col_out0 + c0 + c;
        const int64_t o = (col * a.V + v) * a.nb + jb;
        // neighbouring edge's total through a lane shift (lane 63 has no bin)
        const double Cn = __shfl_down(Ce[c], 1, 64);
        const double Mn = __shfl_down(Me[c], 1, 64);
        double yv = 0.0, Dv = 0.0;
        if (has_bin) {
            if (PROJ) {
                yv = (Cn - Ce[c]) * inv_ds;
                if (a.y) a.y[o] = (float)(a.write_resid ? yv - (double)bv : yv);
            }
            if (MOM) {
                Dv = (Me[c] - Mn) * inv_ds;
                if (a.dy) a.dy[o] = (float)Dv;
            }
        }
        if (a.part != nullptr) {
            const double rv = (a.bres != nullptr && has_bin) ? yv - (double)bv : 0.0;
            const double gv = a.bres != nullptr ? rv : (double)gv_in;
            const double sg = wave_sum(Dv * gv);
            const double sh = wave_sum(Dv * Dv);
            const double sr = wave_sum(rv * rv);
            if (lane == 0) {
                const int64_t po = (col * a.V + v) * a.nchunks + q;
                const int64_t ps = a.part_cols * a.V * a.nchunks;
                a.part[po] = sg;
                a.part[ps + po] = sh;
                a.part[2 * ps + po] = sr;
            }
        }
    }
}

__global__ void finalize_parts_k(const double *__restrict__ part, int64_t ncols, int64_t V,
                                 int nchunks, double *gdot, double *dnorm2, double *rnorm2,
                                 const int *skip)
{
    if (skip != nullptr && *skip != 0) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncols * V) return;
    const int64_t ps = ncols * V * nchunks;
    double sg = 0.0, sh = 0.0, sr = 0.0;
    for (int q = 0; q < nchunks; ++q) {
        sg += part[i * nchunks + q];
        sh += part[ps + i * nchunks + q];
        sr += part[2 * ps + i * nchunks + q];
    }
    if (gdot) gdot[i] = sg;
    if (dnorm2) dnorm2[i] = sh;
    if (rnorm2) rnorm2[i] = sr;
}

// ---------------------------------------------------------------------------
// backward: pixel-driven gather
// ---------------------------------------------------------------------------
struct BwdArgs {
    const float *y;
    const double *theta;
    const int64_t *view_off;
    int nframes;
    int64_t V;
    int nx, ny, nb;
    double x0, y0, d, s0, ds;
    int tiles_x;
    int W;           // staged bins per view (<= WMAX)
    float *x;
    int nsplit;      // views of a frame split over blockIdx.z; partial images when > 1
    float *part;     // [nsplit][col][frame][ny][nx] partial images (nsplit > 1)
    int accumulate;  // x += result instead of x = result
    TvEpilogue tv;   // one column: x += lam Psi^T (w Psi u) (tv.u null: none)
};

// Backprojection per pixel and view, summed by parts over the bin edges inside its footprint.
// With the footprint's bins y_0 .. y_E (E edges inside, offsets v_i of edge i from the pixel
// centre), x = (1/ds) [sum_i Phi(v_i) (y_{i-1} - y_i) + d^2 y_E].  Writing Phi / h = C + psi
// with C = d^2 / (2h) (Phi is C + an odd function of v) gives
//   x ds = (d^2 / 2)(y_0 + y_E) + sum_i psi(v_i) h (y_{i-1} - y_i),
//   psi(v) = c1 - q |q| / (2 rho),  c1 = med3(v, -wo, wo),  q = c1 - med3(v, -wi, wi),
// (c1 is the clamped offset; q, the part of it beyond the plateau, is the ramp coordinate:
// the plateau gives psi = v, a ramp v - (v -+ wi)^2 / (2 rho), outside the footprint
// psi = +-C; rho = 0 is the box limit with 1 / (2 rho) := 0).  h C = d^2 / 2 is the same for
// every view, so the window of view v is staged as pairs (h_v (y_{j-1} - y_j), y_j) and one
// pixel-view costs two medians, a subtraction, a multiplication and two multiply-adds per edge.
//
// Per-view constants of one backward tile: the footprint start of the tile centre in bin
// units, split as jb (staged-window index of its bin) + a fraction in [0, 1), stored as
// T0 = fraction + TSHIFT and jb - TSHIFT so that every pixel's start T0 + pk ax + pl ay is
// positive (its truncation is its floor); the bin-unit steps of one pixel along x and y; for
// edge i of the window its offset from the pixel centre at fraction 0 (i ds - wo); wo, wi and
// 1 / (2 rho).
constexpr int TSHIFT = 64;
template <int E>
struct BView {
    double T0, ax, ay;
    int jb;
    float cm[E];
    float wo, wi, fk;
};

// One thread per PX pixels of a 16x16 tile, rows ll, ll + 16/PX, ...: the per-view constants
// staged in LDS serve PX pixels per read.
template <int PX>
struct BwdShape {
    static constexpr int threads = TILE * TILE / PX;
    static constexpr int rows = TILE / PX;   // row step between a thread's pixels
};
constexpr int BWD_PX = 2;
constexpr int BWD_BLK = BwdShape<BWD_PX>::threads;

// The window of a pixel's footprint lies inside the staged one: with j0 the window's first bin
// (one bin below the tile footprint's floor) jj = floor(pixel footprint start) - j0 >= 1, and
// jj + E <= (TILE - 1) d sqrt(2) / ds + 2 + E <= W - 2 (bwd_window), exactly; FP64 rounding of
// the footprint starts cannot move them by a bin.  Debug builds check it.
template <int E>
__device__ __forceinline__ void check_window(int jj, int W)
{
#ifdef NLRMM_DEBUG
    if (jj < 0 || jj + E >= W) __builtin_trap();
#endif
}

template <int E, int PX>
__global__ __launch_bounds__(BwdShape<PX>::threads) void bwd_tiles_k(BwdArgs a)
{
    constexpr int NT = BwdShape<PX>::threads;
    constexpr int RS = BwdShape<PX>::rows;
    __shared__ BView<E> sv[VCHUNK];
    __shared__ int sj0[VCHUNK];
    __shared__ float sh[VCHUNK];
    extern __shared__ float2 sy_dyn[];   // [VCHUNK][W] (W staged bins per view, dynamic size):
                                         // (h (y_{j-1} - y_j), y_j)
    const int tid = threadIdx.x;
    const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    const int64_t img = blockIdx.y;
    const int64_t col = img / a.nframes;
    const int f = (int)(img - col * a.nframes);
    const int kl = tid % TILE, ll = tid / TILE;   // ll in [0, RS)
    const int k = tx * TILE + kl;
    const int64_t fv0 = (a.view_off && a.nframes > 1) ? a.view_off[f] : 0;
    const int64_t fv1 = (a.view_off && a.nframes > 1) ? a.view_off[f + 1] : a.V;
    const int split = blockIdx.z;
    const int64_t v0 = fv0 + ((fv1 - fv0) * split) / a.nsplit;
    const int64_t v1 = fv0 + ((fv1 - fv0) * (split + 1)) / a.nsplit;
    const float *ycol = a.y + col * a.V * a.nb;
    const double xc = a.x0 + (tx * TILE + 0.5 * TILE) * a.d;
    const double yc = a.y0 + (ty * TILE + 0.5 * TILE) * a.d;
    // pixel centres relative to the tile centre, in pixels
    const double pk = kl + 0.5 - 0.5 * TILE, pl = ll + 0.5 - 0.5 * TILE;
    double acc[PX];
#pragma unroll
    for (int px = 0; px < PX; ++px) acc[px] = 0.0;
    const float fds = (float)a.ds;

    for (int64_t vb = v0; vb < v1; vb += VCHUNK) {
        const int nv = (int)min((int64_t)VCHUNK, v1 - vb);
        if (tid < nv) {
            const ViewC w = make_view(a.theta[vb + tid], a.d);
            const double cC = xc * w.cs + yc * w.sn;
            const double R = (TILE - 1) * 0.5 * a.d * (fabs(w.cs) + fabs(w.sn)) + w.wo;
            const int j0 = (int)floor((cC - R - a.s0) / a.ds) - 1;
            const double T = (cC - w.wo - a.s0) / a.ds;
            const double Tf = floor(T);
            BView<E> q;
            q.T0 = (T - Tf) + TSHIFT;
            q.ax = a.d * w.cs / a.ds;
            q.ay = a.d * w.sn / a.ds;
            q.jb = (int)Tf - j0 - TSHIFT;
            for (int i = 1; i <= E; ++i) q.cm[i - 1] = (float)(i * a.ds - w.wo);
            q.wo = w.fwo;
            q.wi = w.fwi;
            q.fk = w.fk;
            sv[tid] = q;
            sj0[tid] = j0;
            sh[tid] = w.fh;
        }
        __syncthreads();
        for (int i = tid; i < nv * a.W; i += NT) {
            const int vi = i / a.W, jj = i - vi * a.W;
            const int jbin = sj0[vi] + jj;
            const float *yv = ycol + (vb + vi) * a.nb;
            const float y1 = (jbin >= 0 && jbin < a.nb) ? yv[jbin] : 0.0f;
            const float y0 = (jbin >= 1 && jbin - 1 < a.nb) ? yv[jbin - 1] : 0.0f;
            sy_dyn[vi * a.W + jj] = make_float2(sh[vi] * (y0 - y1), y1);
        }
        __syncthreads();
        // this chunk's views in FP32 (chunks summed in FP64): y_0 + y_E and the edge terms
        float ay[PX], ap[PX];
#pragma unroll
        for (int px = 0; px < PX; ++px) ay[px] = ap[px] = 0.0f;
        for (int vi = 0; vi < nv; ++vi) {
            const BView<E> &q = sv[vi];
            // footprint start of each pixel in bin units (shifted positive): window bin jj and
            // fraction fr; edge i of the window sits at (i - fr) ds - wo from the pixel centre
            double t = fma(pk, q.ax, fma(pl, q.ay, q.T0));
#pragma unroll
            for (int px = 0; px < PX; ++px) {
                if (px > 0) t = fma((double)RS, q.ay, t);
                const float fr = (float)__builtin_amdgcn_fract(t);
                const int jj = q.jb + (int)t;
                check_window<E>(jj, a.W);
                const float2 *yy = &sy_dyn[vi * a.W + jj];
                ay[px] += yy[0].y + yy[E].y;     // times d^2 / 2, applied per chunk
#pragma unroll
                for (int i = 1; i <= E; ++i) {
                    const float psi = psi_h(fmaf(-fr, fds, q.cm[i - 1]), q.wo, q.wi, q.fk);
                    ap[px] = fmaf(psi, yy[i].x, ap[px]);   // psi_i h (y_{i-1} - y_i)
                }
            }
        }
        const float hd2 = 0.5f * (float)(a.d * a.d);
#pragma unroll
        for (int px = 0; px < PX; ++px) acc[px] += (double)fmaf(hd2, ay[px], ap[px]);
        __syncthreads();
    }
    const int64_t ibase = (col * a.nframes + f) * (int64_t)a.ny;
#pragma unroll
    for (int px = 0; px < PX; ++px) {
        const int l = ty * TILE + ll + px * RS;
        if (k >= a.nx || l >= a.ny) continue;
        const int64_t o = (ibase + l) * a.nx + k;
        if (a.nsplit > 1) {
            const int64_t tot = (int64_t)gridDim.y * a.nx * a.ny;
            a.part[split * tot + o] = (float)(acc[px] / a.ds);
        } else {
            const double prev = a.accumulate ? (double)a.x[o] : 0.0;
            float v = (float)(prev + acc[px] / a.ds);
            if (a.tv.u != nullptr)
                v += (float)a.tv.lamp[0] *
                     tv_grad_at(a.tv.u, a.tv.w, tvgeo(a.nx, a.ny, a.nframes, a.tv.temporal), o,
                                a.tv.e2);
            a.x[o] = v;
        }
    }
}

// x = D(theta)^T r: the transpose of the angle derivative (per view, bin j carries
// (M(e_j) - M(e_{j+1})) / ds with M the chord first moment), gathered per pixel like the
// backprojection.  Per pixel and view the edges inside the footprint (at most E) carry
// M_i = L_i (t_c + mu_i) and the bins give sum_i M_i (r[jj + i] - r[jj + i - 1]) (the moments
// at the two bounding edges vanish).  One thread per pixel pair of a 16x16 tile, 32-view
// chunks with their windows of r and per-view constants staged in LDS; no view split.
template <int E>
struct BMView {
    double T0, ax, ay;   // footprint start (shifted positive), bin-unit steps per pixel
    int jb;
    float tc0, tkx, tly;  // t-coordinate of the tile centre and its steps per pixel
    float cm[E];          // edge i offset from the pixel centre at fraction 0: i ds - wo
    float fwo, fwi, frho, fh, inv_ab, Kr, tq, kp, kappa;
};

constexpr int MOM_BLK = TILE * TILE / 2;   // one thread per pixel pair

template <int E>
__global__ __launch_bounds__(MOM_BLK) void bwd_moment_tiles_k(BwdArgs a)
{
    __shared__ BMView<E> sv[VCHUNK];
    __shared__ int sj0[VCHUNK];
    __shared__ float sy[VCHUNK][WMAX];
    const int tid = threadIdx.x;
    const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    const int64_t img = blockIdx.y;
    const int64_t col = img / a.nframes;
    const int f = (int)(img - col * a.nframes);
    const int kl = tid % TILE, ll = tid / TILE;
    const int k = tx * TILE + kl;
    const int l0 = ty * TILE + ll, l1 = l0 + TILE / 2;
    const bool act0 = k < a.nx && l0 < a.ny, act1 = k < a.nx && l1 < a.ny;
    const int64_t fv0 = (a.view_off && a.nframes > 1) ? a.view_off[f] : 0;
    const int64_t fv1 = (a.view_off && a.nframes > 1) ? a.view_off[f + 1] : a.V;
    const int split = blockIdx.z;
    const int64_t v0 = fv0 + ((fv1 - fv0) * split) / a.nsplit;
    const int64_t v1 = fv0 + ((fv1 - fv0) * (split + 1)) / a.nsplit;
    const float *ycol = a.y + col * a.V * a.nb;
    const double xc = a.x0 + (tx * TILE + 0.5 * TILE) * a.d;
    const double yc = a.y0 + (ty * TILE + 0.5 * TILE) * a.d;
    const double pk = kl + 0.5 - 0.5 * TILE, pl = ll + 0.5 - 0.5 * TILE;
    const double hl = 0.5 * TILE;
    double acc0 = 0.0, acc1 = 0.0;

    for (int64_t vb = v0; vb < v1; vb += VCHUNK) {
        const int nv = (int)min((int64_t)VCHUNK, v1 - vb);
        if (tid < nv) {
            const ViewC w = make_view(a.theta[vb + tid], a.d);
            const double cC = xc * w.cs + yc * w.sn;
            const double R = (TILE - 1) * 0.5 * a.d * (fabs(w.cs) + fabs(w.sn)) + w.wo;
            const int j0 = (int)floor((cC - R - a.s0) / a.ds) - 1;
            const double T = (cC - w.wo - a.s0) / a.ds;
            const double Tf = floor(T);
            BMView<E> q;
            q.T0 = (T - Tf) + TSHIFT;
            q.ax = a.d * w.cs / a.ds;
            q.ay = a.d * w.sn / a.ds;
            q.jb = (int)Tf - j0 - TSHIFT;
            q.tc0 = (float)(-xc * w.sn + yc * w.cs);
            q.tkx = (float)(-a.d * w.sn);
            q.tly = (float)(a.d * w.cs);
            for (int i = 1; i <= E; ++i) q.cm[i - 1] = (float)(i * a.ds - w.wo);
            q.fwo = w.fwo;
            q.fwi = w.fwi;
            q.frho = w.frho;
            q.fh = w.fh;
            q.inv_ab = w.inv_ab;
            q.Kr = w.Kr;
            q.tq = w.tq;
            q.kp = w.kp;
            q.kappa = w.kappa;
            sv[tid] = q;
            sj0[tid] = j0;
        }
        __syncthreads();
        // staged as differences r_j - r_{j-1} (r = 0 outside the detector): the same FP32
        // subtraction the per-pixel sum would make, done once per view
        for (int i = tid; i < nv * a.W; i += MOM_BLK) {
            const int vi = i / a.W, jj = i - vi * a.W;
            const int jbin = sj0[vi] + jj;
            const float *yv = ycol + (vb + vi) * a.nb;
            const float r1 = (jbin >= 0 && jbin < a.nb) ? yv[jbin] : 0.0f;
            const float r0 = (jbin >= 1 && jbin - 1 < a.nb) ? yv[jbin - 1] : 0.0f;
            sy[vi][jj] = r1 - r0;
        }
        __syncthreads();
        const float fds = (float)a.ds;
        float accf0 = 0.0f, accf1 = 0.0f;
        for (int vi = 0; vi < nv; ++vi) {
            const BMView<E> &q = sv[vi];
            ViewC w;
            w.fwo = q.fwo;
            w.fwi = q.fwi;
            w.frho = q.frho;
            w.fh = q.fh;
            w.inv_ab = q.inv_ab;
            w.Kr = q.Kr;
            w.tq = q.tq;
            w.kp = q.kp;
            w.kappa = q.kappa;
            const double t0 = fma(pk, q.ax, fma(pl, q.ay, q.T0));
            const double t1 = fma(hl, q.ay, t0);
            const float tcp0 = fmaf((float)pk, q.tkx, fmaf((float)pl, q.tly, q.tc0));
            const float tcp1 = fmaf((float)hl, q.tly, tcp0);
            float sum[2];
#pragma unroll
            for (int px = 0; px < 2; ++px) {
                const double t = px == 0 ? t0 : t1;
                const float tc = px == 0 ? tcp0 : tcp1;
                const float fr = (float)__builtin_amdgcn_fract(t);
                const int jj = q.jb + (int)t;
                check_window<E>(jj, a.W);
                const float *yy = &sy[vi][jj];
                float sm = 0.0f;
#pragma unroll
                for (int i = 1; i <= E; ++i) {
                    float L, mu;
                    moment_f(fmaf(-fr, fds, q.cm[i - 1]), w, L, mu);
                    sm = fmaf(L * (tc + mu), yy[i], sm);
                }
                sum[px] = sm;
            }
            accf0 += sum[0];
            accf1 += sum[1];
        }
        acc0 += (double)accf0;
        acc1 += (double)accf1;
        __syncthreads();
    }
    const int64_t ibase = (col * a.nframes + f) * (int64_t)a.ny;
    // one image, or this split's partial image (summed in split order by sum_splits_k)
    float *out = a.nsplit > 1 ? a.part + split * ((int64_t)gridDim.y * a.nx * a.ny) : a.x;
    if (act0) out[(ibase + l0) * a.nx + k] = (float)(acc0 / a.ds);
    if (act1) out[(ibase + l1) * a.nx + k] = (float)(acc1 / a.ds);
}

// MD: also the block partials of <X_i, x> (i < nv) and <x, x> over the written image (one
// element per thread; blocks of 256 threads, as multidot_k forms them).
struct MdDev {
    const float *X;
    int64_t ldx;
    int nv;
    double *part;
};

template <int NS>
__device__ __forceinline__ double split_sum(const float *__restrict__ part, int64_t n, int64_t i,
                                            double s)
{
    float pv[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) pv[k] = part[k * n + i];
#pragma unroll
    for (int k = 0; k < NS; ++k) s += (double)pv[k];
    return s;
}

template <bool MD>
__global__ __launch_bounds__(256) void sum_splits_k(const float *__restrict__ part, int nsplit,
                                                    int64_t n, float *__restrict__ x,
                                                    int accumulate, TvEpilogue tv, int nx, int ny,
                                                    int nframes, MdDev md)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        // the partials of all splits loaded together (the tuned split counts), then summed
        // in split order
        double s = accumulate ? (double)x[i] : 0.0;
        switch (nsplit) {
            case 1: s = split_sum<1>(part, n, i, s); break;
            case 2: s = split_sum<2>(part, n, i, s); break;
            case 4: s = split_sum<4>(part, n, i, s); break;
            case 8: s = split_sum<8>(part, n, i, s); break;
            case 16: s = split_sum<16>(part, n, i, s); break;
            default:
                for (int k = 0; k < nsplit; ++k) s += (double)part[k * n + i];
        }
        float v = (float)s;
        if (tv.u != nullptr)
            v += (float)tv.lamp[0] *
                 tv_grad_at(tv.u, tv.w, tvgeo(nx, ny, nframes, tv.temporal), i, tv.e2);
        x[i] = v;
    } else if (!MD) {
        return;
    }
    if constexpr (MD) {
        // every thread takes part (the block reductions have barriers); each reads back only
        // the element it wrote
        __shared__ double sacc[16][md::MD_BLK];
        md::multidot_body<md::MD_MAX>(md.X, md.ldx, md.nv, x, x, n, md.part, sacc, blockIdx.x,
                                      gridDim.x);
    }
}

int edges_inside(const nlrmm_geom &g)
{
    // maximum number of bin edges strictly inside a pixel footprint (width <= d sqrt 2)
    return (int)ceil(g.d * 1.4142135623730951 / g.ds - 1e-12);
}

// Staged detector window of a backward tile, in bins: the footprint of the tile's pixels
// (TILE - 1 pixel pitches times at most d sqrt 2 between the outer centres), the E + 1 bins of
// one pixel footprint and a margin of 3 bins for the floor of the window start and rounding.
int bwd_window(const nlrmm_geom &g)
{
    return (int)ceil((TILE - 1) * g.d * 1.4142135623730951 / g.ds) + edges_inside(g) + 4;
}

}  // namespace

int fwd_geom_ok(const nlrmm_geom &g) { return g.nx <= MAX_LINE && g.ny <= MAX_LINE; }

int bwd_geom_ok(const nlrmm_geom &g)
{
    const int E = edges_inside(g);
    return E >= 1 && E <= 4 && bwd_window(g) <= WMAX;
}

// Images with more lines than this get prefix sums of their line totals from a launch of
// their own: the forward kernel's own sums over the skipped lines would take each wave
// several loads per lane and line group.
constexpr int FWD_PREFIX_MIN_LINES = 1024;
static bool fwd_prefixed(const nlrmm_geom &g)
{
    return g.nx > FWD_PREFIX_MIN_LINES || g.ny > FWD_PREFIX_MIN_LINES;
}

// Workspace for the forward pass of `gcols` columns.
static size_t fwd_ws_bytes(const nlrmm_geom &g, int nframes, int gcols, int64_t V, int nchunks,
                           int ncols_total)
{
    const int64_t nimg = (int64_t)gcols * nframes;
    const int64_t nx = g.nx, ny = g.ny;
    size_t b = 0;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    b += 2 * al(sizeof(PackEntry) * nimg * ny * (nx + 3));   // row packs, direct and mirrored
    b += 2 * al(sizeof(PackEntry) * nimg * nx * (ny + 3));   // column packs, likewise
    b += al(sizeof(double) * nimg * (ny + nx));              // line totals
    if (fwd_prefixed(g)) b += al(sizeof(double) * nimg * (ny + nx + 2));   // their prefixes
    b += al(sizeof(double) * 2 * (size_t)ncols_total * V * nchunks);   // reduction partials
    return b;
}

template <int MODE, int NC>
static void launch_fwd_seg(int seg, dim3 grid, const FwdArgs &a, hipStream_t s)
{
    switch (seg) {
        case 1: fwd_edges_k<MODE, NC, 1><<<grid, 64, 0, s>>>(a); break;
        case 2: fwd_edges_k<MODE, NC, 2><<<grid, 128, 0, s>>>(a); break;
        case 8: fwd_edges_k<MODE, NC, 8><<<grid, 512, 0, s>>>(a); break;
        default: fwd_edges_k<MODE, NC, 4><<<grid, 256, 0, s>>>(a); break;
    }
}

template <int MODE>
static void launch_fwd_mode(int NC, int seg, dim3 grid, const FwdArgs &a, hipStream_t s)
{
    switch (NC) {
        case 1: launch_fwd_seg<MODE, 1>(seg, grid, a, s); break;
        case 2: launch_fwd_seg<MODE, 2>(seg, grid, a, s); break;
        case 4: launch_fwd_seg<MODE, 4>(seg, grid, a, s); break;
        default: launch_fwd_seg<MODE, 8>(seg, grid, a, s); break;
    }
}

int launch_project(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols,
                   const float *x, const double *theta, float *y, float *dy, const float *gres,
                   double *gdot, double *dnorm2, hipStream_t s)
{
    FwdOptions o;
    o.y = y;
    o.dy = dy;
    o.g = gres;
    o.gdot = gdot;
    o.dnorm2 = dnorm2;
    return launch_project_ex(ctx, g, b, ncols, x, theta, o, s);
}

int launch_project_ex(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols,
                      const float *x, const double *theta, const FwdOptions &o, hipStream_t s)
{
    if (!fwd_geom_ok(g)) return NLRMM_ESHAPE;
    const int F = b.nframes;
    const int64_t V = b.nviews;
    const int nchunks = (g.nbins + BINS - 1) / BINS;
    const bool mom = o.dy || o.gdot || o.dnorm2;
    const bool proj = o.y != nullptr || o.bres != nullptr;
    const bool red = o.gdot || o.dnorm2 || o.rnorm2;
    if (o.bres && !proj) return NLRMM_ENOTSUP;
    if (o.norm_part && (ncols != 1 || !o.norm_src || !o.norm_scal || !o.norm_out ||
                        !o.norm_status || o.norm_nblk < 1))
        return NLRMM_ENOTSUP;
    const int GC = 8;                       // columns prepared per group
    const int gcols = ncols < GC ? ncols : GC;
    size_t need = fwd_ws_bytes(g, F, gcols, V, nchunks, 0);
    const size_t part_bytes = red ? sizeof(double) * 3 * (size_t)ncols * V * nchunks : 0;
    double *part = o.part_buf;
    if (red && part == nullptr) need += part_bytes + 256;
    int rc = ensure_workspace(ctx, need, s);
    if (rc) return rc;
    const int64_t nx = g.nx, ny = g.ny;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    char *p = (char *)ctx->ws.ptr;
    PackEntry *rowpack = (PackEntry *)p;
    p += al(sizeof(PackEntry) * (int64_t)gcols * F * ny * (nx + 3));
    PackEntry *rowpack_m = (PackEntry *)p;
    p += al(sizeof(PackEntry) * (int64_t)gcols * F * ny * (nx + 3));
    PackEntry *colpack = (PackEntry *)p;
    p += al(sizeof(PackEntry) * (int64_t)gcols * F * nx * (ny + 3));
    PackEntry *colpack_m = (PackEntry *)p;
    p += al(sizeof(PackEntry) * (int64_t)gcols * F * nx * (ny + 3));
    double *tot = (double *)p;
    p += al(sizeof(double) * (int64_t)gcols * F * (ny + nx));
    const bool prefixed = fwd_prefixed(g);
    double *pre = nullptr;
    if (prefixed) {
        pre = (double *)p;
        p += al(sizeof(double) * (int64_t)gcols * F * (ny + nx + 2));
    }
    if (red && part == nullptr) part = (double *)p;

    const int64_t npix = nx * ny;
    for (int cbeg = 0; cbeg < ncols; cbeg += gcols) {
        const int nc = ncols - cbeg < gcols ? ncols - cbeg : gcols;
        const int64_t nimg = (int64_t)nc * F;
        const float *xg = x + (int64_t)cbeg * F * npix;
        // row and column packs of every image in one launch (with the line totals)
        double *ctot = tot + nimg * ny;
        NormJob nj{o.norm_src, o.norm_part, o.norm_nblk, o.norm_scal, o.norm_tol, o.norm_out,
                   o.norm_status};
        pack_lines_k<<<dim3((unsigned)(ny + nx), (unsigned)nimg), BLK, 0, s>>>(
            xg, (int)nx, (int)ny, rowpack, colpack, rowpack_m, colpack_m, tot, ctot, nj);
        double *rowpre = nullptr, *colpre = nullptr;
        if (prefixed) {
            rowpre = pre;
            colpre = pre + nimg * (ny + 1);
            line_prefix_k<<<dim3((unsigned)nimg, 2), BLK, 0, s>>>(tot, ctot, (int)nx, (int)ny,
                                                                 rowpre, colpre);
        }

        FwdArgs a;
        a.rowpack = rowpack;
        a.colpack = colpack;
        a.rowpack_m = rowpack_m;
        a.colpack_m = colpack_m;
        a.rowtot = tot;
        a.coltot = ctot;
        a.rowpre = rowpre;
        a.colpre = colpre;
        a.theta = theta;
        a.view_off = b.view_off;
        a.nframes = F;
        a.V = V;
        a.nx = g.nx;
        a.ny = g.ny;
        a.nb = g.nbins;
        a.x0 = g.x0;
        a.y0 = g.y0;
        a.d = g.d;
        a.s0 = g.s0;
        a.ds = g.ds;
        a.ncols = nc;
        a.col_out0 = cbeg;
        a.nchunks = nchunks;
        a.y = o.y;
        a.dy = o.dy;
        a.g = o.g;
        a.part = red ? part : nullptr;
        a.part_cols = ncols;
        a.bres = o.bres;
        a.tdir = o.tdir;
        a.talpha = o.talpha;
        a.skip = o.skip;
        a.write_resid = o.write_resid ? 1 : 0;
        const int NC = fwd_nc_bucket(nc);
        const int seg = fwd_seg_for(ctx, g, b, NC);
        dim3 grid((unsigned)(V * nchunks), (unsigned)((nc + NC - 1) / NC));
        // every output of the kernel is a function of the packs and angles only, so repeated
        // timing launches leave the result unchanged
        const int reps = timing_reps(ctx, 0, true);
        // per-launch accumulation times full one-column projections only
        const bool eligible = ncols == 1 && proj && !mom && !red && o.skip == nullptr;
        timing_mark(ctx, 0, 0, s, eligible);
        for (int rep = 0; rep < reps; ++rep) {
            if (proj && mom) launch_fwd_mode<3>(NC, seg, grid, a, s);
            else if (mom) launch_fwd_mode<2>(NC, seg, grid, a, s);
            else launch_fwd_mode<1>(NC, seg, grid, a, s);
        }
        timing_mark(ctx, 0, 1, s);
    }
    if (red && (o.gdot || o.dnorm2 || o.rnorm2) && !o.keep_parts) {
        const int64_t n = (int64_t)ncols * V;
        finalize_parts_k<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(part, ncols, V, nchunks,
                                                                     o.gdot, o.dnorm2, o.rnorm2,
                                                                     o.skip);
    }
    NLRMM_HIP_CHECK(hipGetLastError());
    return NLRMM_OK;
}

int fwd_chunks(const nlrmm_geom &g) { return (g.nbins + BINS - 1) / BINS; }

size_t fwd_workspace_bytes(const nlrmm_geom &g, int nframes, int ncols)
{
    const int gcols = ncols < 8 ? ncols : 8;
    return fwd_ws_bytes(g, nframes, gcols, 1, 1, 0);
}

int fwd_nc_bucket(int nc) { return nc >= 8 ? 8 : nc >= 4 ? 4 : nc >= 2 ? 2 : 1; }

int fwd_seg_for(const nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int nc_bucket)
{
    if (ctx->force_fwd_seg) return ctx->force_fwd_seg;
    const int t = tune_lookup(ctx, TUNE_FWD_SEG, g, b, nc_bucket);
    return t ? t : FSEG_DEFAULT;
}

// Largest view split: at most 16 partial images, at least 16 views per split and frame.
int bwd_split_max(const nlrmm_geom &, const nlrmm_batch &b)
{
    int64_t ns = (b.nviews / b.nframes) / 16;
    if (ns > 16) ns = 16;
    if (ns < 1) ns = 1;
    return (int)ns;
}

// Default view split (without a tuned choice): about 6 resident waves per SIMD.
int bwd_splits(const nlrmm_geom &g, const nlrmm_batch &b, int ncols, int cu_count)
{
    const int64_t tiles = (int64_t)((g.nx + TILE - 1) / TILE) * ((g.ny + TILE - 1) / TILE);
    const int64_t waves = tiles * ncols * b.nframes * (BWD_BLK / 64);
    const int64_t target = (int64_t)6 * 4 * cu_count;   // ~6 resident waves per SIMD
    int64_t ns = (target + waves - 1) / waves;
    const int64_t vper = b.nviews / b.nframes;
    if (ns > vper / 16) ns = vper / 16;
    if (ns > 16) ns = 16;
    if (ns < 1) ns = 1;
    return (int)ns;
}

// Partial images of a view split of `nsplit` (none for a single split).
static size_t bwd_part_bytes(const nlrmm_geom &g, const nlrmm_batch &b, int ncols, int nsplit)
{
    if (nsplit <= 1) return 0;
    return sizeof(float) * (size_t)nsplit * ncols * b.nframes * g.nx * g.ny;
}

// Workspace bound of any view split the backprojection may use for this shape: every split
// it launches is clamped to bwd_split_max (bwd_split_for), and the default never exceeds it.
size_t bwd_workspace_bytes(const nlrmm_geom &g, const nlrmm_batch &b, int ncols, int)
{
    return bwd_part_bytes(g, b, ncols, bwd_split_max(g, b));
}

// View split of one backprojection launch: the split forced by the autotuner, else the tuned
// choice for this shape, else the default; clamped to [1, bwd_split_max] whatever its source
// (a tune file may hold a choice made for another device or library version).
int bwd_split_for(const nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols)
{
    int ns = ctx->force_bwd_split;
    if (ns <= 0) ns = tune_lookup(ctx, TUNE_BWD_SPLIT, g, b, ncols);
    if (ns <= 0) ns = bwd_splits(g, b, ncols, ctx->cu_count);
    const int mx = bwd_split_max(g, b);
    if (ns > mx) ns = mx;
    if (ns < 1) ns = 1;
    return ns;
}

int launch_backproject_dtheta(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b,
                              int ncols, const float *y, const double *theta, float *x,
                              hipStream_t s)
{
    if (!bwd_geom_ok(g)) return NLRMM_ESHAPE;
    const int E = edges_inside(g);
    const int W = bwd_window(g);
    BwdArgs a;
    a.y = y;
    a.theta = theta;
    a.view_off = b.view_off;
    a.nframes = b.nframes;
    a.V = b.nviews;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nb = g.nbins;
    a.x0 = g.x0;
    a.y0 = g.y0;
    a.d = g.d;
    a.s0 = g.s0;
    a.ds = g.ds;
    a.tiles_x = (g.nx + TILE - 1) / TILE;
    a.W = W;
    a.x = x;
    // the backprojection's view split for this shape
    a.nsplit = bwd_split_for(ctx, g, b, ncols);
    a.part = nullptr;
    a.accumulate = 0;
    a.tv = TvEpilogue();
    if (a.nsplit > 1) {
        int rc = ensure_workspace(ctx, bwd_part_bytes(g, b, ncols, a.nsplit), s);
        if (rc) return rc;
        a.part = (float *)ctx->ws.ptr;
    }
    const int tiles_y = (g.ny + TILE - 1) / TILE;
    dim3 grid((unsigned)(a.tiles_x * tiles_y), (unsigned)((int64_t)ncols * b.nframes),
              (unsigned)a.nsplit);
    switch (E) {
        case 1: bwd_moment_tiles_k<1><<<grid, MOM_BLK, 0, s>>>(a); break;
        case 2: bwd_moment_tiles_k<2><<<grid, MOM_BLK, 0, s>>>(a); break;
        case 3: bwd_moment_tiles_k<3><<<grid, MOM_BLK, 0, s>>>(a); break;
        default: bwd_moment_tiles_k<4><<<grid, MOM_BLK, 0, s>>>(a); break;
    }
    if (a.nsplit > 1) {
        const int64_t n = (int64_t)ncols * b.nframes * g.nx * g.ny;
        sum_splits_k<false><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
            a.part, a.nsplit, n, x, 0, a.tv, g.nx, g.ny, b.nframes, MdDev{});
    }
    NLRMM_HIP_CHECK(hipGetLastError());
    return NLRMM_OK;
}

int launch_backproject(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols,
                       const float *y, const double *theta, float *x, hipStream_t s,
                       int accumulate, const TvEpilogue *tv, MdEpilogue *md)
{
    return launch_backproject_into(ctx, g, b, ncols, y, theta, x, s, accumulate, tv, nullptr, 0,
                                   md);
}

size_t bwd_split_bytes(const nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols)
{
    return bwd_part_bytes(g, b, ncols, bwd_split_for(ctx, g, b, ncols));
}

int launch_backproject_into(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols,
                            const float *y, const double *theta, float *x, hipStream_t s,
                            int accumulate, const TvEpilogue *tv, float *part_buf,
                            size_t part_cap, MdEpilogue *md)
{
    if (md) {
        md->fused = false;
        md->nblk = 0;
    }
    if (tv && tv->u && ncols != 1) return NLRMM_ENOTSUP;
    if (!bwd_geom_ok(g)) return NLRMM_ESHAPE;
    const int E = edges_inside(g);
    const int W = bwd_window(g);
    BwdArgs a;
    a.y = y;
    a.theta = theta;
    a.view_off = b.view_off;
    a.nframes = b.nframes;
    a.V = b.nviews;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nb = g.nbins;
    a.x0 = g.x0;
    a.y0 = g.y0;
    a.d = g.d;
    a.s0 = g.s0;
    a.ds = g.ds;
    a.tiles_x = (g.nx + TILE - 1) / TILE;
    a.W = W;
    a.x = x;
    a.nsplit = bwd_split_for(ctx, g, b, ncols);
    a.part = nullptr;
    a.accumulate = accumulate;
    a.tv = tv ? *tv : TvEpilogue();
    if (a.nsplit > 1) {
        const size_t need = bwd_part_bytes(g, b, ncols, a.nsplit);
        if (part_buf) {
            // caller-provided partial images (never grown here)
            if (need > part_cap) return NLRMM_ESHAPE;
            a.part = part_buf;
        } else {
            int rc = ensure_workspace(ctx, need, s);
            if (rc) return rc;
            a.part = (float *)ctx->ws.ptr;
        }
    }
    const int tiles_y = (g.ny + TILE - 1) / TILE;
    dim3 grid((unsigned)(a.tiles_x * tiles_y), (unsigned)((int64_t)ncols * b.nframes),
              (unsigned)a.nsplit);
    // repeated timing launches are harmless unless the kernel adds into x itself
    const int reps = timing_reps(ctx, 1, a.nsplit > 1 || (!accumulate && a.tv.u == nullptr));
    timing_mark(ctx, 1, 0, s, ncols == 1);
    for (int rep = 0; rep < reps; ++rep) {
        switch (E) {
            case 1: bwd_tiles_k<1, BWD_PX><<<grid, BWD_BLK, sizeof(float2) * VCHUNK * a.W, s>>>(a); break;
            case 2: bwd_tiles_k<2, BWD_PX><<<grid, BWD_BLK, sizeof(float2) * VCHUNK * a.W, s>>>(a); break;
            case 3: bwd_tiles_k<3, BWD_PX><<<grid, BWD_BLK, sizeof(float2) * VCHUNK * a.W, s>>>(a); break;
            default: bwd_tiles_k<4, BWD_PX><<<grid, BWD_BLK, sizeof(float2) * VCHUNK * a.W, s>>>(a); break;
        }
    }
    timing_mark(ctx, 1, 1, s);
    if (a.nsplit > 1) {
        const int64_t n = (int64_t)ncols * b.nframes * g.nx * g.ny;
        const int64_t nblk = (n + 255) / 256;
        if (md && md->X && ncols == 1 && nblk <= md->nblk_cap && md->nv >= 1 &&
            md->nv + 1 <= md::MD_MAX) {
            sum_splits_k<true><<<(unsigned)nblk, 256, 0, s>>>(
                a.part, a.nsplit, n, x, accumulate, a.tv, g.nx, g.ny, b.nframes,
                MdDev{md->X, md->ldx, md->nv, md->part});
            md->fused = true;
            md->nblk = (int)nblk;
        } else {
            sum_splits_k<false><<<(unsigned)nblk, 256, 0, s>>>(
                a.part, a.nsplit, n, x, accumulate, a.tv, g.nx, g.ny, b.nframes, MdDev{});
        }
    }
    NLRMM_HIP_CHECK(hipGetLastError());
    return NLRMM_OK;
}

}  // namespace nlrmm
