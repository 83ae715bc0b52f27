// Register-resident single-wave FP64 kernels of the projected problem (padded size NB):
// the discrepancy-principle solve of eq. "reduced_problem" (Section 3.2) and the
// eigen-decomposition of the recycling compression (Alg. "compress").  The kernels are
// templates over the padded size; each size is instantiated in one of the solve_reg_*.hip
// translation units (they compile slowly, so the sizes are spread over several units).
#pragma once
#include "internal.h"
#include "wave.h"

#include <math.h>

#include <type_traits>

namespace nlrmm {
namespace reg {

using wave::lane_bcast;
using wave::wave_sum_dpp;

// Register-resident form of the same solve.  One wave; lane i keeps row i of the working
// matrix in VGPRs, the problem is padded to NB (GA with the identity, GP with zeros, which
// leaves every quantity of the first ell rows unchanged), and all loops over the padded size
// are unrolled so that every register index is static.  Column broadcasts go through LDS
// (one write, then broadcast reads), wave sums through DPP.  The discrepancy residual uses
// continuants of I + lam T (no divisions):
//   P_n = 1, P_{n+1} = 0, P_k = (1 + lam d_k) P_{k+1} - lam^2 e_k^2 P_{k+2},
//   S_n = 0, S_k = lam^2 e_{k-1}^2 (P_{k+1}^2 + S_{k+1}),
//   ||AV z(lam) - b||^2 = out2 + ||c||^2 (Q^2 + S_1) / P_0^2,  Q = lam d_0 P_1 - lam^2 e_0^2 P_2,
// where Q / P_1 = D_0 - 1 and S_1 / P_1^2 = sum_{i>=1} (y_i / y_0)^2 in the notation above;
// P, S are rescaled by powers of two so that they stay in range.
// Compile-time loop: calls f(std::integral_constant<int, I>) for I = B .. E-1, so that loop
// bodies too large for the unroller still see constant register indices.
template <int B, int E>
struct StaticFor {
    template <class F>
    static __device__ __forceinline__ void run(F &&f)
    {
        f(std::integral_constant<int, B>{});
        StaticFor<B + 1, E>::run(f);
    }
};
template <int E>
struct StaticFor<E, E> {
    template <class F>
    static __device__ __forceinline__ void run(F &&)
    {
    }
};

// Empty register pins: force every element of a register array to be materialised here, so
// that the compiler does not sink the updates of one elimination step into later steps (which
// keeps the broadcast operands of all steps live at once).
template <int NB>
__device__ __forceinline__ void pin_regs(double (&v)[NB])
{
#pragma unroll
    for (int k = 0; k < NB; ++k) asm volatile("" : "+v"(v[k]));
}

// The kernels here run as a single wave (one 64-lane workgroup).  The LDS operations of a wave
// complete in program order, so a compiler-level wave barrier (no s_barrier, no wait for
// outstanding memory operations) is enough to order the lanes' exchanges through LDS.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// Reciprocal to full double precision: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// X <- L^-1 X for the column held by this lane (p[c] = X[c][lane]); L from the LDS copy
// sLt[k * LD + c] = L[c][k] with reciprocal diagonal sdi.  The next step's broadcast column is
// loaded while the current step's updates run.
template <int NB, int LD>
__device__ __forceinline__ void lower_solve_cols(double (&p)[NB], const double *sLt,
                                                 const double *sdi)
{
    double lc[NB];
#pragma unroll
    for (int c = 1; c < NB; ++c) lc[c] = sLt[c];
    StaticFor<0, NB>::run([&](auto K) __attribute__((always_inline)) {
        constexpr int k = decltype(K)::value;
        double ln[NB];
#pragma unroll
        for (int c = k + 2; c < NB; ++c) ln[c] = sLt[(k + 1) * LD + c];
        const double dk = sdi[k];
        p[k] *= dk;
#pragma unroll
        for (int c = k + 1; c < NB; ++c) p[c] = fma(-lc[c], p[k], p[c]);
#pragma unroll
        for (int c = k + 2; c < NB; ++c) lc[c] = ln[c];
        pin_regs(p);
    });
}

// One Householder step of the tridiagonalisation (column J), with J a compile-time constant so
// that every register index stays static (the step is too large for the loop unroller).
template <int J, int NB>
__device__ __forceinline__ void tri_step(double (&p)[NB], int lane, double *sv, double *sw,
                                         double *sdd, double *see, double *stau)
{
    constexpr int j = J;
    const double xi = (lane > j) ? p[j] : 0.0;
    const double s2 = wave_sum_dpp(xi * xi);
    const double x0 = lane_bcast(p[j], j + 1);
    const double dj = lane_bcast(p[j], j);
    const double tail = s2 - x0 * x0;
    // no branches: every step is straight-line code (a step without a reflector has v = 0,
    // tau = 0 and leaves p unchanged), so the steps schedule as one block
    const bool refl = tail > 0.0;
    const double sigma = sqrt(s2);
    const double alpha = refl ? ((x0 >= 0.0) ? -sigma : sigma) : x0;
    const double v0 = refl ? x0 - alpha : 0.0;
    const double tj = refl ? 2.0 * rcp_nr(tail + v0 * v0) : 0.0;
    sdd[j] = dj;
    see[j] = alpha;
    stau[j] = tj;
    const double vi = (tj != 0.0 && lane > j) ? ((lane == j + 1) ? v0 : xi) : 0.0;
    {
        sv[lane] = vi;
        wave_sync();
        double vc[NB];
#pragma unroll
        for (int c = j + 1; c < NB; ++c) vc[c] = sv[c];
        __builtin_amdgcn_sched_barrier(0);
        double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = j + 1; c < NB; ++c) q[c & 3] = fma(p[c], vc[c], q[c & 3]);
        const double pi = tj * ((q[0] + q[1]) + (q[2] + q[3]));
        const double mu = 0.5 * tj * wave_sum_dpp(pi * vi);
        const double wi = pi - mu * vi;
        sw[lane] = wi;
        wave_sync();
        double wc[NB];
#pragma unroll
        for (int c = j + 1; c < NB; ++c) wc[c] = sw[c];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = j + 1; c < NB; ++c) p[c] -= vi * wc[c] + wi * vc[c];
        pin_regs(p);
        wave_sync();
    }
    p[j] = vi;
}

template <int J, int NB, bool DONE = (J + 2 >= NB)>
struct TriSteps {
    static __device__ __forceinline__ void run(double (&p)[NB], int lane, double *sv, double *sw,
                                               double *sdd, double *see, double *stau)
    {
        tri_step<J, NB>(p, lane, sv, sw, sdd, see, stau);
        TriSteps<J + 1, NB>::run(p, lane, sv, sw, sdd, see, stau);
    }
};
template <int J, int NB>
struct TriSteps<J, NB, true> {
    static __device__ __forceinline__ void run(double (&)[NB], int, double *, double *, double *,
                                               double *, double *)
    {
    }
};

// ||AV z(lam) - b||^2 from the continuants of I + lam T (see gks_solve_reg_k); e2 holds the
// squared off-diagonal, l2 = lam^2.  lam^2 e_{k-1}^2 of one step is lam^2 e_k^2 of the next,
// so a step costs seven FP64 operations.  P is non-decreasing (the pivots of I + lam T are
// >= 1) and grows by at most 1 + lam ||T|| per step (below 2^91 within the search bracket
// even for Grams near singularity), so P and S ~ P^2 are rescaled by powers of two, without
// a branch, every fourth step once |P| exceeds 2^100 (P < 2^470, S < 2^940).
template <int NB>
__device__ __forceinline__ double dp_residual(double lam, double l2, const double (&dd)[NB],
                                              const double (&e2)[NB], double out2, double cn2)
{
    double P2 = 0.0, P1 = 1.0, S = 0.0;
    double t = l2 * e2[NB - 1];   // lam^2 e_k^2 of the current step
#pragma unroll
    for (int k = NB - 1; k >= 1; --k) {
        const double tm = l2 * e2[k - 1];
        const double Pk = fma(fma(lam, dd[k], 1.0), P1, -t * P2);
        P2 = P1;
        P1 = Pk;
        S = fma(tm, S, tm * (P2 * P2));
        t = tm;
        if ((k & 3) == 0) {
            const double sc = fabs(P1) > 0x1p100 ? 0x1p-100 : 1.0;
            P1 *= sc;
            P2 *= sc;
            S *= sc * sc;
        }
    }
    const double Q = fma(lam * dd[0], P1, -t * P2);
    const double P0 = P1 + Q;
    return out2 + cn2 * (fma(Q, Q, S) / (P0 * P0));
}

template <int NB, bool INC>
__global__ __launch_bounds__(64) void gks_solve_reg_k(const double *__restrict__ GA,
                                                     const double *__restrict__ GP, int ldg,
                                                     const double *__restrict__ rb,
                                                     const double *__restrict__ scal, int ell,
                                                     double lam_fix, double *__restrict__ z,
                                                     double *__restrict__ out,
                                                     int *__restrict__ status,
                                                     double *__restrict__ Lst)
{
    constexpr int LD = NB + 2;
    __shared__ double sLt[NB * LD];   // sLt[k * LD + c] = L[c][k]
    __shared__ double sX[NB * LD];    // transposes
    __shared__ double sv[64], sw[64], sc[64], sdd[64], see[64], sy[64], sdi[64], stau[64];
    const int n = ell;
    const int lane = threadIdx.x;
    const bool row = lane < NB;
    // both diagonals' loads in flight together (unconditional, lanes past n read entry 0)
    const int ld = lane < n ? lane : 0;
    const double gad = GA[ld * ldg + ld], gpd = GP[ld * ldg + ld];
    const double trA = wave_sum_dpp(lane < n ? gad : 0.0);
    const double trP = wave_sum_dpp(lane < n ? gpd : 0.0);
    double a[NB], p[NB];
    int bad = 0;
    // L (rows, lane i = row i) and its reciprocal diagonal are kept in Lst[i * ldg + k] and
    // Lst[ldg * ldg + i] for the next solve.  INC: Lst holds the factor of the leading
    // ell - 1 rows and columns of this GA (the previous solve's, before one row and column
    // were appended), so only the new row is formed (a kernel of its own: one straight path
    // keeps the row in registers).
    double *const Ldi = Lst != nullptr ? Lst + (int64_t)ldg * ldg : nullptr;
    if constexpr (INC) {
        // New row by forward substitution x = L^-1 g, g = GA[ell-1][0..ell-2]: lane k holds row
        // k of L, its g_k, its reciprocal diagonal and the running sum s_k; step j takes x_j
        // = (g_j - s_j) / L_jj from lane j and every lane adds L_kj x_j.  Lane ell-1 collects
        // the x_j (its row) and their squares, so at step ell-1 its own value is the pivot
        // g_nn - sum x_j^2; the steps beyond are identity rows (x = 0).  No branches: the row
        // stays in registers.
        const int nm = n - 1;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            a[c] = (lane < nm && c < nm) ? Lst[lane * ldg + c] : ((lane >= n && lane == c) ? 1.0 : 0.0);
        const double g = lane < n ? GA[lane * ldg + nm] : 0.0;
        const double inv = lane < nm ? Ldi[lane] : 1.0;
        double acc = 0.0, piv = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const double xj = lane_bcast((g - acc) * inv, j);
            piv = (j == nm) ? xj : piv;
            a[j] = (lane == nm && j < nm) ? xj : a[j];
            acc = fma(a[j], xj, acc);
        }
        if (!(piv > 0.0)) {
            bad = 1;
            piv = 1e-300;
        }
        const double d = sqrt(piv);
        const double di = rcp_nr(d);
#pragma unroll
        for (int j = 0; j < NB; ++j) a[j] = (lane == nm && j == nm) ? d : a[j];
        sdi[lane] = lane < nm ? inv : (lane == nm ? di : 1.0);
        wave_sync();
    } else {
#pragma unroll
        for (int c = 0; c < NB; ++c)
            a[c] = (lane < n && c < n) ? GA[lane * ldg + c] : (lane == c ? 1.0 : 0.0);
        // 1. Cholesky GA = L L^T (lane i ends with row i of L; its upper part is never read).
        //    The unscaled column is broadcast while the pivot reciprocal is formed, and the
        //    update uses A_ij A_kj / pivot, so the square root stays off the dependency chain.
        StaticFor<0, NB>::run([&](auto J) __attribute__((always_inline)) {
            constexpr int j = decltype(J)::value;
            sv[lane] = a[j];
            wave_sync();
            double lc[NB];
    #pragma unroll
            for (int k = j + 1; k < NB; ++k) lc[k] = sv[k];
            double piv = lane_bcast(a[j], j);
            if (!(piv > 0.0)) {
                bad = 1;
                piv = 1e-300;
            }
            const double r = rcp_nr(piv);
            __builtin_amdgcn_sched_barrier(0);
            const double t = a[j] * r;
    #pragma unroll
            for (int k = j + 1; k < NB; ++k) a[k] = fma(-t, lc[k], a[k]);
            const double d = sqrt(piv);
            const double di = rcp_nr(d);
            a[j] = (lane == j) ? d : a[j] * di;
            sdi[j] = di;
            pin_regs(a);
            wave_sync();
        });
    }
    if (Lst != nullptr) {
        // this factor for the next solve (only the new row when it was appended)
        if (lane < n && (!INC || lane == n - 1)) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < n) Lst[lane * ldg + c] = a[c];
        }
        if (lane < n) Ldi[lane] = sdi[lane];
    }
    if (row) {
#pragma unroll
        for (int k = 0; k < NB; ++k) sLt[k * LD + lane] = a[k];
    }
    // lane i < ell: row i of GP (= column i); lane ell: rb
#pragma unroll
    for (int c = 0; c < NB; ++c)
        p[c] = (lane < n && c < n) ? GP[lane * ldg + c] : ((lane == n && c < n) ? rb[c] : 0.0);
    wave_sync();
    // 2. K = L^-1 GP L^-T: column-wise forward substitutions, transposes through LDS
    lower_solve_cols<NB, LD>(p, sLt, sdi);
    if (lane == n) {
#pragma unroll
        for (int k = 0; k < NB; ++k) sc[k] = p[k];   // c = L^-1 rb
    }
    if (row) {
#pragma unroll
        for (int k = 0; k < NB; ++k) sX[k * LD + lane] = (lane < n) ? p[k] : 0.0;
    }
    wave_sync();
#pragma unroll
    for (int c = 0; c < NB; ++c) p[c] = row ? sX[lane * LD + c] : 0.0;
    wave_sync();
    lower_solve_cols<NB, LD>(p, sLt, sdi);
    if (row) {
#pragma unroll
        for (int c = 0; c < NB; ++c) sX[c * LD + lane] = p[c];
    }
    wave_sync();
#pragma unroll
    for (int c = 0; c < NB; ++c) p[c] = row ? 0.5 * (p[c] + sX[lane * LD + c]) : 0.0;
    // 3. reflector H0 with H0 c = s ||c|| e1; K <- H0 K H0
    const double cl = (lane < n) ? sc[lane] : 0.0;
    const double cn2 = wave_sum_dpp(cl * cl);
    const double cn = sqrt(cn2);
    const double out2 = fmax(scal[0] - cn2, 0.0);
    const double sgn = (sc[0] >= 0.0) ? -1.0 : 1.0;
    const double hv = cl - ((lane == 0) ? sgn * cn : 0.0);
    const double vtv = wave_sum_dpp(hv * hv);
    const double t0 = vtv > 0.0 ? 2.0 / vtv : 0.0;
    sv[lane] = hv;
    wave_sync();
    {
        double vc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) vc[c] = sv[c];
        __builtin_amdgcn_sched_barrier(0);
        double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < NB; ++c) q[c & 3] = fma(p[c], vc[c], q[c & 3]);
        const double pi = t0 * ((q[0] + q[1]) + (q[2] + q[3]));
        const double mu = 0.5 * t0 * wave_sum_dpp(pi * hv);
        const double wi = pi - mu * hv;
        sw[lane] = wi;
        wave_sync();
        double wc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) wc[c] = sw[c];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < NB; ++c) p[c] -= hv * wc[c] + wi * vc[c];
        pin_regs(p);
        wave_sync();
    }
    // 4. Householder tridiagonalisation; reflector j kept in register j of lanes > j, and
    //    stored to row j of sX at the end (sX is free after step 2)
    TriSteps<0, NB>::run(p, lane, sv, sw, sdd, see, stau);
    {
        const double d2 = lane_bcast(p[NB - 2], NB - 2);
        const double e2 = lane_bcast(p[NB - 2], NB - 1);
        const double d1 = lane_bcast(p[NB - 1], NB - 1);
        sdd[NB - 2] = d2;
        see[NB - 2] = e2;
        sdd[NB - 1] = d1;
        see[NB - 1] = 0.0;
        stau[NB - 2] = 0.0;
        stau[NB - 1] = 0.0;
    }
    if (row) {
#pragma unroll
        for (int j = 0; j + 2 < NB; ++j) sX[j * LD + lane] = (lane > j) ? p[j] : 0.0;
    }
    wave_sync();
    // 5. discrepancy principle.  The padded tail (d = e = 0) leaves P and S unchanged, so the
    //    sweep runs over the whole padded size with T in registers.
    double dd[NB], e2[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        dd[k] = sdd[k];
        e2[k] = see[k] * see[k];
    }
    auto phi = [&](double lam) { return dp_residual<NB>(lam, lam * lam, dd, e2, out2, cn2); };
    const double t2 = scal[1] * scal[1];
    double lam;
    int flag = 0;
    if (lam_fix >= 0.0) {
        lam = lam_fix;
    } else {
        const double scale = trA / fmax(trP, 1e-300);
        double lo = log(1e-10 * scale), hi = log(1e10 * scale);
        // lanes 0 and 1 evaluate the two bracket ends
        const double pe = phi(exp(lane == 0 ? lo : hi));
        const double plo = lane_bcast(pe, 0), phh = lane_bcast(pe, 1);
        if (plo >= t2) {
            lam = exp(lo);
            flag = NLRMM_ST_DP_LOW;
        } else if (phh <= t2) {
            lam = exp(hi);
            flag = NLRMM_ST_DP_HIGH;
        } else {
            // Two rounds on a uniform 65-part grid of the bracket, then rounds on a grid around
            // the regula-falsi point c of the bracket, 32 points on each side: 16 at distances
            // 1.5e-16 max(1, |c|) times powers of two up to a sixteenth of that side's span, 16
            // in equal steps from there to the bracket's end.  The points increase with the
            // lane, so the first lane with f >= 0 (f = residual - target) and its predecessor
            // are the new bracket: it shrinks at least 16-fold per round, superlinearly once c
            // is close, and both ends stay verified values of opposite sign.
            double flo = plo - t2, fhi = phh - t2;
            for (int round = 0; round < 16; ++round) {
                double x;
                if (round < 2) {
                    x = fma(hi - lo, (double)(lane + 1) * (1.0 / 65.0), lo);
                } else {
                    const double c = fma(hi - lo, flo / (flo - fhi), lo);
                    const bool up = lane >= 32;
                    const int idx = up ? lane - 32 : 31 - lane;
                    // innermost points 1.5e-16 |c| away: a bracket found there meets the stop test
                    const double d0 = 1.5e-16 * fmax(1.0, fabs(c));
                    const double span = up ? hi - c : c - lo;
                    const double lin = span * (1.0 / 16.0);
                    double off;
                    if (idx < 16) {
                        const int sh = max(1, (ilogb(lin) - ilogb(d0) + 15) / 15);
                        off = fmin(ldexp(d0, idx * sh), lin);
                    } else {
                        off = lin * (double)(idx - 15);
                    }
                    x = up ? fmin(c + off, hi) : fmax(c - off, lo);
                }
                const double f = phi(exp(x)) - t2;
                const unsigned long long m = __ballot(f >= 0.0);
                const int k = m ? (__ffsll((unsigned long long)m) - 1) : 64;
                if (k < 64) {
                    hi = lane_bcast(x, k);
                    fhi = lane_bcast(f, k);
                }
                if (k > 0) {
                    lo = lane_bcast(x, k - 1);
                    flo = lane_bcast(f, k - 1);
                }
                if (hi - lo <= 4e-16 * fmax(1.0, fabs(lo))) break;
            }
            lam = exp(0.5 * (lo + hi));
        }
    }
    const double res2 = phi(lam);
    // 6. y = (I + lam T)^-1 (s ||c|| e1) from the bottom-up pivots (computed in every lane,
    //    reciprocals kept in sy), then the reflectors in reverse order and H0
    double ee[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) ee[k] = see[k];
    {
        double D = fma(lam, dd[NB - 1], 1.0);
        double r = rcp_nr(D);
        sy[NB - 1] = r;
#pragma unroll
        for (int i = NB - 2; i >= 0; --i) {
            const double b = lam * ee[i];
            D = fma(lam, dd[i], 1.0) - (b * b) * r;
            r = rcp_nr(D);
            sy[i] = r;
        }
    }
    wave_sync();
    double yl;
    {
        double rD[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) rD[i] = sy[i];
        __builtin_amdgcn_sched_barrier(0);
        double y = sgn * cn * rD[0];
        yl = (lane == 0) ? y : 0.0;
#pragma unroll
        for (int i = 1; i < NB; ++i) {
            y = -(lam * ee[i - 1]) * rD[i] * y;
            yl = (lane == i) ? y : yl;
        }
        yl = (lane < n) ? yl : 0.0;
    }
#pragma unroll
    for (int j = NB - 3; j >= 0; --j) {
        // unconditional (tau = 0 leaves y unchanged), so the reflector loads are issued early
        const double tj = stau[j];
        const double vi = row ? sX[j * LD + lane] : 0.0;
        const double dot = wave_sum_dpp(vi * yl);
        yl = fma(-tj * dot, vi, yl);
    }
    {
        const double dot = wave_sum_dpp(hv * yl);
        yl = fma(-t0 * dot, hv, yl);
    }
    // 7. z = L^-T y (lane i reads row i of L^T, i.e. column i of L, once)
    {
        double lr[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) lr[j] = row ? sLt[lane * LD + j] : 0.0;
        double di[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) di[j] = sdi[j];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = NB - 1; j >= 0; --j) {
            const double zj = lane_bcast(yl, j) * di[j];
            if (lane == j) yl = zj;
            else if (lane < j) yl = fma(-lr[j], zj, yl);
        }
    }
    if (lane < n) z[lane] = yl;
    if (lane == 0) {
        out[0] = lam;
        out[1] = res2;
        int st = flag;
        if (bad) st |= NLRMM_ST_NONFINITE;
        if (!isfinite(lam) || !isfinite(res2)) st |= NLRMM_ST_NONFINITE;
        if (st) atomicOr(status, st);
    }
}

// Number of eigenvalues of the symmetric tridiagonal T (diagonal dd, off-diagonal ee) below
// x: sign changes of the leading-minor sequence p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}
// (p_{-1} = 0, p_0 = 1), i.e. the negative pivots of the LDL^T factorisation of T - x I,
// without divisions; the pair (p_i, p_{i-1}) is rescaled by powers of two to stay in range.
template <int NB>
__device__ __forceinline__ int sturm_below(double x, const double (&dd)[NB], const double (&ee)[NB])
{
    double p1 = 1.0, p2 = 0.0;   // p_{i-1}, p_{i-2}
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const double em = i > 0 ? ee[i - 1] : 0.0;
        double p = fma(dd[i] - x, p1, -(em * em) * p2);
        // an exact zero counts as a sign change (x treated as just above the root)
        if ((p < 0.0) != (p1 < 0.0) || p == 0.0) ++cnt;
        if (p == 0.0) p = -copysign(0x1p-600, p1);
        p2 = p1;
        p1 = p;
        if (i & 1) {
            const double m = fmax(fabs(p1), fabs(p2));
            if (m > 0x1p200) {
                p1 *= 0x1p-200;
                p2 *= 0x1p-200;
            } else if (m < 0x1p-200) {
                p1 *= 0x1p200;
                p2 *= 0x1p200;
            }
        }
    }
    return cnt;
}

// Compression in one wave (same result as compress_eig_k): S = GA + lam GP is reduced to a
// tridiagonal T = Q^T S Q (Householder, reflectors kept in registers), the kmin - 1 largest
// eigenvalues of T are found together by Sturm bisection (a group of lanes each), lane t
// computes the eigenvector of
// eigenvalue t by two steps of inverse iteration (LDL^T of T - mu I, pivots perturbed away
// from zero), the vectors are orthonormalised in order (classical Gram-Schmidt, twice) and
// mapped back by Q.  The sign rule, W^T z, the remainder c and the outputs follow
// compress_eig_k.  S is padded to NB with zeros: the padding adds zero eigenvalues below
// the positive ones that are wanted.
template <int NB>
__global__ __launch_bounds__(64) void compress_reg_k(const double *__restrict__ GA,
                                                    const double *__restrict__ GP, int ldg,
                                                    const double *__restrict__ lamp, int ell,
                                                    int kmin, const double *__restrict__ zin,
                                                    double *__restrict__ T, int ldt,
                                                    double *__restrict__ zout,
                                                    int *__restrict__ out_k,
                                                    int *__restrict__ status)
{
    constexpr int LD = NB + 2;
    constexpr int KW = 15;   // kmin - 1 <= 15
    __shared__ double sX[NB * LD];   // symmetrisation, then the reflectors (row j: reflector j)
    __shared__ double sY[16 * LD];   // eigenvectors of T (row t)
    __shared__ double sv[64], sw[64], sdd[64], see[64], stau[64], smu[16], swz[16];
    const int n = ell;
    const int lane = threadIdx.x;
    const bool row = lane < NB;
    const int kw = kmin - 1;
    const double lam = lamp[0];
    double p[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c)
        p[c] = (lane < n && c < n) ? GA[lane * ldg + c] + lam * GP[lane * ldg + c] : 0.0;
    // symmetrise through LDS
    if (row) {
#pragma unroll
        for (int c = 0; c < NB; ++c) sX[c * LD + lane] = p[c];
    }
    wave_sync();
#pragma unroll
    for (int c = 0; c < NB; ++c) p[c] = row ? 0.5 * (p[c] + sX[lane * LD + c]) : 0.0;
    wave_sync();
    // 1. tridiagonalise
    TriSteps<0, NB>::run(p, lane, sv, sw, sdd, see, stau);
    {
        const double d2 = lane_bcast(p[NB - 2], NB - 2);
        const double e2 = lane_bcast(p[NB - 2], NB - 1);
        const double d1 = lane_bcast(p[NB - 1], NB - 1);
        sdd[NB - 2] = d2;
        see[NB - 2] = e2;
        sdd[NB - 1] = d1;
        see[NB - 1] = 0.0;
        stau[NB - 2] = 0.0;
        stau[NB - 1] = 0.0;
    }
    if (row) {
#pragma unroll
        for (int j = 0; j + 2 < NB; ++j) sX[j * LD + lane] = (lane > j) ? p[j] : 0.0;
    }
    wave_sync();
    double dd[NB], ee[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        dd[k] = sdd[k];
        ee[k] = see[k];
    }
    // 2. the kw largest eigenvalues by bisection on Gershgorin bounds
    double glo = 0.0, ghi = 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const double r = fabs(ee[i]) + (i > 0 ? fabs(ee[i - 1]) : 0.0);
        glo = i == 0 ? dd[i] - r : fmin(glo, dd[i] - r);
        ghi = i == 0 ? dd[i] + r : fmax(ghi, dd[i] + r);
    }
    const double span = fmax(ghi - glo, 1e-300);
    glo -= 1e-12 * span;
    ghi += 1e-12 * span;
    {
        // All kw eigenvalues at once: the wave splits into groups of gs lanes (16, 8 or 4),
        // group t bisects the smallest x with #(eig < x) >= NB - t (just above the (t+1)-th
        // largest eigenvalue) on a (gs + 1)-part grid of its own bracket each round.
        const int gs = kw <= 4 ? 16 : (kw <= 8 ? 8 : 4);
        const int grp = lane / gs, li = lane - grp * gs;
        const int need = NB - grp;
        const double step = 1.0 / (double)(gs + 1);
        const unsigned long long gmask = (1ull << gs) - 1;
        double lo = glo, hi = ghi;
        for (int round = 0; round < 48; ++round) {
            const double x = fma(hi - lo, (double)(li + 1) * step, lo);
            const unsigned long long m = __ballot(sturm_below<NB>(x, dd, ee) >= need);
            const unsigned long long bits = (m >> (grp * gs)) & gmask;
            const int k = bits ? (__ffsll(bits) - 1) : gs;
            const double nlo = (k == 0) ? lo : fma(hi - lo, (double)k * step, lo);
            const double nhi = (k == gs) ? hi : fma(hi - lo, (double)(k + 1) * step, lo);
            lo = nlo;
            hi = nhi;
            const bool done = grp >= kw || hi - lo <= 2e-16 * fmax(fabs(lo), fabs(hi));
            if (__ballot(!done) == 0) break;
        }
        if (li == 0 && grp < kw) smu[grp] = 0.5 * (lo + hi);
    }
    wave_sync();
    // 3. inverse iteration, lane t < kw for eigenvalue t (tridiagonal basis)
    double y[NB];
    {
        const double mu = lane < kw ? smu[lane] : 0.0;
        const double tiny = 0x1p-52 * fmax(fabs(mu), span);
        double rq[NB];
        // LDL^T pivots of T - mu I, kept as reciprocals (refined hardware estimates)
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            double v = dd[i] - mu;
            if (i > 0) v -= ee[i - 1] * ee[i - 1] * rq[i - 1];
            if (fabs(v) < tiny) v = v < 0.0 ? -tiny : tiny;
            rq[i] = rcp_nr(v);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) y[i] = i < n ? 1.0 + 1e-3 * i : 0.0;
        for (int it = 0; it < 2; ++it) {
            // solve L D L^T y = y: forward (unit L, l_i = e_{i-1} / q_{i-1}), diagonal, back
#pragma unroll
            for (int i = 1; i < NB; ++i) y[i] -= (ee[i - 1] * rq[i - 1]) * y[i - 1];
#pragma unroll
            for (int i = 0; i < NB; ++i) y[i] *= rq[i];
#pragma unroll
            for (int i = NB - 2; i >= 0; --i) y[i] -= (ee[i] * rq[i]) * y[i + 1];
            double nrm = 0.0;
#pragma unroll
            for (int i = 0; i < NB; ++i) nrm = fma(y[i], y[i], nrm);
            const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
#pragma unroll
            for (int i = 0; i < NB; ++i) y[i] *= inv;
        }
    }
    // 4. vectors to LDS rows sX[t][*]; orthonormalise in order across lanes (component per
    //    lane), classical Gram-Schmidt applied twice
    if (lane < kw) {
#pragma unroll
        for (int i = 0; i < NB; ++i) sY[lane * LD + i] = y[i];
    }
    wave_sync();
    double wv[KW];   // lane i holds component i of every vector
#pragma unroll
    for (int t = 0; t < KW; ++t) wv[t] = (t < kw && row) ? sY[t * LD + lane] : 0.0;
#pragma unroll
    for (int t = 0; t < KW; ++t) {
        if (t < kw) {
            for (int pass = 0; pass < 2; ++pass) {
                double cf[KW];
#pragma unroll
                for (int s2 = 0; s2 < KW; ++s2) cf[s2] = s2 < t ? wave_sum_dpp(wv[s2] * wv[t]) : 0.0;
#pragma unroll
                for (int s2 = 0; s2 < KW; ++s2)
                    if (s2 < t) wv[t] = fma(-cf[s2], wv[s2], wv[t]);
            }
            const double nn = wave_sum_dpp(wv[t] * wv[t]);
            wv[t] *= nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        }
    }
    // 5. back to the basis of S: w = H_1 ... H_{NB-2} y
#pragma unroll
    for (int j = NB - 3; j >= 0; --j) {
        // unconditional (tau = 0 leaves the vectors unchanged)
        const double tj = stau[j];
        const double vi = row ? sX[j * LD + lane] : 0.0;
#pragma unroll
        for (int t = 0; t < KW; ++t) {
            if (t < kw) {
                const double dot = wave_sum_dpp(vi * wv[t]);
                wv[t] = fma(-tj * dot, vi, wv[t]);
            }
        }
    }
    // 6. sign rule (largest magnitude positive, first such index), W^T z, remainder c
    const double zl = lane < n ? zin[lane] : 0.0;
#pragma unroll
    for (int t = 0; t < KW; ++t) {
        if (t < kw) {
            double am = fabs(wv[t]);
            int im = lane;
            for (int off = 32; off > 0; off >>= 1) {
                const double oa = __shfl_xor(am, off, 64);
                const int oi = __shfl_xor(im, off, 64);
                if (oa > am || (oa == am && oi < im)) {
                    am = oa;
                    im = oi;
                }
            }
            const double vm = __shfl(wv[t], im, 64);
            if (vm < 0.0) wv[t] = -wv[t];
            const double wz = wave_sum_dpp(wv[t] * zl);
            if (lane == 0) swz[t] = wz;
            if (lane < n) T[lane * ldt + t] = wv[t];
        }
    }
    wave_sync();
    double cl = zl;
#pragma unroll
    for (int t = 0; t < KW; ++t)
        if (t < kw) cl = fma(-swz[t], wv[t], cl);
    const double cn = sqrt(wave_sum_dpp(cl * cl));
    const double zn = sqrt(wave_sum_dpp(zl * zl));
    const bool keep = cn > 1e-12 * zn;
    if (lane < n) T[lane * ldt + kw] = keep ? cl / cn : 0.0;
    if (lane < kw) zout[lane] = swz[lane];
    if (lane == 0) {
        if (keep) zout[kw] = cn;
        out_k[0] = keep ? kmin : kw;
        int st = keep ? 0 : NLRMM_ST_COMPRESS_SKIP;
        if (!isfinite(cn)) st |= NLRMM_ST_NONFINITE;
        if (st) atomicOr(status, st);
    }
}

template <int NB>
int launch_gks_solve_reg(const double *GA, const double *GP, int ldg, const double *rb,
                         const double *scal, int ell, double lam_fix, double *z, double *out,
                         int *status, hipStream_t s, double *Lst, int linc)
{
    if (linc && (Lst == nullptr || ell < 1)) return NLRMM_EINVAL;
    if (linc)
        gks_solve_reg_k<NB, true><<<1, 64, 0, s>>>(GA, GP, ldg, rb, scal, ell, lam_fix, z, out,
                                                   status, Lst);
    else
        gks_solve_reg_k<NB, false><<<1, 64, 0, s>>>(GA, GP, ldg, rb, scal, ell, lam_fix, z, out,
                                                    status, Lst);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

template <int NB>
int launch_compress_reg(const double *GA, const double *GP, int ldg, const double *lam, int ell,
                        int kmin, const double *z, double *T, int ldt, double *zout, int *kout,
                        int *status, hipStream_t s)
{
    compress_reg_k<NB><<<1, 64, 0, s>>>(GA, GP, ldg, lam, ell, kmin, z, T, ldt, zout, kout,
                                        status);
    return hipGetLastError() == hipSuccess ? NLRMM_OK : NLRMM_EHIP;
}

}  // namespace reg
}  // namespace nlrmm
