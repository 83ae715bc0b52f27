// Launchers of the Krylov-side and Gauss-Newton kernels (krylov.hip, gn.hip).
#pragma once
#include "internal.h"

namespace nlrmm {

// temporal: TEMPORAL_NONE / _DIFF / _OF (tv.h); flow: the velocities of the motion rows
// ([F-1][2][ny][nx]), required with TEMPORAL_OF
int k_psi_weights(const float *u, int nx, int ny, int F, int temporal, float eps, float *w,
                  hipStream_t s, const float *flow = nullptr);
int k_psi_apply(const float *u, int nx, int ny, int F, int temporal, float *out, hipStream_t s,
                const float *flow = nullptr);
// w == nullptr: the weights are formed from u with eps (equal to k_psi_weights' values)
int k_tv_grad_add(const float *u, const float *w, int nx, int ny, int F, int temporal,
                  const double *lamp, float *r, hipStream_t s, float eps = 0.0f);
// A data-Gram column left to the regulariser Gram launch (k_multidot_gram_col's work): the
// inner products <X_i, xnew> (i <= ell, X's column ell being xnew) and <b, xnew> over n
// entries, written as the new row and column ell of the symmetric G and rb[ell].  part holds
// part_cap doubles; md_blocks bounds the blocks of the stand-alone launches.
struct GramColJob {
    const float *X;
    int64_t ldx;
    int ell;
    const float *xnew, *b;
    int64_t n;
    double *part;
    int64_t part_cap;
    int md_blocks;
    double *G;
    int ldg;
    double *rb;
    int cblk;   // blocks of the launch that take the column (set by the launcher)
};
// mode: 0 FP64 VALU, 1 FP32 MFMA, 2 BF16 MFMA (FP32 accumulation per chunk, FP64 across)
// w == nullptr: the weights are formed from u with eps (inside the kernel in modes 1, 2);
// with wout they are also stored there (as k_psi_weights stores them).  col: a pending
// data-Gram column, computed inside this launch and reduced with the Gram (mode 1), or by
// k_multidot_gram_col first (modes 0 and 2, or when its partials do not fit part_cap).
int k_gram_psi(const float *V, int64_t ldv, int ell, const float *w, int nx, int ny, int F,
               int temporal, double *part, int nblk, double *G, int ldg, hipStream_t s,
               int mode = 0, const float *u = nullptr, float eps = 0.0f,
               const float *flow = nullptr, float *wout = nullptr,
               const GramColJob *col = nullptr);
// Optical flow (of.hip).  Velocities of every frame pair of u [F][ny][nx] (SOLVE-OF, eq.
// "of_forward", l2/l2 with a ridge) by `iters` conjugate-gradient steps from zero, into
// flow [F-1][2][ny][nx]; work: of_work_floats(nx, ny, F) floats, part: of_part_doubles(...).
size_t of_work_floats(int nx, int ny, int F);
size_t of_part_doubles(int nx, int ny, int F);
int k_of_estimate(const float *u, int nx, int ny, int F, float gamma, float ridge, int iters,
                  float *flow, float *work, double *part, hipStream_t s);
// r += lam * M_hat^T (w * M_hat u): the motion rows' part of the regulariser gradient (w ==
// nullptr: weights formed from u with eps); acc: F * nx * ny int64 accumulators.
int k_of_grad_add(const float *u, const float *w, const float *flow, int nx, int ny, int F,
                  const double *lamp, float *r, long long *acc, hipStream_t s, float eps);
// part: per-block partials, md_part_doubles(nblk) doubles.
int k_multidot(const float *X, int64_t ldx, int nv, const float *y, const float *z, int64_t n,
               double *part, int nblk, double *out, int ostride, hipStream_t s,
               const int *skip = nullptr);
inline size_t md_part_doubles(int nblk) { return (size_t)nblk * 72; }
int k_gemv(const float *X, int64_t ldx, int nv, const double *c, double beta, const float *a,
           double alpha, int64_t n, float *out, hipStream_t s);
// Two gemv_k jobs in one launch.
int k_gemv2(const float *X0, int64_t ldx0, int nv0, const double *c0, double beta0,
            const float *a0, double alpha0, int64_t n0, float *out0, const float *X1,
            int64_t ldx1, int nv1, const double *c1, double beta1, const float *a1,
            double alpha1, int64_t n1, float *out1, hipStream_t s);
// r <- r - X c, scal[1] = ||r||^2, vout = r / ||r|| with the breakdown test against
// sqrt(scal[0]) (two launches; part holds nblk per-block partials).
int k_gemv_norm_normalize(const float *X, int64_t ldx, int nv, const double *c, float *r,
                          int64_t n, double *part, int nblk, double *scal, double tol,
                          float *vout, int *status, hipStream_t s);
// New row / column ell of the data Gram and rb[ell]: <X_i, xnew> for i <= ell (X's column
// ell is xnew) and <b, xnew>, written straight into G (both triangles) and rb.
int k_multidot_gram_col(const float *X, int64_t ldx, int ell, const float *xnew, const float *b,
                        int64_t n, double *part, int nblk, double *G, int ldg, double *rb,
                        hipStream_t s);
// CGS2 of r against the first nv columns of X and the normalised result into vout (Alg.
// "enlarge"): h1[0..nv-1] = X^T r, h1[nv] = ||r||^2, r -= X h1, h2 = X^T r, r -= X h2,
// vout = r / ||r|| with the breakdown test of k_gemv_norm_normalize.  Four launches (each
// consumer sums its producer's partials itself) while the inner products need at most 512
// blocks, the launch-per-reduction sequence otherwise (the same arithmetic except for the
// order in which the block partials are added).
// part1, part2: md_part_doubles(nblk) doubles each.  p1_blocks > 0: part1 already holds the
// first products <X_i, r>, <r, r> from that many blocks (formed by the launch that wrote r;
// it must be the grid the first launch here would use, at most 512 blocks).
// norm_blocks: the normalisation is left to the caller (k_normalize_red, or the projection's
// packing launch); part1 then holds the squared norm's partials from *norm_blocks blocks.
int k_cgs2(const float *X, int64_t ldx, int nv, float *r, int64_t n, double *part1,
           double *part2, int nblk, double *h1, double *h2, double tol, float *vout,
           int *status, hipStream_t s, int p1_blocks = 0, int *norm_blocks = nullptr);
// vout = r / sqrt(sum of part[0..nblk)), scal[1] = that sum, breakdown test against
// sqrt(scal[0]) (the last launch of k_cgs2).
int k_normalize_red(const float *r, const double *part, int nblk, double *scal, double tol,
                    int64_t n, float *vout, int *status, hipStream_t s);
// Largest producer grid whose partials k_cgs2's consumers sum themselves.
constexpr int CGS2_FUSED_MAXBLK = 512;
// The data Gram from scratch in two launches: G = X^T X (both triangles), rb = X^T b and
// bn2[0] = b^T b for nc <= 10 columns of X (the same values as one multidot per column);
// part: md_part_doubles(nblk) doubles.
int k_gram_cols(const float *X, int64_t ldx, int nc, const float *b, int64_t n, double *part,
                int nblk, double *G, int ldg, double *rb, double *bn2, hipStream_t s);
// precision 0: FP32 operands, FP64 accumulation (vector units); 2: BF16 operands, FP32
// accumulation (matrix cores)
int k_block_update(const float *X, int64_t ldx, int nin, const double *T, int ldt, int kout,
                   int64_t n, float *Y, int64_t ldy, hipStream_t s, int precision = 0);
int k_copy_cols(const float *src, int64_t lds, float *dst, int64_t ldd, int ncols, int64_t n,
                hipStream_t s);
int k_normalize_into(const float *r, const double *scal, double tol, int64_t n, float *vout,
                     int *status, double *norm_out, hipStream_t s);
// method: 0 Jacobi eigen-decomposition (4 waves), 1 register-resident tridiagonal form,
// 2 LDS tridiagonal form
// Lst (method 1 only; ldg * ldg + ldg doubles): receives the Cholesky factor of GA and its
// reciprocal diagonal; linc: it holds them for the leading ell - 1 rows and columns of this GA
// (one row and column appended since), so only the new row is formed.
int k_gks_solve(const double *GA, const double *GP, int ldg, const double *rb, const double *scal,
                int ell, double lam_fix, double *z, double *out, int *status, hipStream_t s,
                int method = 1, double *Lst = nullptr, int linc = 0);
// method: 0 Jacobi (4 waves), 1 tridiagonal + Sturm bisection + inverse iteration (1 wave)
int k_compress_eig(const double *GA, const double *GP, int ldg, const double *lam, int ell,
                   int kmin, const double *z, double *T, int ldt, double *zout, int *kout,
                   int *status, hipStream_t s, int method = 1);
int k_gram_transform(double *G, int ldg, double *rb, int ell, const double *T, int ldt,
                     const int *kp, hipStream_t s);

// small device helpers (gn.hip)
int k_scatter_gram(const double *col, int ell, double *G, int ldg, double *rb, hipStream_t s);
int k_symmetrize(double *G, int ldg, int ell, hipStream_t s);
int k_copy_f64(const double *src, double *dst, int64_t n, hipStream_t s);
int k_gn_prepare(const double *g, const double *h, const double *rn2, int64_t V, int scalar_mode,
                 double mu_rel, double *dir, double *sc, int *accepted, hipStream_t s);
int k_armijo_check(const double *part_r, int64_t nparts, const double *alphas, int q, double c1,
                   double *sc, int *accepted, hipStream_t s);
int k_gn_apply(double *theta, const double *dir, int64_t V, const double *sc,
               const int *accepted, int *status, hipStream_t s);
int k_fill_f64(double *dst, int64_t n, double value, hipStream_t s);
int k_cg_coef(double *c, int mode, hipStream_t s);
int k_offset_gn(const double *d1, const double *d2, const double *lamp, double *out,
                hipStream_t s);
int k_grid_residual(const double *G, int ldg, const double *rb, const double *bnorm2, int ell,
                    double *res2, hipStream_t s);
int k_grid_pick(const double *res2, int ncand, const double *shifts, double *theta, int64_t V,
                int *best, hipStream_t s);
int k_fill_i32(int *dst, int64_t n, int value, hipStream_t s);
int k_fill_f32(float *dst, int64_t n, float value, hipStream_t s);
int k_offset_dir(const double *gh, double mu_rel, int64_t V, double *dir, double *sc,
                 hipStream_t s);
int k_lin_image(const float *u, const float *up, int64_t n, const double *alphas, int q,
                const double *dir, const int *accepted, float *out, hipStream_t s);
int k_sens_objective(const double *rn2, int64_t V, const double *reg, const double *lamp,
                     const double *alphas, int q, double c1, double *sc, int *accepted,
                     hipStream_t s);
int k_view_dots(const float *X, int64_t ldx, int k, const float *e, int nb, int64_t V, double *out,
                hipStream_t s);
int k_varpro_reduced(const double *GA, int ldg, const double *GP, const double *ab,
                     const double *lamp, const double *bn2, int k, double *yout, double *Mout,
                     double *sc, const double *alphas, int trial, double c1, int *accepted,
                     int *status, hipStream_t s);
int k_varpro_dir(const double *M, int k, const double *gd, const double *en2, const double *ETr,
                 const double *Ate, int64_t V, double mu_rel, double *Yw, double *dir, double *sc,
                 int *status, hipStream_t s);
int k_scale_into(const float *src, const double *norm2, int64_t n, float *dst, double *norm_out,
                 int *status, hipStream_t s);

}  // namespace nlrmm
