// Native driver of NL-RMM-GKS on one device stream (Alg. "nl_rmmgks_two_solves" with the
// high-regularisation solve off, Alg. "rmmgks" with one Enlarge/Compress cycle per outer
// iteration, Alg. "update_param" for the angles).  Every decision (lambda, breakdown,
// compression size, Armijo step) is taken by device kernels; the host only sequences
// launches, so an outer iteration can be captured in a HIP graph and replayed.
//
// Basis storage: V [kmax+1][n] and A V [kmax+1][m] column-contiguous FP32; Psi V is not
// stored (the weighted regulariser Gram recomputes Psi v from V on the fly).  Small
// projected quantities (Grams, coefficients, lambda) live on the device in FP64.
#include "internal.h"
#include "krylov.h"
#include "tv.h"

#include <math.h>
#include <new>
#include <vector>

namespace nlrmm {

enum {
    S_BNORM2 = 0,   // ||b||^2
    S_TARGET = 1,   // tau * delta
    S_LAM = 2,      // lambda of the last projected solve
    S_RES2 = 3,     // model residual ||AVz - b||^2 of the last solve
    S_LAMK = 4,     // lambda_k of the primary solve while the high-regularisation solve runs
    S_GN = 8,       // [f0, g^T d, alpha, mu, f_accepted] of the last Gauss-Newton step
    S_NB = 16,      // scalars
};

// Largest image (pixels times frames) whose IRN weights the Gram launch forms itself; larger
// ones get them from their own launch first.
constexpr int64_t GRAM_FUSED_WEIGHTS_MAX = int64_t(1) << 19;

struct Solver {
    nlrmm_ctx *ctx = nullptr;
    nlrmm_geom g{};
    int F = 1;
    int64_t maxV = 0;
    nlrmm_solver_cfg cfg{};
    int64_t n = 0, npsi = 0, mmax = 0;
    int kcap = 0;   // kmax + 1 columns
    int ld = 0;     // Gram leading dimension
    int ell = 0;    // current number of basis columns (host bookkeeping)
    int md_blocks = 512, gram_blocks = 512, nchunks = 1;
    bool rho_ready = false;   // rho = A V z - b already formed for the next residual
    bool w_from_u = true;     // weights of u may be formed on the fly (false: caller's w)
    // device buffers
    float *V = nullptr, *AV = nullptr, *Vtmp = nullptr, *u = nullptr, *r = nullptr,
          *rho = nullptr, *w = nullptr, *uh = nullptr;
    double *zh = nullptr;   // coefficients of the high-regularisation solve
    double *cgs = nullptr;  // scalars of the sensitivity solve
    double *GA = nullptr, *GP = nullptr, *rb = nullptr, *z = nullptr, *T = nullptr,
           *zt = nullptr, *sc = nullptr, *hb = nullptr, *hb2 = nullptr, *gv = nullptr,
           *hv = nullptr, *rv = nullptr, *dir = nullptr, *alphas = nullptr, *thk = nullptr,
           *part_md = nullptr, *part_md2 = nullptr, *part_gram = nullptr, *part_fwd = nullptr,
           *gkb = nullptr;
    // a data-Gram column whose reduction the next regulariser Gram launch completes
    GramColJob gc{};
    bool gc_pending = false;
    // Cholesky factor of GA kept between projected solves (ld * ld + ld doubles): valid for
    // l_ell columns; ga_appended: an expansion appended one row and column since
    double *Lst = nullptr;
    int l_ell = 0;
    bool ga_appended = false;
    // VarPro buffers
    float *Ahat = nullptr, *evec = nullptr;
    double *vp_GA = nullptr, *vp_ab = nullptr, *vp_M = nullptr, *vp_y = nullptr, *vp_gd = nullptr,
           *vp_en2 = nullptr, *vp_ETr = nullptr, *vp_Ate = nullptr, *vp_Y = nullptr;
    int *status = nullptr, *kout = nullptr, *accepted = nullptr;
    // optical-flow regulariser (temporal mode 2): velocities of the frame pairs, the
    // conjugate-gradient work of their estimation, the fixed-point accumulators of the motion
    // rows' transpose; outer iterations run (the velocity update period)
    float *flow = nullptr, *of_work = nullptr;
    double *of_part = nullptr;
    long long *of_acc = nullptr;
    int64_t outer_count = 0;
    std::vector<void *> allocs;
    // plain mode: one launch per frame (and per column) instead of one batched launch
    int plain = 0;
    std::vector<int64_t> vo_host;

    template <typename T_>
    int alloc(T_ **p, size_t count)
    {
        void *q = nullptr;
        if (hipMalloc(&q, sizeof(T_) * (count ? count : 1)) != hipSuccess) {
            (void)hipGetLastError();
            return NLRMM_ENOMEM;
        }
        allocs.push_back(q);
        *p = (T_ *)q;
        return NLRMM_OK;
    }
    ~Solver()
    {
        if (!allocs.empty()) (void)hipDeviceSynchronize();
        for (void *p : allocs) (void)hipFree(p);
    }
};

}  // namespace nlrmm

struct nlrmm_solver : nlrmm::Solver {};

namespace nlrmm {

#define RC(x)                      \
    do {                           \
        int _rc = (x);             \
        if (_rc) return _rc;       \
    } while (0)

static int64_t m_of(const Solver &S, const nlrmm_batch &b) { return b.nviews * S.g.nbins; }

// Enough blocks for the inner products and the regulariser Gram to keep every CU busy on
// large images (a few elements per thread, 16 pixel chunks per Gram block); the minimum of
// 512 serves images up to 512x512 (512 Gram blocks measured best at 256x256).
static void size_blocks(Solver &S, int64_t n, int64_t m)
{
    const int64_t big = n > m ? n : m;
    const int64_t md = (big + 1023) / 1024, gb = (n / 64 + 15) / 16;
    S.md_blocks = (int)(md < 512 ? 512 : md > 2048 ? 2048 : md);
    S.gram_blocks = (int)(gb < 512 ? 512 : gb > 2048 ? 2048 : gb);
}

static bool per_frame(const Solver &S, const nlrmm_batch &b)
{
    return S.plain && b.nframes > 1 && (int64_t)S.vo_host.size() == (int64_t)b.nframes + 1;
}

// Projection of ncols columns with the solver's launch policy.  In plain mode every
// (column, frame) pair is its own launch on its frame's views.
static int proj(Solver &S, const nlrmm_batch &b, int ncols, const float *x, const double *theta,
                const FwdOptions &o, hipStream_t s)
{
    if (!per_frame(S, b)) return launch_project_ex(S.ctx, S.g, b, ncols, x, theta, o, s);
    const int F = b.nframes;
    const int64_t npix = (int64_t)S.g.nx * S.g.ny, nb = S.g.nbins, V = b.nviews;
    const int nch = fwd_chunks(S.g);
    for (int c = 0; c < ncols; ++c) {
        for (int f = 0; f < F; ++f) {
            const int64_t v0 = S.vo_host[f], nv = S.vo_host[f + 1] - v0;
            if (nv <= 0) continue;
            nlrmm_batch fb{1, nv, nullptr};
            FwdOptions q = o;
            const int64_t yo = (int64_t)c * V * nb + v0 * nb;
            if (o.y) q.y = o.y + yo;
            if (o.dy) q.dy = o.dy + yo;
            if (o.g) q.g = o.g + v0 * nb;
            if (o.bres) q.bres = o.bres + v0 * nb;
            if (o.gdot) q.gdot = o.gdot + (int64_t)c * V + v0;
            if (o.dnorm2) q.dnorm2 = o.dnorm2 + (int64_t)c * V + v0;
            if (o.rnorm2) q.rnorm2 = o.rnorm2 + (int64_t)c * V + v0;
            if (o.tdir) q.tdir = o.tdir + v0;
            if (o.part_buf) q.part_buf = o.part_buf + 3 * ((int64_t)c * V + v0) * nch;
            RC(launch_project_ex(S.ctx, S.g, fb, 1, x + ((int64_t)c * F + f) * npix, theta + v0, q,
                                 s));
        }
    }
    return NLRMM_OK;
}

static int proj_plain(Solver &S, const nlrmm_batch &b, int ncols, const float *x,
                      const double *theta, float *y, hipStream_t s)
{
    FwdOptions o;
    o.y = y;
    return proj(S, b, ncols, x, theta, o, s);
}

static int bproj(Solver &S, const nlrmm_batch &b, const float *y, const double *theta, float *x,
                 hipStream_t s)
{
    if (!per_frame(S, b)) return launch_backproject(S.ctx, S.g, b, 1, y, theta, x, s);
    const int64_t npix = (int64_t)S.g.nx * S.g.ny, nb = S.g.nbins;
    for (int f = 0; f < b.nframes; ++f) {
        const int64_t v0 = S.vo_host[f], nv = S.vo_host[f + 1] - v0;
        if (nv <= 0) {
            RC(k_fill_f32(x + f * npix, npix, 0.0f, s));   // a frame without views
            continue;
        }
        nlrmm_batch fb{1, nv, nullptr};
        RC(launch_backproject(S.ctx, S.g, fb, 1, y + v0 * nb, theta + v0, x + f * npix, s));
    }
    return NLRMM_OK;
}

// G_A = (AV)^T AV and rb = (AV)^T b for the first ell columns, plus ||b||^2.
static int gram_from_scratch(Solver &S, int ell, int64_t m, const float *b, hipStream_t s)
{
    S.l_ell = 0;   // GA is rebuilt: the kept factor no longer applies
    S.ga_appended = false;
    if (ell >= 1 && ell <= 10)
        return k_gram_cols(S.AV, m, ell, b, m, S.part_md, S.md_blocks, S.GA, S.ld, S.rb,
                           S.sc + S_BNORM2, s);
    for (int j = 0; j < ell; ++j)
        RC(k_multidot(S.AV, m, j + 1, S.AV + (int64_t)j * m, nullptr, m, S.part_md, S.md_blocks,
                      S.GA + j, S.ld, s));
    RC(k_symmetrize(S.GA, S.ld, ell, s));
    RC(k_multidot(S.AV, m, ell, b, b, m, S.part_md, S.md_blocks, S.hb, 1, s));
    // hb = [rb (ell), ||b||^2]
    RC(k_copy_f64(S.hb, S.rb, ell, s));
    RC(k_copy_f64(S.hb + ell, S.sc + S_BNORM2, 1, s));
    return NLRMM_OK;
}

// r <- r - V V^T r twice (CGS2) against the first ell columns; hb[ell] = ||r_in||^2,
// hb[ell+1] = ||r_out||^2; then V[:, ell] = r_out / ||r_out|| with the breakdown test.
static int cgs2_append(Solver &S, int ell, hipStream_t s, int p1_blocks = 0,
                       int *norm_blocks = nullptr)
{
    return k_cgs2(S.V, S.n, ell, S.r, S.n, S.part_md, S.part_md2, S.md_blocks, S.hb, S.hb2,
                  S.cfg.breakdown_tol, S.V + (int64_t)ell * S.n, S.status, s, p1_blocks,
                  norm_blocks);
}

// The first CGS2 products of the residual, formed by the backprojection's split-sum launch
// when it has one (the multidot's grid: one element per thread, within its block budget).
static MdEpilogue cgs2_products(const Solver &S, int ell)
{
    MdEpilogue md;
    md.X = S.V;
    md.ldx = S.n;
    md.nv = ell;
    md.part = S.part_md;
    md.nblk_cap = S.md_blocks < CGS2_FUSED_MAXBLK ? S.md_blocks : CGS2_FUSED_MAXBLK;
    return md;
}

// r = A^T (A V z - b) + lam Psi^T (w * Psi u), with u = V z already in S.u.
// weights_of_u: the weights are those of the current u (formed on the fly); otherwise the
// stored S.w (the weights of the step's solve).
static int mm_residual(Solver &S, const nlrmm_batch &b, const double *theta, int ell,
                       const float *bvec, hipStream_t s, bool weights_of_u = false,
                       MdEpilogue *md = nullptr)
{
    if (md) md->fused = false;
    const bool inl = weights_of_u && S.w_from_u;
    const int64_t m = m_of(S, b);
    if (!S.rho_ready) RC(k_gemv(S.AV, m, ell, S.z, 1.0, bvec, -1.0, m, S.rho, s));
    S.rho_ready = false;
    const bool motion = S.cfg.temporal == TEMPORAL_OF && S.F > 1;
    if (!per_frame(S, b) && !motion) {
        // one launch pair: backprojection with the TV-gradient term as its epilogue
        TvEpilogue tv;
        tv.u = S.u;
        tv.w = inl ? nullptr : S.w;   // null: weights of u formed in the epilogue
        tv.lamp = S.sc + S_LAM;
        tv.temporal = S.cfg.temporal;
        tv.e2 = (float)S.cfg.eps * (float)S.cfg.eps;
        return launch_backproject(S.ctx, S.g, b, 1, S.rho, theta, S.r, s, 0, &tv, md);
    }
    RC(bproj(S, b, S.rho, theta, S.r, s));
    RC(k_tv_grad_add(S.u, inl ? nullptr : S.w, S.g.nx, S.g.ny, S.F, S.cfg.temporal,
                     S.sc + S_LAM, S.r, s, (float)S.cfg.eps));
    // the motion rows of the optical-flow operator (their transpose is a scatter)
    if (motion)
        RC(k_of_grad_add(S.u, inl ? nullptr : S.w, S.flow, S.g.nx, S.g.ny, S.F, S.sc + S_LAM,
                         S.r, S.of_acc, s, (float)S.cfg.eps));
    return NLRMM_OK;
}

// Append one GKS direction (Alg. "enlarge" body after u = V z): residual, CGS2, A v and the
// new row of the data Gram.  defer: the Gram row is left to the regulariser Gram launch of the
// projected solve that follows, which computes and reduces it with its own work (two launches
// fewer per expansion).
static int expand(Solver &S, const nlrmm_batch &b, const double *theta, const float *bvec,
                  hipStream_t s, bool defer = false)
{
    const int ell = S.ell;
    const int64_t m = m_of(S, b);
    MdEpilogue md = cgs2_products(S, ell);
    RC(mm_residual(S, b, theta, ell, bvec, s, false, &md));
    // the new column's normalisation rides on the packing launch of its projection (batched
    // launches; per-frame launches normalise first)
    float *vnew = S.V + (int64_t)ell * S.n;
    int nblk3 = 0;
    RC(cgs2_append(S, ell, s, md.fused ? md.nblk : 0, &nblk3));
    if (per_frame(S, b)) {
        RC(k_normalize_red(S.r, S.part_md, nblk3, S.hb + ell, S.cfg.breakdown_tol, S.n, vnew,
                           S.status, s));
        RC(proj_plain(S, b, 1, vnew, theta, S.AV + (int64_t)ell * m, s));
    } else {
        FwdOptions o;
        o.y = S.AV + (int64_t)ell * m;
        o.norm_src = S.r;
        o.norm_part = S.part_md;
        o.norm_nblk = nblk3;
        o.norm_scal = S.hb + ell;
        o.norm_tol = S.cfg.breakdown_tol;
        o.norm_out = vnew;
        o.norm_status = S.status;
        RC(proj(S, b, 1, vnew, theta, o, s));
    }
    if (defer) {
        S.gc = GramColJob{S.AV, m, ell, S.AV + (int64_t)ell * m, bvec, m, S.part_md,
                          (int64_t)md_part_doubles(S.md_blocks), S.md_blocks, S.GA, S.ld, S.rb};
        S.gc_pending = true;
    } else {
        RC(k_multidot_gram_col(S.AV, m, ell, S.AV + (int64_t)ell * m, bvec, m, S.part_md,
                               S.md_blocks, S.GA, S.ld, S.rb, s));
    }
    S.ell = ell + 1;
    S.ga_appended = true;
    return NLRMM_OK;
}

// One projected solve on the current basis: weights from u, weighted regulariser Gram,
// lambda and z, then u = V z.
static int projected_solve(Solver &S, hipStream_t s, const nlrmm_batch *b = nullptr,
                           const float *bvec = nullptr)
{
    // this step's weights (from the u the solve starts from): the Gram and, in the expansion
    // that follows, the residual use them (Alg. "enlarge").  On small images the Gram launch
    // forms them and stores them in S.w (each of its waves forms them again for its own
    // columns, which costs more than the saved launch beyond about half a million pixels);
    // it also completes a pending row of the data Gram.
    const GramColJob *side = S.gc_pending ? &S.gc : nullptr;
    S.gc_pending = false;
    const bool wfused = S.n <= GRAM_FUSED_WEIGHTS_MAX;
    if (!wfused)
        RC(k_psi_weights(S.u, S.g.nx, S.g.ny, S.F, S.cfg.temporal, (float)S.cfg.eps, S.w, s,
                         S.flow));
    RC(k_gram_psi(S.V, S.n, S.ell, wfused ? nullptr : S.w, S.g.nx, S.g.ny, S.F, S.cfg.temporal,
                  S.part_gram, S.gram_blocks, S.GP, S.ld, s, S.cfg.gram_precision,
                  wfused ? S.u : nullptr, (float)S.cfg.eps, S.flow, wfused ? S.w : nullptr,
                  side));
    // the factor of GA is extended by one row when an expansion appended one since the last
    // solve, else formed anew
    const int linc = (S.Lst != nullptr && S.ga_appended && S.l_ell == S.ell - 1) ? 1 : 0;
    RC(k_gks_solve(S.GA, S.GP, S.ld, S.rb, S.sc + S_BNORM2, S.ell, S.cfg.lam_fix, S.z,
                   S.sc + S_LAM, S.status, s, 1, S.Lst, linc));
    S.l_ell = S.Lst != nullptr ? S.ell : 0;
    S.ga_appended = false;
    if (b && bvec) {
        // u = V z and the data residual A V z - b of the expansion that follows, one launch
        const int64_t m = m_of(S, *b);
        RC(k_gemv2(S.V, S.n, S.ell, S.z, 1.0, nullptr, 0.0, S.n, S.u, S.AV, m, S.ell, S.z, 1.0,
                   bvec, -1.0, m, S.rho, s));
        S.rho_ready = true;
        return NLRMM_OK;
    }
    RC(k_gemv(S.V, S.n, S.ell, S.z, 1.0, nullptr, 0.0, S.n, S.u, s));
    return NLRMM_OK;
}

// Alg. "compress": basis -> kmin columns, A V transformed alongside, z -> z'.
static int compress(Solver &S, const nlrmm_batch &b, hipStream_t s)
{
    const int kmin = S.cfg.kmin;
    const int64_t m = m_of(S, b);
    RC(k_compress_eig(S.GA, S.GP, S.ld, S.sc + S_LAM, S.ell, kmin, S.z, S.T, kmin, S.zt,
                      S.kout, S.status, s));
    RC(k_block_update(S.V, S.n, S.ell, S.T, kmin, kmin, S.n, S.Vtmp, S.n, s,
                      S.cfg.compress_precision));
    RC(k_copy_cols(S.Vtmp, S.n, S.V, S.n, kmin, S.n, s));
    RC(k_block_update(S.AV, m, S.ell, S.T, kmin, kmin, m, S.Vtmp, m, s,
                      S.cfg.compress_precision));
    RC(k_copy_cols(S.Vtmp, m, S.AV, m, kmin, m, s));
    RC(k_gram_transform(S.GA, S.ld, S.rb, S.ell, S.T, kmin, S.kout, s));
    S.l_ell = 0;   // GA transformed: the kept factor no longer applies
    S.ga_appended = false;
    RC(k_copy_f64(S.zt, S.z, kmin, s));
    S.ell = kmin;
    RC(k_gemv(S.V, S.n, kmin, S.z, 1.0, nullptr, 0.0, S.n, S.u, s));
    return NLRMM_OK;
}

// Alg. "update_param" with u fixed: damped Gauss-Newton, Armijo on one global alpha.
static int gn_update(Solver &S, const nlrmm_batch &b, double *theta, const float *bvec,
                     hipStream_t s)
{
    const int64_t V = b.nviews;
    const int nch = fwd_chunks(S.g);
    for (int it = 0; it < S.cfg.maxiter_p; ++it) {
        FwdOptions o;
        o.bres = bvec;
        o.gdot = S.gv;
        o.dnorm2 = S.hv;
        o.rnorm2 = S.rv;
        o.part_buf = S.part_fwd;
        RC(proj(S, b, 1, S.u, theta, o, s));
        RC(k_gn_prepare(S.gv, S.hv, S.rv, V, S.cfg.param_mode, S.cfg.mu_rel, S.dir, S.sc + S_GN,
                        S.accepted, s));
        for (int q = 0; q < S.cfg.armijo_trials; ++q) {
            FwdOptions t;
            t.bres = bvec;
            t.rnorm2 = S.rv;   // per-view ||r_v||^2 at the trial angles
            t.part_buf = S.part_fwd;
            t.tdir = S.dir;
            t.talpha = S.alphas + q;
            t.skip = S.accepted;
            RC(proj(S, b, 1, S.u, theta, t, s));
            RC(k_armijo_check(S.rv, V, S.alphas, q, S.cfg.c1, S.sc + S_GN, S.accepted, s));
        }
        (void)nch;
        RC(k_gn_apply(theta, S.dir, V, S.sc + S_GN, S.accepted, S.status, s));
    }
    return NLRMM_OK;
}

// k x k Gram of A_hat and A_hat^T b (vp_GA, vp_ab).
static int varpro_grams(Solver &S, int k, int64_t m, const float *bvec, hipStream_t s,
                        const int *skip)
{
    for (int j = 0; j < k; ++j)
        RC(k_multidot(S.Ahat, m, j + 1, S.Ahat + (int64_t)j * m, nullptr, m, S.part_md,
                      S.md_blocks, S.vp_GA + j, S.ld, s, skip));
    RC(k_symmetrize(S.vp_GA, S.ld, k, s));
    RC(k_multidot(S.Ahat, m, k, bvec, nullptr, m, S.part_md, S.md_blocks, S.vp_ab, 1, s, skip));
    return NLRMM_OK;
}

// VarPro angle update on the compressed basis (k = kmin columns), weights from u.
static int varpro_update(Solver &S, const nlrmm_batch &b, double *theta, const float *bvec,
                         hipStream_t s)
{
    const int k = S.ell;
    const int64_t V = b.nviews;
    const int64_t m = m_of(S, b);
    RC(k_psi_weights(S.u, S.g.nx, S.g.ny, S.F, S.cfg.temporal, (float)S.cfg.eps, S.w, s,
                     S.flow));
    RC(k_gram_psi(S.V, S.n, k, S.w, S.g.nx, S.g.ny, S.F, S.cfg.temporal, S.part_gram,
                  S.gram_blocks, S.GP, S.ld, s, S.cfg.gram_precision, nullptr, 0.0f, S.flow));
    double *sc = S.sc + S_GN;
    for (int it = 0; it < S.cfg.maxiter_p; ++it) {
        RC(proj_plain(S, b, k, S.V, theta, S.Ahat, s));
        RC(varpro_grams(S, k, m, bvec, s, nullptr));
        RC(k_varpro_reduced(S.vp_GA, S.ld, S.GP, S.vp_ab, S.sc + S_LAM, S.sc + S_BNORM2, k,
                            S.vp_y, S.vp_M, sc, S.alphas, -1, S.cfg.c1, S.accepted, S.status, s));
        // u_hat = V y, r = A_hat y - b
        RC(k_gemv(S.V, S.n, k, S.vp_y, 1.0, nullptr, 0.0, S.n, S.r, s));
        RC(k_gemv(S.Ahat, m, k, S.vp_y, 1.0, bvec, -1.0, m, S.rho, s));
        FwdOptions o;
        o.dy = S.evec;
        o.g = S.rho;
        o.gdot = S.vp_gd;
        o.dnorm2 = S.vp_en2;
        o.part_buf = S.part_fwd;
        RC(proj(S, b, 1, S.r, theta, o, s));
        FwdOptions oc;
        oc.g = S.rho;
        oc.gdot = S.vp_ETr;
        oc.part_buf = S.part_fwd;
        RC(proj(S, b, k, S.V, theta, oc, s));
        RC(k_view_dots(S.Ahat, m, k, S.evec, S.g.nbins, V, S.vp_Ate, s));
        RC(k_varpro_dir(S.vp_M, k, S.vp_gd, S.vp_en2, S.vp_ETr, S.vp_Ate, V, S.cfg.mu_rel, S.vp_Y,
                        S.dir, sc, S.status, s));
        for (int q = 0; q < S.cfg.armijo_trials; ++q) {
            FwdOptions t;
            t.y = S.Ahat;
            t.tdir = S.dir;
            t.talpha = S.alphas + q;
            t.skip = S.accepted;
            RC(proj(S, b, k, S.V, theta, t, s));
            RC(varpro_grams(S, k, m, bvec, s, S.accepted));
            RC(k_varpro_reduced(S.vp_GA, S.ld, S.GP, S.vp_ab, S.sc + S_LAM, S.sc + S_BNORM2, k,
                                S.vp_y, S.vp_M, sc, S.alphas, q, S.cfg.c1, S.accepted, S.status,
                                s));
        }
        RC(k_gn_apply(theta, S.dir, V, sc, S.accepted, S.status, s));
    }
    return NLRMM_OK;
}

static int offset_sensitivity(Solver &S, const nlrmm_batch &b, const double *theta,
                              const float *bvec, int iters, double *out, float *up_out,
                              hipStream_t s, float *xw, float *rw);

// Parameter update of one global angle offset from the full-space sensitivity equation
// (Section 4.2, eqs. "sensitivity" and "GN_system"): u_p, g and h (conjugate gradients,
// sens_iters steps) at the image u, the damped step dp = -g / (h + mu), mu = mu_rel h, for
// every view, and Armijo backtracking on the reduced objective
// f(p) = 1/2 ||A(theta + p) u(p) - b||^2 + lam/2 ||sqrt(w) Psi u(p)||^2 with u(p) to first order,
// u + (p - p_k) u_p (its slope at p_k is g dp).  xw, rw: work columns of the sensitivity solve
// (null: the spare columns after V's first ell); u_p stays in the first of xw, the trial
// image goes to its fifth.
static int sensitivity_update(Solver &S, const nlrmm_batch &b, double *theta, const float *bvec,
                              hipStream_t s, float *xw, float *rw)
{
    const int64_t V = b.nviews;
    const int64_t n = S.n;
    if (xw == nullptr || rw == nullptr) {
        if (S.kcap - S.ell < 6) return NLRMM_ESHAPE;
        xw = S.V + (int64_t)S.ell * n;
        rw = S.AV + (int64_t)S.ell * m_of(S, b);
    }
    const float *up = xw;
    float *ua = xw + 4 * n;
    double *sc = S.sc + S_GN;
    double *gh = S.cgs + 12;    // [g, h, dp] of the sensitivity solve
    double *reg = S.cgs + 15;   // ||sqrt(w) Psi u||^2 of the current image or trial
    struct {
        int nx, ny, F, temporal;
    } const tg{S.g.nx, S.g.ny, S.F, S.cfg.temporal};
    auto reduced = [&](const float *img, const double *th, const double *tdir,
                       const double *talpha, const int *skip, int q) -> int {
        FwdOptions o;
        o.bres = bvec;
        o.rnorm2 = S.rv;   // per-view ||A(theta') img - b||^2
        o.part_buf = S.part_fwd;
        o.tdir = tdir;
        o.talpha = talpha;
        o.skip = skip;
        RC(proj(S, b, 1, img, th, o, s));
        RC(k_gram_psi(img, n, 1, S.w, tg.nx, tg.ny, tg.F, tg.temporal, S.part_gram,
                      S.gram_blocks, reg, 1, s, 0));
        return k_sens_objective(S.rv, V, reg, S.sc + S_LAM, S.alphas, q, S.cfg.c1, sc,
                                S.accepted, s);
    };
    for (int it = 0; it < S.cfg.maxiter_p; ++it) {
        // (offset_sensitivity leaves the weights of u in S.w)
        RC(offset_sensitivity(S, b, theta, bvec, S.cfg.sens_iters, gh, nullptr, s, xw, rw));
        RC(k_offset_dir(gh, S.cfg.mu_rel, V, S.dir, sc, s));
        RC(reduced(S.u, theta, nullptr, nullptr, nullptr, -1));
        for (int q = 0; q < S.cfg.armijo_trials; ++q) {
            RC(k_lin_image(S.u, up, n, S.alphas, q, S.dir, S.accepted, ua, s));
            RC(reduced(ua, theta, S.dir, S.alphas + q, S.accepted, q));
        }
        RC(k_gn_apply(theta, S.dir, V, sc, S.accepted, S.status, s));
    }
    return NLRMM_OK;
}

// The optional high-regularisation solve of Alg. "nl_rmmgks_two_solves" (Section 4.3), run
// after Compress: one RMM-GKS cycle with lambda fixed at lam_hi from the compressed basis
// V_kmin and u_{k+1}, then the parameter update on its image u_hat (VarPro: on its own
// compressed basis, in Vtmp, and lam_hi).  Its basis grows in the columns kmin.. of V and
// A V, which the primary state does not use after Compress, and in the data Gram (rebuilt
// by the next rebase); it keeps its own image and coefficients (uh, zh) and saves the
// primary lambda, so V_kmin, A V_kmin, u, z and lambda_k leave unchanged.
static int hi_solve_update(Solver &S, const nlrmm_batch &b, double *theta, const float *bvec,
                           hipStream_t s)
{
    const int ell0 = S.ell;
    float *const u0 = S.u;
    double *const z0 = S.z;
    const double lam_fix0 = S.cfg.lam_fix;
    RC(k_copy_f64(S.sc + S_LAM, S.sc + S_LAMK, 1, s));
    RC(k_copy_cols(u0, S.n, S.uh, S.n, 1, S.n, s));
    S.u = S.uh;
    S.z = S.zh;
    S.cfg.lam_fix = S.cfg.lam_hi;
    S.rho_ready = false;
    int rc = NLRMM_OK;
    const int nsolve = S.cfg.solves;
    for (int t = 0; t < nsolve && !rc; ++t) {
        const bool more = t < nsolve - 1;
        rc = projected_solve(S, s, more ? &b : nullptr, more ? bvec : nullptr);
        if (!rc && more) rc = expand(S, b, S.thk, bvec, s, true);
    }
    if (!rc && S.cfg.param_update == 1) rc = gn_update(S, b, theta, bvec, s);
    if (!rc && S.cfg.param_update == 3) {
        // on u_hat; the columns kmin.. of the basis hold this solve's basis, no longer needed
        const int64_t m = m_of(S, b);
        rc = sensitivity_update(S, b, theta, bvec, s, S.V + (int64_t)S.cfg.kmin * S.n,
                                S.AV + (int64_t)S.cfg.kmin * m);
    }
    if (!rc && S.cfg.param_update == 2) {
        // compressed basis of this solve into Vtmp; VarPro rebuilds A V_hat itself
        const int kmin = S.cfg.kmin;
        rc = k_compress_eig(S.GA, S.GP, S.ld, S.sc + S_LAM, S.ell, kmin, S.z, S.T, kmin, S.zt,
                            S.kout, S.status, s);
        if (!rc)
            rc = k_block_update(S.V, S.n, S.ell, S.T, kmin, kmin, S.n, S.Vtmp, S.n, s,
                                S.cfg.compress_precision);
        if (!rc) {
            float *const V0 = S.V;
            S.V = S.Vtmp;
            S.ell = kmin;
            rc = varpro_update(S, b, theta, bvec, s);
            S.V = V0;
        }
    }
    S.u = u0;
    S.z = z0;
    S.cfg.lam_fix = lam_fix0;
    S.ell = ell0;
    S.rho_ready = false;
    if (rc) return rc;
    return k_copy_f64(S.sc + S_LAMK, S.sc + S_LAM, 1, s);
}

static int solver_outer(Solver &S, const nlrmm_batch &b, double *theta, const float *bvec,
                        double delta, hipStream_t s)
{
    const int64_t V = b.nviews;
    const int64_t m = m_of(S, b);
    if (V > S.maxV) return NLRMM_ESHAPE;
    S.gc_pending = false;
    S.ga_appended = false;
    // optical-flow branch of Alg. "dyn_nl_rmmgks": the velocities of every frame pair from
    // u^(k) (SOLVE-OF) every of_every outer iterations; Theta^(k) = [Psi; M_hat] follows
    if (S.cfg.temporal == TEMPORAL_OF && S.F > 1 && S.outer_count % S.cfg.of_every == 0)
        RC(k_of_estimate(S.u, S.g.nx, S.g.ny, S.F, (float)S.cfg.of_gamma, (float)S.cfg.of_ridge,
                         S.cfg.of_iters, S.flow, S.of_work, S.of_part, s));
    ++S.outer_count;
    // theta_k: the operator H_k of this outer iteration
    RC(k_copy_f64(theta, S.thk, V, s));
    RC(k_fill_f64(S.sc + S_TARGET, 1, S.cfg.tau * delta, s));
    // rebase A V on the current views and angles
    RC(proj_plain(S, b, S.ell, S.V, S.thk, S.AV, s));
    RC(gram_from_scratch(S, S.ell, m, bvec, s));
    const int nsolve = S.cfg.solves;
    for (int t = 0; t < nsolve; ++t) {
        const bool more = t < nsolve - 1;
        RC(projected_solve(S, s, more ? &b : nullptr, more ? bvec : nullptr));
        if (more) RC(expand(S, b, S.thk, bvec, s, true));
    }
    RC(compress(S, b, s));
    if (S.cfg.lam_hi > 0.0) {
        RC(hi_solve_update(S, b, theta, bvec, s));
    } else {
        if (S.cfg.param_update == 1) RC(gn_update(S, b, theta, bvec, s));
        if (S.cfg.param_update == 2) RC(varpro_update(S, b, theta, bvec, s));
        if (S.cfg.param_update == 3) RC(sensitivity_update(S, b, theta, bvec, s, nullptr, nullptr));
    }
    // weights from u_{k+1} (formed inside the residual); residual with the old operator H_k;
    // project out; append
    MdEpilogue md = cgs2_products(S, S.ell);
    RC(mm_residual(S, b, S.thk, S.ell, bvec, s, true, &md));
    RC(cgs2_append(S, S.ell, s, md.fused ? md.nblk : 0));
    S.ell += 1;
    (void)m;
    return NLRMM_OK;
}

// Golub-Kahan bidiagonalisation from b (k right vectors, CGS2 on both sides); u = 0.
static int solver_init(Solver &S, const nlrmm_batch &b, const double *theta, const float *bvec,
                       hipStream_t s, int kvec = 0)
{
    const int k = kvec > 0 ? kvec : S.cfg.kmin + 1;
    const int64_t m = m_of(S, b);
    if (b.nviews > S.maxV) return NLRMM_ESHAPE;
    float *U = S.AV;   // left vectors stored where A V lives later
    double *nrm = S.gkb;   // [0..k) alpha_i, [k..2k) beta_i
    RC(k_fill_i32(S.status, 1, 0, s));
    RC(k_fill_f64(S.z, S.kcap, 0.0, s));
    // u_1 = b / ||b||
    RC(k_multidot(S.V, S.n, 0, bvec, bvec, m, S.part_md, S.md_blocks, S.hb, 1, s));
    RC(k_scale_into(bvec, S.hb, m, U, nrm + k, S.status, s));
    for (int i = 0; i < k; ++i) {
        // v = A^T u_i - beta_i v_{i-1}, reorthogonalised against V, normalised
        RC(bproj(S, b, U + (int64_t)i * m, theta, S.r, s));
        if (i > 0)
            RC(k_gemv(S.V + (int64_t)(i - 1) * S.n, S.n, 1, nrm + k + i, -1.0, S.r, 1.0, S.n,
                      S.r, s));
        if (i > 0) {
            RC(k_multidot(S.V, S.n, i, S.r, nullptr, S.n, S.part_md, S.md_blocks, S.hb, 1, s));
            RC(k_gemv(S.V, S.n, i, S.hb, -1.0, S.r, 1.0, S.n, S.r, s));
            RC(k_multidot(S.V, S.n, i, S.r, nullptr, S.n, S.part_md, S.md_blocks, S.hb, 1, s));
            RC(k_gemv(S.V, S.n, i, S.hb, -1.0, S.r, 1.0, S.n, S.r, s));
        }
        RC(k_multidot(S.V, S.n, 0, S.r, S.r, S.n, S.part_md, S.md_blocks, S.hb, 1, s));
        RC(k_scale_into(S.r, S.hb, S.n, S.V + (int64_t)i * S.n, nrm + i, S.status, s));
        if (i == k - 1) break;
        // p = A v_i - alpha_i u_i, reorthogonalised against U, normalised
        RC(proj_plain(S, b, 1, S.V + (int64_t)i * S.n, theta, S.rho, s));
        RC(k_gemv(U + (int64_t)i * m, m, 1, nrm + i, -1.0, S.rho, 1.0, m, S.rho, s));
        RC(k_multidot(U, m, i + 1, S.rho, nullptr, m, S.part_md, S.md_blocks, S.hb, 1, s));
        RC(k_gemv(U, m, i + 1, S.hb, -1.0, S.rho, 1.0, m, S.rho, s));
        RC(k_multidot(U, m, i + 1, S.rho, nullptr, m, S.part_md, S.md_blocks, S.hb, 1, s));
        RC(k_gemv(U, m, i + 1, S.hb, -1.0, S.rho, 1.0, m, S.rho, s));
        RC(k_multidot(U, m, 0, S.rho, S.rho, m, S.part_md, S.md_blocks, S.hb, 1, s));
        RC(k_scale_into(S.rho, S.hb, m, U + (int64_t)(i + 1) * m, nrm + k + i + 1, S.status, s));
    }
    S.ell = k;
    RC(k_fill_f32(S.u, S.n, 0.0f, s));   // u = 0
    return NLRMM_OK;
}

// Parameter initialisation by a coarse grid search over a global angle offset (the
// experiments section): a GKB basis of ell0 vectors from b at the nominal angles, then for
// every candidate s_c the reduced least-squares residual min_z ||A(theta + s_c) V z - b||^2
// (one multi-column projection at the shifted angles, the data Gram, a Cholesky), and
// theta += s_best.
static int grid_search(Solver &S, const nlrmm_batch &b, double *theta, const float *bvec,
                       const double *shifts, int ncand, int ell0, double *res2, int *best,
                       hipStream_t s)
{
    const int64_t V = b.nviews;
    const int64_t m = m_of(S, b);
    RC(solver_init(S, b, theta, bvec, s, ell0));
    // trial-angle projections theta + shifts[c] * 1 of the basis, into the A V storage
    RC(k_fill_f64(S.dir, V, 1.0, s));
    for (int c = 0; c < ncand; ++c) {
        FwdOptions o;
        o.y = S.AV;
        o.tdir = S.dir;
        o.talpha = shifts + c;
        RC(proj(S, b, ell0, S.V, theta, o, s));
        RC(gram_from_scratch(S, ell0, m, bvec, s));
        RC(k_grid_residual(S.GA, S.ld, S.rb, S.sc + S_BNORM2, ell0, res2 + c, s));
    }
    return k_grid_pick(res2, ncand, shifts, theta, V, best, s);
}

// Full-space sensitivity of the VarPro reduced problem for one global angle offset p
// (Section 4.2, eq. "sensitivity", with u the current RMM-GKS image standing in for the
// closed form u(p), as the paper does in practice): weights w of u, r = A u - b and A_p u = D u
// in one projection, right-hand side -(D^T r + A^T D u), then `iters` conjugate-gradient
// steps on M = A^T A + lam Psi^T diag(w) Psi (one projection and one backprojection with the
// weighted regulariser term as its epilogue per step) for u_p, J_r = D u + A u_p, and the
// Gauss-Newton scalars g = J_r^T r + lam u_p^T Psi^T w Psi u, h = J_r^T J_r + lam u_p^T
// Psi^T w Psi u_p, dp = -g / h.  The vectors live in the spare basis columns (six of V, three
// of A V), so the solver state carried between outer iterations is untouched.
static int offset_sensitivity(Solver &S, const nlrmm_batch &b, const double *theta,
                              const float *bvec, int iters, double *out, float *up_out,
                              hipStream_t s, float *xw = nullptr, float *rw = nullptr)
{
    const int64_t n = S.n, m = m_of(S, b);
    // work vectors: six image-sized and three sinogram-sized columns, by default the spare
    // columns of the basis after the current ones
    if (xw == nullptr || rw == nullptr) {
        const int base = S.ell;
        if (S.kcap - base < 6) return NLRMM_ESHAPE;
        xw = S.V + (int64_t)base * n;
        rw = S.AV + (int64_t)base * m;
    }
    float *x = xw, *rc = x + n, *p = x + 2 * n, *q = x + 3 * n, *t1 = x + 4 * n, *t2 = x + 5 * n;
    float *r = rw, *du = r + m, *jr = r + 2 * m;
    double *c = S.cgs;
    double *one = c + 6, *d1 = c + 7, *d2 = c + 9;
    struct {
        int nx, ny, F, temporal;
    } const dims{S.g.nx, S.g.ny, S.F, S.cfg.temporal};
    RC(k_fill_f64(one, 1, 1.0, s));
    RC(k_psi_weights(S.u, dims.nx, dims.ny, dims.F, dims.temporal, (float)S.cfg.eps, S.w, s));
    {
        FwdOptions o;
        o.y = r;
        o.bres = bvec;
        o.write_resid = 1;
        o.dy = du;
        RC(launch_project_ex(S.ctx, S.g, b, 1, S.u, theta, o, s));
    }
    // rhs = -(D^T r + A^T D u); x = 0, residual = p = rhs
    RC(launch_backproject_dtheta(S.ctx, S.g, b, 1, r, theta, t1, s));
    RC(launch_backproject(S.ctx, S.g, b, 1, du, theta, t1, s, 1));
    RC(k_gemv(t1, n, 1, one, -1.0, nullptr, 0.0, n, rc, s));
    RC(k_gemv(rc, n, 1, one, 1.0, nullptr, 0.0, n, p, s));
    RC(k_fill_f32(x, n, 0.0f, s));
    RC(k_multidot(rc, n, 1, rc, nullptr, n, S.part_md, S.md_blocks, c + 0, 1, s));
    TvEpilogue tv;
    tv.w = S.w;
    tv.lamp = S.sc + S_LAM;
    tv.temporal = S.cfg.temporal;
    tv.e2 = (float)S.cfg.eps * (float)S.cfg.eps;
    for (int it = 0; it < iters; ++it) {
        FwdOptions o;
        o.y = jr;
        RC(launch_project_ex(S.ctx, S.g, b, 1, p, theta, o, s));
        tv.u = p;
        RC(launch_backproject(S.ctx, S.g, b, 1, jr, theta, q, s, 0, &tv));   // q = M p
        RC(k_multidot(p, n, 1, q, nullptr, n, S.part_md, S.md_blocks, c + 1, 1, s));
        RC(k_cg_coef(c, 0, s));
        RC(k_gemv(p, n, 1, c + 3, 1.0, x, 1.0, n, x, s));     // x += alpha p
        RC(k_gemv(q, n, 1, c + 4, 1.0, rc, 1.0, n, rc, s));   // r -= alpha M p
        RC(k_multidot(rc, n, 1, rc, nullptr, n, S.part_md, S.md_blocks, c + 2, 1, s));
        RC(k_cg_coef(c, 1, s));
        RC(k_gemv(p, n, 1, c + 5, 1.0, rc, 1.0, n, p, s));    // p = r + beta p
    }
    // J_r = D u + A u_p; [J_r^T J_r, r^T J_r]
    {
        FwdOptions o;
        o.y = jr;
        RC(launch_project_ex(S.ctx, S.g, b, 1, x, theta, o, s));
    }
    RC(k_gemv(du, m, 1, one, 1.0, jr, 1.0, m, jr, s));
    RC(k_multidot(jr, m, 1, jr, r, m, S.part_md, S.md_blocks, d1, 1, s));
    // [u_p^T Psi^T w Psi u, u_p^T Psi^T w Psi u_p]
    // the spare columns may hold anything: clear them with a fill (never by scaling)
    RC(k_fill_f32(t1, n, 0.0f, s));
    RC(k_fill_f32(t2, n, 0.0f, s));
    RC(k_tv_grad_add(S.u, S.w, dims.nx, dims.ny, dims.F, dims.temporal, one, t1, s));
    RC(k_tv_grad_add(x, S.w, dims.nx, dims.ny, dims.F, dims.temporal, one, t2, s));
    RC(k_multidot(t1, n, 2, x, nullptr, n, S.part_md, S.md_blocks, d2, 1, s));
    RC(k_offset_gn(d1, d2, S.sc + S_LAM, out, s));
    if (up_out) RC(k_copy_cols(x, n, up_out, n, 1, n, s));
    return NLRMM_OK;
}

}  // namespace nlrmm

using namespace nlrmm;

extern "C" {

int nlrmm_solver_create(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes,
                        int64_t max_views, const nlrmm_solver_cfg *cfg, nlrmm_solver **out)
{
    int rc = check_op_geom(NLRMM_OPS_FORWARD | NLRMM_OPS_BACKWARD, geom);
    if (rc) return rc;
    if (!ctx || !cfg || !out) return NLRMM_EINVAL;
    if (nframes < 1 || max_views < 1) return NLRMM_ESHAPE;
    nlrmm_solver_cfg c = *cfg;
    if (c.kmin < 2 || c.kmin > 16 || c.kmax <= c.kmin || c.kmax > 55) return NLRMM_ESHAPE;
    if (c.solves <= 0) c.solves = c.kmax - c.kmin;
    if (c.kmin + c.solves > c.kmax + 1 || c.solves < 1) return NLRMM_ESHAPE;
    if (c.armijo_trials < 0 || c.armijo_trials > 32 || c.maxiter_p < 0) return NLRMM_EINVAL;
    if (!(c.eps > 0.0) || !(c.tau > 0.0)) return NLRMM_EINVAL;
    if (c.lam_hi > 0.0 && !(c.lam_hi < HUGE_VAL)) return NLRMM_EINVAL;
    if (c.param_update < 0 || c.param_update > 3) return NLRMM_ENOTSUP;
    // the sensitivity update moves one global offset and needs six spare basis columns
    if (c.param_update == 3 && (c.param_mode != 1 || c.kmax + 1 - c.kmin < 6))
        return NLRMM_ENOTSUP;
    if (c.sens_iters <= 0) c.sens_iters = 50;
    // temporal rows: 0 none, 1 frame differences (ANISO-TV), 2 optical-flow motion rows
    if (c.temporal < 0 || c.temporal > 2) return NLRMM_ENOTSUP;
    if (c.temporal == TEMPORAL_OF) {
        if (nframes > 1 && (geom->nx < 2 || geom->ny < 2)) return NLRMM_ESHAPE;
        // the sensitivity solve forms its regulariser without the motion rows
        if (c.param_update == 3) return NLRMM_ENOTSUP;
        if (c.of_iters <= 0) c.of_iters = 200;
        if (!(c.of_gamma > 0.0)) c.of_gamma = 0.05;
        if (!(c.of_ridge > 0.0)) c.of_ridge = 1e-3;
        if (c.of_every <= 0) c.of_every = 1;
        if (!(c.of_gamma < HUGE_VAL) || !(c.of_ridge < HUGE_VAL) || c.of_iters > 100000)
            return NLRMM_EINVAL;
    }
    if (c.gram_precision < 0 || c.gram_precision > 2) return NLRMM_ENOTSUP;
    if (c.compress_precision != 0 && c.compress_precision != 2) return NLRMM_ENOTSUP;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    nlrmm_solver *S = new (std::nothrow) nlrmm_solver();
    if (!S) return NLRMM_ENOMEM;
    S->ctx = ctx;
    S->g = *geom;
    S->F = nframes;
    S->maxV = max_views;
    S->cfg = c;
    S->n = (int64_t)nframes * geom->nx * geom->ny;
    S->mmax = max_views * geom->nbins;
    S->kcap = c.kmax + 1;
    S->ld = S->kcap;
    S->nchunks = fwd_chunks(*geom);
    const int64_t big = S->n > S->mmax ? S->n : S->mmax;
    size_blocks(*S, S->n, S->mmax);
    // spatial rows (< 2 per pixel) plus temporal rows (1 per pixel, 2 with optical flow)
    const int64_t npsi_max = (int64_t)nframes * geom->nx * geom->ny *
                             (c.temporal == TEMPORAL_OF ? 4 : 3);
    if ((rc = S->alloc(&S->V, (size_t)S->kcap * S->n)) ||
        (rc = S->alloc(&S->AV, (size_t)S->kcap * S->mmax)) ||
        (rc = S->alloc(&S->Vtmp, (size_t)c.kmin * big)) || (rc = S->alloc(&S->u, S->n)) ||
        (rc = S->alloc(&S->uh, S->n)) || (rc = S->alloc(&S->zh, S->ld)) ||
        (rc = S->alloc(&S->cgs, 16)) ||
        (rc = S->alloc(&S->r, S->n)) || (rc = S->alloc(&S->rho, S->mmax)) ||
        (rc = S->alloc(&S->w, npsi_max)) || (rc = S->alloc(&S->GA, S->ld * S->ld)) ||
        (rc = S->alloc(&S->Lst, S->ld * S->ld + S->ld)) ||
        (rc = S->alloc(&S->GP, S->ld * S->ld)) || (rc = S->alloc(&S->rb, S->ld)) ||
        (rc = S->alloc(&S->z, S->ld)) || (rc = S->alloc(&S->T, S->ld * c.kmin)) ||
        (rc = S->alloc(&S->zt, S->ld)) || (rc = S->alloc(&S->sc, S_NB)) ||
        (rc = S->alloc(&S->hb, S->ld + 4)) || (rc = S->alloc(&S->hb2, S->ld + 4)) ||
        (rc = S->alloc(&S->gv, max_views)) || (rc = S->alloc(&S->hv, max_views)) ||
        (rc = S->alloc(&S->rv, max_views)) || (rc = S->alloc(&S->dir, max_views)) ||
        (rc = S->alloc(&S->alphas, 32)) || (rc = S->alloc(&S->thk, max_views)) ||
        (rc = S->alloc(&S->part_md, md_part_doubles(S->md_blocks))) ||
        (rc = S->alloc(&S->part_md2, md_part_doubles(S->md_blocks))) ||
        (rc = S->alloc(&S->part_gram, (size_t)S->gram_blocks * 64 * 64)) ||
        (rc = S->alloc(&S->part_fwd, (size_t)3 * c.kmin * max_views * S->nchunks)) ||
        (rc = S->alloc(&S->gkb, 2 * (size_t)S->kcap + 2)) || (rc = S->alloc(&S->status, 1)) ||
        (rc = S->alloc(&S->kout, 1)) || (rc = S->alloc(&S->accepted, 1)) ||
        (rc = S->alloc(&S->Ahat, (size_t)c.kmin * S->mmax)) || (rc = S->alloc(&S->evec, S->mmax)) ||
        (rc = S->alloc(&S->vp_GA, S->ld * S->ld)) || (rc = S->alloc(&S->vp_ab, S->ld)) ||
        (rc = S->alloc(&S->vp_M, 16 * 16)) || (rc = S->alloc(&S->vp_y, 16)) ||
        (rc = S->alloc(&S->vp_gd, max_views)) || (rc = S->alloc(&S->vp_en2, max_views)) ||
        (rc = S->alloc(&S->vp_ETr, (size_t)c.kmin * max_views)) ||
        (rc = S->alloc(&S->vp_Ate, (size_t)c.kmin * max_views)) ||
        (rc = S->alloc(&S->vp_Y, (size_t)c.kmin * max_views))) {
        delete S;
        return rc;
    }
    if (c.temporal == TEMPORAL_OF && nframes > 1) {
        const int64_t npix = (int64_t)geom->nx * geom->ny;
        if ((rc = S->alloc(&S->flow, (size_t)(2 * (nframes - 1) * npix))) ||
            (rc = S->alloc(&S->of_work, of_work_floats(geom->nx, geom->ny, nframes))) ||
            (rc = S->alloc(&S->of_part, of_part_doubles(geom->nx, geom->ny, nframes))) ||
            (rc = S->alloc(&S->of_acc, (size_t)(nframes * npix)))) {
            delete S;
            return rc;
        }
        if (hipMemset(S->flow, 0, sizeof(float) * 2 * (nframes - 1) * npix) != hipSuccess) {
            delete S;
            return NLRMM_EHIP;
        }
    }
    double al[32];
    for (int q = 0; q < 32; ++q) al[q] = c.alpha0 * pow(c.beta, q);
    if (hipMemcpy(S->alphas, al, sizeof(al), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(S->sc, 0, sizeof(double) * S_NB) != hipSuccess ||
        hipMemset(S->status, 0, sizeof(int)) != hipSuccess ||
        hipMemset(S->GA, 0, sizeof(double) * S->ld * S->ld) != hipSuccess ||
        hipMemset(S->GP, 0, sizeof(double) * S->ld * S->ld) != hipSuccess) {
        delete S;
        return NLRMM_EHIP;
    }
    // size the projector workspace for the widest call (rebase of kmin+1 columns)
    {
        nlrmm_batch bb{nframes, max_views, nullptr};
        size_t need = fwd_workspace_bytes(*geom, nframes, c.kmin + 1);
        const size_t nb2 = bwd_workspace_bytes(*geom, bb, 1, ctx->cu_count);
        if (nb2 > need) need = nb2;
        rc = ensure_workspace(ctx, need, nullptr);
    }
    if (rc) {
        delete S;
        return rc;
    }
    *out = S;
    return NLRMM_OK;
}

void nlrmm_solver_destroy(nlrmm_solver *S) { delete S; }

int nlrmm_solver_init(nlrmm_solver *S, const nlrmm_batch *batch, const double *theta,
                      const float *b, void *stream)
{
    if (!S || !theta || !b) return NLRMM_EINVAL;
    int rc = check_batch(batch);
    if (rc) return rc;
    if (batch->nframes != S->F) return NLRMM_ESHAPE;
    return solver_init(*S, *batch, theta, b, (hipStream_t)stream);
}

int nlrmm_solver_grid_search(nlrmm_solver *S, const nlrmm_batch *batch, double *theta,
                             const float *b, const double *shifts, int32_t ncand, int32_t ell0,
                             double *res2, int32_t *best, void *stream)
{
    if (!S || !theta || !b || !shifts) return NLRMM_EINVAL;
    int rc = check_batch(batch);
    if (rc) return rc;
    if (batch->nframes != S->F) return NLRMM_ESHAPE;
    if (ncand < 1 || ell0 < 1 || ell0 > S->kcap || ell0 > 56) return NLRMM_ESHAPE;
    if (res2 == nullptr) {
        if (ncand > S->maxV) return NLRMM_EINVAL;
        res2 = S->gv;   // scratch of max_views doubles
    }
    return grid_search(*S, *batch, theta, b, shifts, ncand, ell0, res2, best,
                       (hipStream_t)stream);
}

int nlrmm_solver_offset_sensitivity(nlrmm_solver *S, const nlrmm_batch *batch,
                                    const double *theta, const float *b, int32_t iters,
                                    double *out, float *up, void *stream)
{
    if (!S || !theta || !b || !out) return NLRMM_EINVAL;
    int rc = check_batch(batch);
    if (rc) return rc;
    if (batch->nframes != S->F || batch->nviews > S->maxV) return NLRMM_ESHAPE;
    if (iters < 1) return NLRMM_EINVAL;
    if (S->cfg.temporal == TEMPORAL_OF && S->F > 1) return NLRMM_ENOTSUP;
    return offset_sensitivity(*S, *batch, theta, b, iters, out, up, (hipStream_t)stream);
}

int nlrmm_solver_outer(nlrmm_solver *S, const nlrmm_batch *batch, double *theta, const float *b,
                       double delta, void *stream)
{
    if (!S || !theta || !b) return NLRMM_EINVAL;
    if (!(delta >= 0.0)) return NLRMM_EINVAL;
    int rc = check_batch(batch);
    if (rc) return rc;
    if (batch->nframes != S->F) return NLRMM_ESHAPE;
    if (S->ell != S->cfg.kmin + 1) return NLRMM_EINVAL;   // not initialised
    return solver_outer(*S, *batch, theta, b, delta, (hipStream_t)stream);
}

int nlrmm_solver_set_launch(nlrmm_solver *S, int32_t per_frame, const int64_t *view_off_host,
                            int32_t nframes)
{
    if (!S) return NLRMM_EINVAL;
    if (per_frame && (!view_off_host || nframes != S->F)) return NLRMM_EINVAL;
    S->plain = per_frame ? 1 : 0;
    S->vo_host.clear();
    if (per_frame) S->vo_host.assign(view_off_host, view_off_host + nframes + 1);
    return NLRMM_OK;
}

int nlrmm_solver_state(nlrmm_solver *S, float **u, float **V, double **scal, int32_t **status,
                       int32_t *ell)
{
    if (!S) return NLRMM_EINVAL;
    if (u) *u = S->u;
    if (V) *V = S->V;
    if (scal) *scal = S->sc;
    if (status) *status = S->status;
    if (ell) *ell = S->ell;
    return NLRMM_OK;
}

int nlrmm_solver_read(nlrmm_solver *S, float *u_out, double *scal_out, int32_t *status_out,
                      void *stream)
{
    if (!S) return NLRMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (u_out &&
        hipMemcpyAsync(u_out, S->u, sizeof(float) * S->n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return NLRMM_EHIP;
    if (scal_out && hipMemcpyAsync(scal_out, S->sc, sizeof(double) * S_NB,
                                   hipMemcpyDeviceToDevice, s) != hipSuccess)
        return NLRMM_EHIP;
    if (status_out && hipMemcpyAsync(status_out, S->status, sizeof(int32_t),
                                     hipMemcpyDeviceToDevice, s) != hipSuccess)
        return NLRMM_EHIP;
    return NLRMM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// standalone Krylov entry points (scratch from the context's Krylov workspace)
// ---------------------------------------------------------------------------
namespace nlrmm {

// Carve a non-owning Solver view with scratch in ctx->kws.
static int scratch_view(nlrmm_ctx *ctx, Solver &S, int64_t n, int64_t m, int kcap, int kmin,
                        hipStream_t s)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_blocks(S, n, m);
    const int64_t big = n > m ? n : m;
    const size_t bytes = al(sizeof(float) * n) * 2 + al(sizeof(float) * m) +
                         al(sizeof(float) * (size_t)kmin * big) +
                         al(sizeof(double) * md_part_doubles(S.md_blocks)) * 2 +
                         al(sizeof(double) * (size_t)S.gram_blocks * 64 * 64) +
                         al(sizeof(double) * (kcap + 4)) * 2 + al(sizeof(double) * kcap * 16) +
                         al(sizeof(double) * (kcap + 4)) + al(sizeof(int) * 4) + 4096;
    int rc = ensure_buffer(ctx->kws, bytes, s);
    if (rc) return rc;
    char *p = (char *)ctx->kws.ptr;
    auto take = [&](size_t b) {
        char *q = p;
        p += al(b);
        return (void *)q;
    };
    S.u = (float *)take(sizeof(float) * n);
    S.r = (float *)take(sizeof(float) * n);
    S.rho = (float *)take(sizeof(float) * m);
    S.Vtmp = (float *)take(sizeof(float) * (size_t)kmin * big);
    S.part_md = (double *)take(sizeof(double) * md_part_doubles(S.md_blocks));
    S.part_md2 = (double *)take(sizeof(double) * md_part_doubles(S.md_blocks));
    S.part_gram = (double *)take(sizeof(double) * (size_t)S.gram_blocks * 64 * 64);
    S.hb = (double *)take(sizeof(double) * (kcap + 4));
    S.hb2 = (double *)take(sizeof(double) * (kcap + 4));
    S.T = (double *)take(sizeof(double) * kcap * 16);
    S.zt = (double *)take(sizeof(double) * (kcap + 4));
    S.kout = (int *)take(sizeof(int) * 4);
    S.ctx = ctx;
    S.n = n;
    return NLRMM_OK;
}

}  // namespace nlrmm

extern "C" {

int nlrmm_tv_weights(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, int32_t temporal,
                     const float *u, double eps, float *w, void *stream)
{
    if (!ctx || !u || !w || !(eps > 0.0)) return NLRMM_EINVAL;
    int rc = check_geom(geom);
    if (rc) return rc;
    if (nframes < 1) return NLRMM_ESHAPE;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return k_psi_weights(u, geom->nx, geom->ny, nframes, temporal, (float)eps, w,
                         (hipStream_t)stream);
}

int nlrmm_gram_psi(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, int32_t temporal,
                   int32_t ell, const float *V, const float *w, double *G, int32_t ldg,
                   int32_t precision, void *stream)
{
    if (!ctx || !V || !w || !G) return NLRMM_EINVAL;
    if (precision < 0 || precision > 2) return NLRMM_ENOTSUP;
    int rc = check_geom(geom);
    if (rc) return rc;
    if (nframes < 1 || ell < 1 || ell > 64 || ldg < ell) return NLRMM_ESHAPE;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    Solver S;
    const int64_t n = (int64_t)nframes * geom->nx * geom->ny;
    if ((rc = scratch_view(ctx, S, n, 1, ell + 1, 2, (hipStream_t)stream))) return rc;
    return k_gram_psi(V, n, ell, w, geom->nx, geom->ny, nframes, temporal, S.part_gram,
                      S.gram_blocks, G, ldg, (hipStream_t)stream, precision);
}

static int theta_args(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, int32_t temporal,
                      const float *flow)
{
    if (!ctx) return NLRMM_EINVAL;
    int rc = check_geom(geom);
    if (rc) return rc;
    if (nframes < 1) return NLRMM_ESHAPE;
    if (temporal < 0 || temporal > 2) return NLRMM_ENOTSUP;
    if (temporal == TEMPORAL_OF && nframes > 1) {
        if (!flow) return NLRMM_EINVAL;
        if (geom->nx < 2 || geom->ny < 2) return NLRMM_ESHAPE;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return NLRMM_OK;
}

int nlrmm_of_estimate(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, const float *u,
                      double gamma, double ridge, int32_t iters, float *flow, void *stream)
{
    if (!ctx || !u || !flow || !(gamma >= 0.0) || !(ridge >= 0.0) || !(gamma < HUGE_VAL) ||
        !(ridge < HUGE_VAL) || iters < 0 || iters > 100000)
        return NLRMM_EINVAL;
    int rc = theta_args(ctx, geom, nframes, TEMPORAL_OF, flow);
    if (rc) return rc;
    if (nframes < 2) return NLRMM_OK;
    if (nframes - 1 > 65535) return NLRMM_ESHAPE;
    const size_t wf = of_work_floats(geom->nx, geom->ny, nframes);
    const size_t pd = of_part_doubles(geom->nx, geom->ny, nframes);
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ensure_buffer(ctx->kws, sizeof(float) * wf + sizeof(double) * pd + 256, s)))
        return rc;
    double *part = (double *)ctx->kws.ptr;
    float *work = (float *)(part + pd);
    return k_of_estimate(u, geom->nx, geom->ny, nframes, (float)gamma, (float)ridge, iters, flow,
                         work, part, s);
}

int nlrmm_theta_apply(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, int32_t temporal,
                      const float *flow, const float *u, float *out, void *stream)
{
    if (!u || !out) return NLRMM_EINVAL;
    int rc = theta_args(ctx, geom, nframes, temporal, flow);
    if (rc) return rc;
    return k_psi_apply(u, geom->nx, geom->ny, nframes, temporal, out, (hipStream_t)stream, flow);
}

int nlrmm_theta_weights(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes,
                        int32_t temporal, const float *flow, const float *u, double eps,
                        float *w, void *stream)
{
    if (!u || !w || !(eps > 0.0)) return NLRMM_EINVAL;
    int rc = theta_args(ctx, geom, nframes, temporal, flow);
    if (rc) return rc;
    return k_psi_weights(u, geom->nx, geom->ny, nframes, temporal, (float)eps, w,
                         (hipStream_t)stream, flow);
}

int nlrmm_theta_grad_add(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes,
                         int32_t temporal, const float *flow, const float *u, const float *w,
                         double eps, const double *lambda, float *r, void *stream)
{
    if (!u || !r || !lambda || (!w && !(eps > 0.0))) return NLRMM_EINVAL;
    int rc = theta_args(ctx, geom, nframes, temporal, flow);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int nx = geom->nx, ny = geom->ny;
    if ((rc = k_tv_grad_add(u, w, nx, ny, nframes, temporal, lambda, r, s, (float)eps))) return rc;
    if (temporal != TEMPORAL_OF || nframes < 2) return NLRMM_OK;
    if ((rc = ensure_buffer(ctx->kws, sizeof(long long) * (size_t)nframes * nx * ny, s)))
        return rc;
    return k_of_grad_add(u, w, flow, nx, ny, nframes, lambda, r, (long long *)ctx->kws.ptr, s,
                         (float)eps);
}

int nlrmm_gram_theta(nlrmm_ctx *ctx, const nlrmm_geom *geom, int32_t nframes, int32_t temporal,
                     const float *flow, int32_t ell, const float *V, const float *w, double *G,
                     int32_t ldg, int32_t precision, void *stream)
{
    if (!V || !w || !G) return NLRMM_EINVAL;
    if (precision < 0 || precision > 2) return NLRMM_ENOTSUP;
    int rc = theta_args(ctx, geom, nframes, temporal, flow);
    if (rc) return rc;
    if (ell < 1 || ell > 64 || ldg < ell) return NLRMM_ESHAPE;
    Solver S;
    const int64_t n = (int64_t)nframes * geom->nx * geom->ny;
    if ((rc = scratch_view(ctx, S, n, 1, ell + 1, 2, (hipStream_t)stream))) return rc;
    return k_gram_psi(V, n, ell, w, geom->nx, geom->ny, nframes, temporal, S.part_gram,
                      S.gram_blocks, G, ldg, (hipStream_t)stream, precision, nullptr, 0.0f, flow);
}

int nlrmm_gks_solve(nlrmm_ctx *ctx, int32_t ell, const double *GA, const double *GP,
                    int32_t ldg, const double *rb, const double *scal, double lam_fix, double *z,
                    double *out, int32_t *status, void *stream)
{
    if (!ctx || !GA || !GP || !rb || !scal || !z || !out || !status) return NLRMM_EINVAL;
    if (ell < 1 || ell > 56 || ldg < ell) return NLRMM_ESHAPE;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return k_gks_solve(GA, GP, ldg, rb, scal, ell, lam_fix, z, out, status, (hipStream_t)stream);
}

int nlrmm_gks_expand(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                     const double *theta, int32_t ell, int32_t temporal, float *V, float *AV,
                     const double *z, const float *b, const float *w, const double *lambda,
                     double *GA, int32_t ldg, double *rb, double breakdown_tol,
                     int32_t *status, void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_FORWARD | NLRMM_OPS_BACKWARD, geom);
    if (rc) return rc;
    if (!ctx || !theta || !V || !AV || !z || !b || !w || !lambda || !GA || !rb || !status)
        return NLRMM_EINVAL;
    if ((rc = check_batch(batch))) return rc;
    if (ell < 1 || ell > 55 || ldg < ell + 1) return NLRMM_ESHAPE;
    if (temporal < 0 || temporal > 1) return NLRMM_ENOTSUP;   // no velocity argument here
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    hipStream_t s = (hipStream_t)stream;
    Solver S;
    const int64_t n = (int64_t)batch->nframes * geom->nx * geom->ny;
    const int64_t m = batch->nviews * geom->nbins;
    if ((rc = scratch_view(ctx, S, n, m, ell + 2, 2, s))) return rc;
    S.g = *geom;
    S.F = batch->nframes;
    S.cfg.temporal = temporal;
    S.cfg.breakdown_tol = breakdown_tol;
    S.V = V;
    S.AV = AV;
    S.GA = GA;
    S.ld = ldg;
    S.rb = rb;
    S.w = w ? const_cast<float *>(w) : nullptr;
    S.w_from_u = false;   // the residual uses the caller's weights
    S.status = status;
    S.ell = ell;
    // z and lambda are read through the solver's scalar slots: point them at the caller's
    S.z = const_cast<double *>(z);
    S.sc = const_cast<double *>(lambda) - S_LAM;
    if ((rc = k_gemv(V, n, ell, z, 1.0, nullptr, 0.0, n, S.u, s))) return rc;
    return expand(S, *batch, theta, b, s);
}

int nlrmm_recycle_compress(nlrmm_ctx *ctx, int64_t n, int64_t m, int32_t ell, int32_t kmin,
                           float *V, float *AV, double *GA, const double *GP, int32_t ldg,
                           double *rb, const double *lambda, double *z, int32_t precision,
                           int32_t *status, void *stream)
{
    if (!ctx || !V || !AV || !GA || !GP || !rb || !lambda || !z || !status) return NLRMM_EINVAL;
    if (precision != 0 && precision != 2) return NLRMM_ENOTSUP;
    if (n < 1 || m < 1 || kmin < 2 || kmin > 16 || ell < kmin || ell > 56 || ldg < ell)
        return NLRMM_ESHAPE;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    hipStream_t s = (hipStream_t)stream;
    Solver S;
    int rc = scratch_view(ctx, S, n, m, ell + 2, kmin, s);
    if (rc) return rc;
    S.V = V;
    S.AV = AV;
    S.GA = GA;
    S.GP = const_cast<double *>(GP);
    S.ld = ldg;
    S.rb = rb;
    S.z = z;
    S.sc = const_cast<double *>(lambda) - S_LAM;
    S.status = status;
    S.ell = ell;
    S.cfg.kmin = kmin;
    S.cfg.compress_precision = precision;
    nlrmm_batch b{1, m, nullptr};
    S.g.nbins = 1;   // m_of(S, b) = nviews * nbins = m
    return compress(S, b, s);
}

}  // extern "C"
