// Internal declarations shared by the library's translation units (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>
#include <vector>
#include "../../include/nlrmm.h"

namespace nlrmm {

// Per-line packed entry of the edge-driven projector: prefix sum of the line up to
// walk position i (exclusive) and the two pixel values at positions i, i+1.
struct __attribute__((aligned(16))) PackEntry {
    double P;
    float a;
    float b;
};

struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Launch-shape cache of the autotuner: one entry per operator kind and problem shape.
enum TuneKind { TUNE_FWD_SEG = 0, TUNE_BWD_SPLIT = 1 };
struct TuneEntry {
    int kind, nx, ny, nb, nframes, nc;
    int64_t nviews;
    int choice;
};

}  // namespace nlrmm

struct nlrmm_ctx {
    int device = 0;
    nlrmm::Workspace ws;    // projector packs (reused by every projection)
    nlrmm::Workspace kws;   // scratch of the standalone Krylov entry points
    int cu_count = 256;
    // optional event timing of the dominant projector kernels (measurement aid)
    int timing = 0;
    hipEvent_t tev[2][2] = {};   // [kernel][start, stop]; 0 forward weights, 1 backprojection
    int tev_set[2] = {0, 0};
    int tev_reps[2] = {1, 1};    // launches of the timed kernel between the recorded pair
    // per-launch accumulation (timing < 0): one event pair per sampled eligible launch, from
    // a pool created when the mode is enabled; every -timing-th eligible launch is recorded
    static constexpr int ACC_CAP = 4096;
    std::vector<hipEvent_t> acc_ev[2];   // [kernel] start, stop of pair i at 2i, 2i + 1
    int acc_used[2] = {0, 0};
    int acc_seen[2] = {0, 0};
    int acc_open[2] = {0, 0};
    // autotuner: cached launch shapes, a candidate forced while tuning, optional cache file
    std::vector<nlrmm::TuneEntry> tune;
    int force_fwd_seg = 0;
    int force_bwd_split = 0;
    std::string tune_path;
    // device address of this device's fixed scratch array (nlrmm_backproject_noalloc)
    void *noalloc_scratch = nullptr;
};

namespace nlrmm {

// Grow the context workspace to at least `bytes` (refused while `stream` is capturing).
int ensure_workspace(nlrmm_ctx *ctx, size_t bytes, hipStream_t stream);
int ensure_buffer(Workspace &w, size_t bytes, hipStream_t stream);

int check_geom(const nlrmm_geom *g);
// Device address of the fixed scratch array of nlrmm_backproject_noalloc on `device`, looked
// up once per device (noalloc.hip).
int noalloc_scratch_address(int device, void **out);
// check_geom plus the kernels' limits for the operator families in `ops` (NLRMM_OPS_*)
int check_op_geom(int ops, const nlrmm_geom *g);

// Autotuner cache: the tuned choice for a shape (0 when none) and storing a new one.
int tune_lookup(const nlrmm_ctx *ctx, int kind, const nlrmm_geom &g, const nlrmm_batch &b, int nc);
void tune_store(nlrmm_ctx *ctx, int kind, const nlrmm_geom &g, const nlrmm_batch &b, int nc,
                int choice);
// Forward: waves per block sharing an edge's lines (1, 2, 4 or 8); column bucket of a group.
int fwd_seg_for(const nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int nc_bucket);
int fwd_nc_bucket(int nc);
// Backprojection: the largest view split (workspace bound) and the split a launch uses
// (forced, tuned or default, clamped to [1, bwd_split_max]).
int bwd_split_max(const nlrmm_geom &g, const nlrmm_batch &b);
int bwd_split_for(const nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols);

// Record the start / stop event of timed kernel `which` on stream s (no-op unless enabled).
// In the per-launch accumulation mode only launches marked eligible (one column, full work)
// are recorded.
void timing_mark(nlrmm_ctx *ctx, int which, int stop, hipStream_t s, bool eligible = true);
// Launches of a timed kernel between its events: the context's repeat count when timing is on
// and the launch can be repeated without changing its result, else 1.
int timing_reps(nlrmm_ctx *ctx, int which, bool repeatable);
int check_batch(const nlrmm_batch *b);

// Forward-kernel outputs and modes (see proj.hip).
struct FwdOptions {
    float *y = nullptr;            // projection [col][V][nb]
    float *dy = nullptr;           // angle derivative [col][V][nb]
    const float *g = nullptr;      // weights of the fused <D_v, g_v>
    double *gdot = nullptr;        // [col][V]
    double *dnorm2 = nullptr;      // [col][V]
    double *rnorm2 = nullptr;      // [col][V] ||y_v - b_v||^2 (residual mode)
    const float *bres = nullptr;   // residual mode: g := y - b
    const double *tdir = nullptr;  // trial angles theta + talpha[0] * tdir
    const double *talpha = nullptr;
    const int *skip = nullptr;     // device flag: skip the whole call when set
    double *part_buf = nullptr;    // caller-provided partials [3][col][V][nchunks]
    bool keep_parts = false;       // leave per-chunk partials unreduced (caller reduces)
    bool write_resid = false;      // with bres: y receives y - b
    // Normalisation folded into the packing launch (one column; x is then not read): the image
    // packed, and written to norm_out, is norm_src / ||norm_src|| with the squared norm summed
    // from norm_nblk block partials norm_part as the Krylov normalisation sums them; that sets
    // norm_scal[1] to it and tests for breakdown against sqrt(norm_scal[0]) (norm_status).
    const float *norm_src = nullptr;
    const double *norm_part = nullptr;
    int norm_nblk = 0;
    double *norm_scal = nullptr;
    double norm_tol = 0.0;
    float *norm_out = nullptr;
    int *norm_status = nullptr;
};

// Geometry limits of the projector kernels (proj.hip): the forward family needs nx, ny <=
// 4096 (line packs); the backward family needs at most 4 bin edges inside a pixel footprint
// and a staged window of at most 64 bins per 16-pixel tile (ds >= about 0.38 d).
int fwd_geom_ok(const nlrmm_geom &g);
int bwd_geom_ok(const nlrmm_geom &g);

// projector launchers (proj.hip); all arguments validated by the caller
int launch_project_ex(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols,
                      const float *x, const double *theta, const FwdOptions &o, hipStream_t s);
int fwd_chunks(const nlrmm_geom &g);
size_t fwd_workspace_bytes(const nlrmm_geom &g, int nframes, int ncols);
size_t bwd_workspace_bytes(const nlrmm_geom &g, const nlrmm_batch &b, int ncols, int cu_count);
int launch_project(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols,
                   const float *x, const double *theta, float *y, float *dy, const float *gres,
                   double *gdot, double *dnorm2, hipStream_t s);
// Optional epilogue of a one-column backprojection: x += lam * Psi^T (w * Psi u).
struct TvEpilogue {
    const float *u = nullptr;
    const float *w = nullptr;       // null: weights formed from u with eps
    const double *lamp = nullptr;   // device scalar lambda
    int temporal = 0;
    float e2 = 0.0f;                // eps^2
};
// Block partials of the inner products <X_i, x> (i < nv) and <x, x> of the image the
// backprojection writes, formed by its split-sum launch when the view split has one (the
// multidot that would read x next is then not needed): one element per thread on
// ceil(n / 256) blocks, the partials part[block][i] as k_multidot forms them.  Taken only
// when that grid is at most nblk_cap blocks; fused and nblk report what was done.
struct MdEpilogue {
    const float *X = nullptr;
    int64_t ldx = 0;
    int nv = 0;
    double *part = nullptr;
    int nblk_cap = 0;
    bool fused = false;
    int nblk = 0;
};
int launch_backproject(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols,
                       const float *y, const double *theta, float *x, hipStream_t s,
                       int accumulate = 0, const TvEpilogue *tv = nullptr,
                       MdEpilogue *md = nullptr);
// The same with the view split's partial images in a caller buffer of part_cap bytes (no
// workspace growth; NLRMM_ESHAPE when the split needs more); part_buf null: the workspace.
int launch_backproject_into(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols,
                            const float *y, const double *theta, float *x, hipStream_t s,
                            int accumulate, const TvEpilogue *tv, float *part_buf,
                            size_t part_cap, MdEpilogue *md = nullptr);
// Bytes of partial images the backprojection of this shape uses (0 without a view split).
size_t bwd_split_bytes(const nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b, int ncols);
int launch_backproject_dtheta(nlrmm_ctx *ctx, const nlrmm_geom &g, const nlrmm_batch &b,
                              int ncols, const float *y, const double *theta, float *x,
                              hipStream_t s);

// Fan-beam family (fan.hip): the smallest accepted source distance for a geometry, and the
// launcher of the four operators (deriv: angle derivative; transpose: the transposes).
double fan_min_distance(const nlrmm_geom &g);
int launch_fan(const nlrmm_geom &g, const nlrmm_batch &b, int ncols, double R, int deriv,
               int transpose, const double *theta, const float *src, float *dst, hipStream_t s);

// Photoacoustic circular-means family (pat.hip): host limits and the launcher (mode 0
// projection, 1 derivative in p, 2 transpose).
int pat_check(const nlrmm_geom &g, const nlrmm_pat_geom &pg, int ncols, double p);
int launch_pat(const nlrmm_geom &g, const nlrmm_pat_geom &pg, int ncols, double p, int mode,
               const float *src, float *dst, hipStream_t s);

}  // namespace nlrmm

#define NLRMM_HIP_CHECK(expr)                       \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return NLRMM_EHIP;    \
    } while (0)
