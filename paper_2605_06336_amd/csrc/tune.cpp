// Autotuner of the projector launch shapes.  The forward kernel can split each edge's lines
// over 1, 2, 4 or 8 waves of a block, and the backprojection can split each frame's views
// over 1, 2, 4, 8 or 16 partial images (at most 16 views per split and frame); which is
// fastest depends on the shape (grid size, views per frame, columns) and on the device.  The
// tuner runs the real operator once per candidate, times it with HIP events on the caller's
// stream and keeps the fastest in the context (and, when a cache file is set, appends it
// there).  Every candidate computes the same operator; only the summation order of FP64
// partial sums differs.  A stored split larger than a shape allows is clamped at launch.
#include "internal.h"

#include <stdio.h>

using namespace nlrmm;

namespace nlrmm {

static bool same_key(const TuneEntry &e, int kind, const nlrmm_geom &g, const nlrmm_batch &b,
                     int nc)
{
    return e.kind == kind && e.nx == g.nx && e.ny == g.ny && e.nb == g.nbins &&
           e.nframes == b.nframes && e.nviews == b.nviews && e.nc == nc;
}

int tune_lookup(const nlrmm_ctx *ctx, int kind, const nlrmm_geom &g, const nlrmm_batch &b, int nc)
{
    for (const TuneEntry &e : ctx->tune)
        if (same_key(e, kind, g, b, nc)) return e.choice;
    return 0;
}

void tune_store(nlrmm_ctx *ctx, int kind, const nlrmm_geom &g, const nlrmm_batch &b, int nc,
                int choice)
{
    bool found = false;
    for (TuneEntry &e : ctx->tune)
        if (same_key(e, kind, g, b, nc)) {
            e.choice = choice;
            found = true;
        }
    if (!found) ctx->tune.push_back({kind, g.nx, g.ny, g.nbins, b.nframes, nc, b.nviews, choice});
    if (!ctx->tune_path.empty()) {
        FILE *f = fopen(ctx->tune_path.c_str(), "a");
        if (f) {
            fprintf(f, "%d %d %d %d %d %d %lld %d\n", kind, g.nx, g.ny, g.nbins, b.nframes, nc,
                    (long long)b.nviews, choice);
            fclose(f);
        }
    }
}

}  // namespace nlrmm

namespace {

// Average time in ms of `reps` calls of fn (after one untimed call); fn returns a status.
template <class F>
int time_calls(F &&fn, hipStream_t s, int reps, float *ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return NLRMM_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return NLRMM_EHIP;
    }
    int rc = fn();
    if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = NLRMM_EHIP;
    for (int r = 0; r < reps && !rc; ++r) rc = fn();
    if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = NLRMM_EHIP;
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = NLRMM_EHIP;
    float t = 0.f;
    if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = NLRMM_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / (float)reps;
    return rc;
}

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

}  // namespace

extern "C" {

int nlrmm_ctx_set_tune_file(nlrmm_ctx *ctx, const char *path)
{
    if (!ctx) return NLRMM_EINVAL;
    ctx->tune_path = path ? path : "";
    if (!path) return NLRMM_OK;
    FILE *f = fopen(path, "r");
    if (!f) return NLRMM_OK;   // created on the first stored choice
    int kind, nx, ny, nb, nf, nc, choice;
    long long nv;
    std::vector<TuneEntry> loaded;
    while (fscanf(f, "%d %d %d %d %d %d %lld %d", &kind, &nx, &ny, &nb, &nf, &nc, &nv, &choice) ==
           8) {
        const bool ok = (kind == TUNE_FWD_SEG && (choice == 1 || choice == 2 || choice == 4 ||
                                                  choice == 8)) ||
                        (kind == TUNE_BWD_SPLIT && (choice == 1 || choice == 2 ||
                                                    choice == 4 || choice == 8 || choice == 16));
        if (!ok || nx < 1 || ny < 1 || nb < 1 || nf < 1 || nv < nf) continue;
        loaded.push_back({kind, nx, ny, nb, nf, nc, (int64_t)nv, choice});
    }
    fclose(f);
    for (const TuneEntry &e : loaded) {   // later lines win
        bool found = false;
        for (TuneEntry &t : ctx->tune)
            if (t.kind == e.kind && t.nx == e.nx && t.ny == e.ny && t.nb == e.nb &&
                t.nframes == e.nframes && t.nviews == e.nviews && t.nc == e.nc) {
                t.choice = e.choice;
                found = true;
            }
        if (!found) ctx->tune.push_back(e);
    }
    return NLRMM_OK;
}

int nlrmm_tune_query(nlrmm_ctx *ctx, int32_t kind, const nlrmm_geom *geom,
                     const nlrmm_batch *batch, int32_t ncols, int32_t *choice)
{
    if (!ctx || !choice || (kind != TUNE_FWD_SEG && kind != TUNE_BWD_SPLIT)) return NLRMM_EINVAL;
    int rc = check_geom(geom);
    if (rc || (rc = check_batch(batch))) return rc;
    const int nc = kind == TUNE_FWD_SEG ? fwd_nc_bucket(ncols) : ncols;
    *choice = tune_lookup(ctx, kind, *geom, *batch, nc);
    return NLRMM_OK;
}

int nlrmm_autotune_project(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                           int32_t ncols, const float *x, const double *theta, float *y,
                           void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_FORWARD, geom);
    if (rc) return rc;
    if (!ctx || !x || !theta || !y) return NLRMM_EINVAL;
    if (ncols < 1) return NLRMM_ESHAPE;
    if ((rc = check_batch(batch))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) return NLRMM_EINVAL;
    const int cand[4] = {1, 2, 4, 8};
    int best = 0;
    float best_ms = 0.f;
    for (int c : cand) {
        ctx->force_fwd_seg = c;
        float ms = 0.f;
        rc = time_calls([&] { return launch_project(ctx, *geom, *batch, ncols, x, theta, y,
                                                    nullptr, nullptr, nullptr, nullptr, s); },
                        s, 3, &ms);
        if (rc) break;
        if (!best || ms < best_ms) {
            best = c;
            best_ms = ms;
        }
    }
    ctx->force_fwd_seg = 0;
    if (rc) return rc;
    // the choice applies to every column group of this call (groups of at most 8 columns)
    for (int cbeg = 0; cbeg < ncols; cbeg += 8) {
        const int nc = ncols - cbeg < 8 ? ncols - cbeg : 8;
        tune_store(ctx, TUNE_FWD_SEG, *geom, *batch, fwd_nc_bucket(nc), best);
    }
    // leave y computed with the chosen shape
    return launch_project(ctx, *geom, *batch, ncols, x, theta, y, nullptr, nullptr, nullptr,
                          nullptr, s);
}

int nlrmm_autotune_backproject(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                               int32_t ncols, const float *y, const double *theta, float *x,
                               void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_BACKWARD, geom);
    if (rc) return rc;
    if (!ctx || !x || !theta || !y) return NLRMM_EINVAL;
    if (ncols < 1) return NLRMM_ESHAPE;
    if ((rc = check_batch(batch))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) return NLRMM_EINVAL;
    // all candidates fit the workspace bound of this shape: grow it once, outside the loop
    if ((rc = ensure_workspace(ctx, bwd_workspace_bytes(*geom, *batch, ncols, ctx->cu_count), s)))
        return rc;
    const int nmax = bwd_split_max(*geom, *batch);
    int best = 0;
    float best_ms = 0.f;
    for (int c = 1; c <= nmax; c *= 2) {
        ctx->force_bwd_split = c;
        float ms = 0.f;
        rc = time_calls([&] { return launch_backproject(ctx, *geom, *batch, ncols, y, theta, x, s,
                                                        0); },
                        s, 3, &ms);
        if (rc) break;
        if (!best || ms < best_ms) {
            best = c;
            best_ms = ms;
        }
    }
    ctx->force_bwd_split = 0;
    if (rc) return rc;
    tune_store(ctx, TUNE_BWD_SPLIT, *geom, *batch, ncols, best);
    return launch_backproject(ctx, *geom, *batch, ncols, y, theta, x, s, 0);
}

}  // extern "C"
