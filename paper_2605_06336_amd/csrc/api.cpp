// Host side of the C ABI declared in include/nlrmm.h: argument validation, context and
// workspace management, dispatch to the HIP launchers.
#include "internal.h"

#include <math.h>
#include <new>

namespace nlrmm {

int ensure_workspace(nlrmm_ctx *ctx, size_t bytes, hipStream_t stream)
{
    return ensure_buffer(ctx->ws, bytes, stream);
}

int ensure_buffer(Workspace &ws, size_t bytes, hipStream_t stream)
{
    if (ws.bytes >= bytes) return NLRMM_OK;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
        return NLRMM_ENOMEM;   // growing the workspace would allocate inside a capture
    size_t nb = bytes + bytes / 4 + (1u << 20);
    void *p = nullptr;
    // the old buffer may still be read by queued work on any stream
    if (ws.ptr) {
        if (hipDeviceSynchronize() != hipSuccess) return NLRMM_EHIP;
        if (hipFree(ws.ptr) != hipSuccess) return NLRMM_EHIP;
        ws.ptr = nullptr;
        ws.bytes = 0;
    }
    if (hipMalloc(&p, nb) != hipSuccess) {
        (void)hipGetLastError();
        return NLRMM_ENOMEM;
    }
    ws.ptr = p;
    ws.bytes = nb;
    return NLRMM_OK;
}

int check_geom(const nlrmm_geom *g)
{
    if (!g) return NLRMM_EINVAL;
    if (g->nx < 1 || g->ny < 1 || g->nx > 16384 || g->ny > 16384) return NLRMM_ESHAPE;
    if (g->nbins < 1 || g->nbins > 65536) return NLRMM_ESHAPE;
    if (!(g->d > 0.0) || !(g->ds > 0.0) || !isfinite(g->d) || !isfinite(g->ds)) return NLRMM_EINVAL;
    if (!isfinite(g->x0) || !isfinite(g->y0) || !isfinite(g->s0)) return NLRMM_EINVAL;
    return NLRMM_OK;
}

int check_op_geom(int ops, const nlrmm_geom *g)
{
    const int rc = check_geom(g);
    if (rc) return rc;
    if ((ops & NLRMM_OPS_FORWARD) && !fwd_geom_ok(*g)) return NLRMM_ESHAPE;
    if ((ops & NLRMM_OPS_BACKWARD) && !bwd_geom_ok(*g)) return NLRMM_ESHAPE;
    return NLRMM_OK;
}

int check_batch(const nlrmm_batch *b)
{
    if (!b) return NLRMM_EINVAL;
    if (b->nframes < 1 || b->nviews < 1 || b->nviews > (int64_t)1 << 31) return NLRMM_ESHAPE;
    if (b->nframes > 1 && b->view_off == nullptr) return NLRMM_EINVAL;
    return NLRMM_OK;
}


void timing_mark(nlrmm_ctx *ctx, int which, int stop, hipStream_t s, bool eligible)
{
    if (!ctx->timing) return;
    if (ctx->timing < 0) {
        if (!stop) {
            if (!eligible) return;
            const int period = -ctx->timing;
            const bool take = ctx->acc_seen[which]++ % period == 0;
            const int i = ctx->acc_used[which];
            if (take && i < nlrmm_ctx::ACC_CAP &&
                hipEventRecord(ctx->acc_ev[which][2 * i], s) == hipSuccess)
                ctx->acc_open[which] = 1;
        } else if (ctx->acc_open[which]) {
            const int i = ctx->acc_used[which];
            if (hipEventRecord(ctx->acc_ev[which][2 * i + 1], s) == hipSuccess)
                ctx->acc_used[which] = i + 1;
            ctx->acc_open[which] = 0;
        }
        return;
    }
    if (hipEventRecord(ctx->tev[which][stop], s) == hipSuccess && stop) ctx->tev_set[which] = 1;
}

int timing_reps(nlrmm_ctx *ctx, int which, bool repeatable)
{
    const int r = (ctx->timing > 1 && repeatable) ? ctx->timing : 1;
    if (ctx->timing) ctx->tev_reps[which] = r;
    return r;
}

}  // namespace nlrmm

using namespace nlrmm;

extern "C" {

const char *nlrmm_strerror(int code)
{
    switch (code) {
        case NLRMM_OK: return "ok";
        case NLRMM_EINVAL: return "invalid argument";
        case NLRMM_ESHAPE: return "inconsistent or unsupported sizes";
        case NLRMM_EHIP: return "HIP runtime error";
        case NLRMM_ENOMEM: return "device workspace allocation failed or refused during capture";
        case NLRMM_ENOTSUP: return "unsupported option";
        default: return "unknown error";
    }
}

int nlrmm_version(void) { return 101; }

int nlrmm_check_geom(int32_t ops, const nlrmm_geom *geom)
{
    if (ops & ~(NLRMM_OPS_FORWARD | NLRMM_OPS_BACKWARD)) return NLRMM_EINVAL;
    return check_op_geom(ops, geom);
}

int nlrmm_ctx_create(nlrmm_ctx **out, int device)
{
    if (!out) return NLRMM_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return NLRMM_EINVAL;
    nlrmm_ctx *c = new (std::nothrow) nlrmm_ctx();
    if (!c) return NLRMM_ENOMEM;
    c->device = device;
    if (noalloc_scratch_address(device, &c->noalloc_scratch) != NLRMM_OK) {
        delete c;
        return NLRMM_EHIP;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        cus > 0)
        c->cu_count = cus;
    *out = c;
    return NLRMM_OK;
}

int nlrmm_ctx_set_timing(nlrmm_ctx *ctx, int enable)
{
    if (!ctx) return NLRMM_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    if (enable < -1000) enable = -1000;
    if (enable && !ctx->timing) {
        for (auto &pr : ctx->tev)
            for (auto &e : pr)
                if (!e && hipEventCreate(&e) != hipSuccess) return NLRMM_EHIP;
        ctx->tev_set[0] = ctx->tev_set[1] = 0;
    }
    if (enable < 0) {
        for (auto &pool : ctx->acc_ev)
            while ((int)pool.size() < 2 * nlrmm_ctx::ACC_CAP) {
                hipEvent_t e = nullptr;
                if (hipEventCreate(&e) != hipSuccess) return NLRMM_EHIP;
                pool.push_back(e);
            }
        for (int k = 0; k < 2; ++k) ctx->acc_used[k] = ctx->acc_seen[k] = ctx->acc_open[k] = 0;
    }
    ctx->timing = enable > 0 ? (enable > 1000 ? 1000 : enable) : enable;
    return NLRMM_OK;
}

int nlrmm_ctx_kernel_avg(nlrmm_ctx *ctx, int which, float *avg_ms, int32_t *launches)
{
    if (!ctx || !avg_ms || which < 0 || which > 1) return NLRMM_EINVAL;
    if (ctx->timing >= 0) return NLRMM_EINVAL;
    const int n = ctx->acc_used[which];
    if (launches) *launches = n;
    *avg_ms = 0.f;
    if (n == 0) return NLRMM_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    if (hipEventSynchronize(ctx->acc_ev[which][2 * n - 1]) != hipSuccess) return NLRMM_EHIP;
    double tot = 0.0;
    for (int i = 0; i < n; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->acc_ev[which][2 * i], ctx->acc_ev[which][2 * i + 1]) !=
            hipSuccess)
            return NLRMM_EHIP;
        tot += ms;
    }
    *avg_ms = (float)(tot / n);
    ctx->acc_used[which] = ctx->acc_seen[which] = ctx->acc_open[which] = 0;
    return NLRMM_OK;
}

int nlrmm_ctx_kernel_ms(nlrmm_ctx *ctx, int which, float *ms)
{
    if (!ctx || !ms || which < 0 || which > 1) return NLRMM_EINVAL;
    if (!ctx->tev_set[which]) return NLRMM_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    if (hipEventSynchronize(ctx->tev[which][1]) != hipSuccess) return NLRMM_EHIP;
    if (hipEventElapsedTime(ms, ctx->tev[which][0], ctx->tev[which][1]) != hipSuccess)
        return NLRMM_EHIP;
    *ms /= (float)ctx->tev_reps[which];
    return NLRMM_OK;
}

void nlrmm_ctx_destroy(nlrmm_ctx *ctx)
{
    if (!ctx) return;
    for (auto &pr : ctx->tev)
        for (auto &e : pr)
            if (e) (void)hipEventDestroy(e);
    for (auto &pool : ctx->acc_ev)
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    if (ctx->ws.ptr || ctx->kws.ptr) (void)hipDeviceSynchronize();
    if (ctx->ws.ptr) (void)hipFree(ctx->ws.ptr);
    if (ctx->kws.ptr) (void)hipFree(ctx->kws.ptr);
    delete ctx;
}

int nlrmm_project(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                  int32_t ncols, const float *x, const double *theta, float *y, void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_FORWARD, geom);
    if (rc) return rc;
    if (!ctx || !x || !theta || !y) return NLRMM_EINVAL;
    if (ncols < 1) return NLRMM_ESHAPE;
    if ((rc = check_batch(batch))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return launch_project(ctx, *geom, *batch, ncols, x, theta, y, nullptr, nullptr, nullptr,
                          nullptr, (hipStream_t)stream);
}

int nlrmm_backproject(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                      int32_t ncols, const float *y, const double *theta, float *x, void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_BACKWARD, geom);
    if (rc) return rc;
    if (!ctx || !x || !theta || !y) return NLRMM_EINVAL;
    if (ncols < 1) return NLRMM_ESHAPE;
    if ((rc = check_batch(batch))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return launch_backproject(ctx, *geom, *batch, ncols, y, theta, x, (hipStream_t)stream);
}

static int fan_call(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                    int32_t ncols, const float *src, const double *theta, double R, float *dst,
                    int deriv, int transpose, void *stream)
{
    int rc = check_geom(geom);
    if (rc) return rc;
    if (!ctx || !src || !theta || !dst) return NLRMM_EINVAL;
    if (!isfinite(R) || !(R >= fan_min_distance(*geom))) return NLRMM_EINVAL;
    if (ncols < 1 || (int64_t)ncols * (batch ? batch->nframes : 1) > 65535) return NLRMM_ESHAPE;
    if ((rc = check_batch(batch))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return launch_fan(*geom, *batch, ncols, R, deriv, transpose, theta, src, dst,
                      (hipStream_t)stream);
}

int nlrmm_fan_project(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                      int32_t ncols, const float *x, const double *theta, double R, float *y,
                      void *stream)
{
    return fan_call(ctx, geom, batch, ncols, x, theta, R, y, 0, 0, stream);
}

int nlrmm_fan_backproject(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                          int32_t ncols, const float *y, const double *theta, double R,
                          float *x, void *stream)
{
    return fan_call(ctx, geom, batch, ncols, y, theta, R, x, 0, 1, stream);
}

int nlrmm_fan_project_dtheta(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                             int32_t ncols, const float *x, const double *theta, double R,
                             float *dy, void *stream)
{
    return fan_call(ctx, geom, batch, ncols, x, theta, R, dy, 1, 0, stream);
}

int nlrmm_fan_backproject_dtheta(nlrmm_ctx *ctx, const nlrmm_geom *geom,
                                 const nlrmm_batch *batch, int32_t ncols, const float *r,
                                 const double *theta, double R, float *x, void *stream)
{
    return fan_call(ctx, geom, batch, ncols, r, theta, R, x, 1, 1, stream);
}

static int pat_call(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_pat_geom *pat,
                    int32_t ncols, const float *src, double p, float *dst, int mode, void *stream)
{
    int rc = check_geom(geom);
    if (rc) return rc;
    if (!ctx || !pat || !src || !dst) return NLRMM_EINVAL;
    if ((rc = pat_check(*geom, *pat, ncols, p))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return launch_pat(*geom, *pat, ncols, p, mode, src, dst, (hipStream_t)stream);
}

int nlrmm_pat_project(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_pat_geom *pat,
                      int32_t ncols, const float *x, double p, float *y, void *stream)
{
    return pat_call(ctx, geom, pat, ncols, x, p, y, 0, stream);
}

int nlrmm_pat_project_dp(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_pat_geom *pat,
                         int32_t ncols, const float *x, double p, float *dy, void *stream)
{
    return pat_call(ctx, geom, pat, ncols, x, p, dy, 1, stream);
}

int nlrmm_pat_backproject(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_pat_geom *pat,
                          int32_t ncols, const float *y, double p, float *x, void *stream)
{
    return pat_call(ctx, geom, pat, ncols, y, p, x, 2, stream);
}

int nlrmm_backproject_dtheta(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                             int32_t ncols, const float *r, const double *theta, float *x,
                             void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_BACKWARD, geom);
    if (rc) return rc;
    if (!ctx || !x || !theta || !r) return NLRMM_EINVAL;
    if (ncols < 1) return NLRMM_ESHAPE;
    if ((rc = check_batch(batch))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return launch_backproject_dtheta(ctx, *geom, *batch, ncols, r, theta, x,
                                     (hipStream_t)stream);
}

int nlrmm_project_dtheta(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                         int32_t ncols, const float *x, const double *theta, float *dy,
                         float *yproj, const float *g, double *gdot, double *dnorm2,
                         void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_FORWARD, geom);
    if (rc) return rc;
    if (!ctx || !x || !theta) return NLRMM_EINVAL;
    if (!dy && !gdot && !dnorm2) return NLRMM_EINVAL;
    if (gdot && !g) return NLRMM_EINVAL;
    if (ncols < 1) return NLRMM_ESHAPE;
    if ((rc = check_batch(batch))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return launch_project(ctx, *geom, *batch, ncols, x, theta, yproj, dy, g, gdot, dnorm2,
                          (hipStream_t)stream);
}

int nlrmm_backproject_acc(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                          int32_t ncols, const float *y, const double *theta, float *x,
                          int32_t accumulate, void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_BACKWARD, geom);
    if (rc) return rc;
    if (!ctx || !x || !theta || !y) return NLRMM_EINVAL;
    if (ncols < 1) return NLRMM_ESHAPE;
    if ((rc = check_batch(batch))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return launch_backproject(ctx, *geom, *batch, ncols, y, theta, x, (hipStream_t)stream,
                              accumulate ? 1 : 0);
}

int nlrmm_project_residual(nlrmm_ctx *ctx, const nlrmm_geom *geom, const nlrmm_batch *batch,
                           const float *x, const double *theta, const float *b, float *r,
                           double *rnorm2, void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_FORWARD, geom);
    if (rc) return rc;
    if (!ctx || !x || !theta || !b) return NLRMM_EINVAL;
    if (!r && !rnorm2) return NLRMM_EINVAL;
    if ((rc = check_batch(batch))) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    FwdOptions o;
    o.bres = b;
    o.y = r;
    o.write_resid = true;
    o.rnorm2 = rnorm2;
    return launch_project_ex(ctx, *geom, *batch, 1, x, theta, o, (hipStream_t)stream);
}

}  // extern "C"
