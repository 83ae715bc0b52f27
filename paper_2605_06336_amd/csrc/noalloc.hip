// Backprojection that allocates nothing, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
//
// The backprojection's view split writes one partial image per split, summed afterwards;
// nlrmm_backproject keeps those partial images in the context workspace, which it grows on
// demand.  Here they live in `scratch`, a file-scope device array of fixed size that each GPU
// holds for the life of the process.  Host code never passes the array's name to a kernel or
// a copy (on the host that name is only a stand-in): its device address is looked up once per
// device with hipGetSymbolAddress, with that device current, when a context is created, and
// only that address is used afterwards.
//
// Every element of the scratch that a call reads was written earlier in the same call (each
// split writes every pixel of its partial image before the summation reads it), so no part of
// it needs clearing.  All calls on one GPU share its array: calls that overlap in time on one
// GPU (on different streams, or from different host threads) race on it.
#include "internal.h"

#include <mutex>

namespace nlrmm {

constexpr size_t NOALLOC_SCRATCH_FLOATS = (size_t)NLRMM_NOALLOC_SCRATCH_BYTES / sizeof(float);
static_assert(NLRMM_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

int noalloc_scratch_address(int device, void **out)
{
    if (device < 0 || device >= MAX_DEVICES || !out) return NLRMM_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess) return NLRMM_EHIP;
        if (hipSetDevice(device) != hipSuccess) return NLRMM_EHIP;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t e2 = hipSetDevice(prev);
        if (e != hipSuccess || p == nullptr || e2 != hipSuccess) {
            (void)hipGetLastError();
            return NLRMM_EHIP;
        }
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return NLRMM_OK;
}

}  // namespace nlrmm

using namespace nlrmm;

extern "C" int nlrmm_backproject_noalloc(nlrmm_ctx *ctx, const nlrmm_geom *geom,
                                         const nlrmm_batch *batch, int32_t ncols, const float *y,
                                         const double *theta, float *x, void *stream)
{
    int rc = check_op_geom(NLRMM_OPS_BACKWARD, geom);
    if (rc) return rc;
    if (!ctx || !x || !theta || !y) return NLRMM_EINVAL;
    if (ncols < 1) return NLRMM_ESHAPE;
    if ((rc = check_batch(batch))) return rc;
    if (!ctx->noalloc_scratch) return NLRMM_EHIP;
    // the split nlrmm_backproject uses for this shape; its partial images must fit the array
    if (bwd_split_bytes(ctx, *geom, *batch, ncols) > (size_t)NLRMM_NOALLOC_SCRATCH_BYTES)
        return NLRMM_ESHAPE;
    if (hipSetDevice(ctx->device) != hipSuccess) return NLRMM_EHIP;
    return launch_backproject_into(ctx, *geom, *batch, ncols, y, theta, x, (hipStream_t)stream, 0,
                                   nullptr, (float *)ctx->noalloc_scratch,
                                   (size_t)NLRMM_NOALLOC_SCRATCH_BYTES);
}
