// Eb/N0 sweep captured in a HIP graph: for every noise level, frame
// generation (channel kernel) -> decoding -> error accounting, recorded once
// on a capture stream and replayed with one launch.  Counters are cleared by
// a fill kernel inside the graph (no memset nodes).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

struct fwbf_sweep {
    int device = 0;
    int N = 0, n_points = 0, max_iter = 0, esz = 1;
    int64_t F = 0;
    void *y = nullptr;
    uint32_t *z = nullptr;
    int32_t *iters = nullptr;
    uint8_t *ok = nullptr;
    int64_t *counters = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace fwbf {
namespace {
__global__ void fill_i64(int64_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

void release(fwbf_sweep *s)
{
    if (!s) return;
    int cur = 0;
    const bool sw = hipGetDevice(&cur) == hipSuccess && hipSetDevice(s->device) == hipSuccess;
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    (void)hipFree(s->y);
    (void)hipFree(s->z);
    (void)hipFree(s->iters);
    (void)hipFree(s->ok);
    (void)hipFree(s->counters);
    if (sw) (void)hipSetDevice(cur);
    delete s;
}
}  // namespace
}  // namespace fwbf

using namespace fwbf;

extern "C" int fwbf_sweep_create(const fwbf_code *code, const fwbf_params *params, const float *sigma_host,
                                 int n_points, int64_t frames_per_point, const uint32_t *pool_dev, int64_t pool_n,
                                 uint64_t seed, float scale, fwbf_sweep **out)
{
    if (!out) return fail(FWBF_E_INVALID, "null out");
    *out = nullptr;
    if (!code || !params || !sigma_host || n_points < 1 || frames_per_point < 1)
        return fail(FWBF_E_INVALID, "invalid argument");
    if (pool_dev && pool_n < 1) return fail(FWBF_E_INVALID, "pool_n must be >= 1");
    if (params->max_iter < 0 || params->max_iter > 8192) return fail(FWBF_E_INVALID, "max_iter out of range");
    for (int i = 0; i < n_points; i++)
        if (!(sigma_host[i] >= 0.0f)) return fail(FWBF_E_INVALID, "sigma must be >= 0");
    fwbf_sweep *s = new (std::nothrow) fwbf_sweep;
    if (!s) return fail(FWBF_E_NOMEM, "out of host memory");
    s->N = code->N;
    s->n_points = n_points;
    s->F = frames_per_point;
    s->max_iter = params->max_iter;
    s->esz = params->dtype == FWBF_I8 ? 1 : params->dtype == FWBF_I16 ? 2 : 4;
    const int NW = (code->N + 31) / 32;
    const int64_t nc = (int64_t)n_points * (7 + params->max_iter);
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc(&s->y, (size_t)s->F * code->N * s->esz);
    if (e == hipSuccess) e = hipMalloc((void **)&s->z, (size_t)s->F * NW * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&s->iters, (size_t)s->F * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&s->ok, (size_t)s->F);
    if (e == hipSuccess) e = hipMalloc((void **)&s->counters, (size_t)nc * 8);
    if (e != hipSuccess) {
        release(s);
        return hip_fail(e, "sweep buffers");
    }
    // device tables must exist before capture (their upload is synchronous)
    DeviceTables tb;
    int rc = device_tables(const_cast<fwbf_code *>(code), &tb);
    if (rc) { release(s); return rc; }
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) { release(s); return hip_fail(e, "capture stream"); }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) { (void)hipStreamDestroy(cs); release(s); return hip_fail(e, "begin capture"); }
    hipLaunchKernelGGL(fill_i64, dim3(1), dim3(256), 0, cs, s->counters, nc);
    rc = hipGetLastError() == hipSuccess ? FWBF_OK : fail(FWBF_E_HIP, "fill launch");
    for (int pnt = 0; pnt < n_points && rc == FWBF_OK; pnt++) {
        rc = fwbf_channel(code->N, s->F, 0, pool_dev, pool_n, seed, (uint32_t)pnt, sigma_host[pnt], nullptr, scale,
                          params->dtype, s->y, code->N, cs);
        if (rc == FWBF_OK) rc = fwbf_decode(code, params, s->y, s->F, code->N, s->z, s->iters, s->ok, cs);
        if (rc == FWBF_OK)
            rc = fwbf_count(code->N, s->F, 0, s->z, pool_dev, pool_n, s->iters, s->ok, params->max_iter,
                            s->counters + (int64_t)pnt * (7 + params->max_iter), cs);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc != FWBF_OK) {
        if (g) (void)hipGraphDestroy(g);
        release(s);
        return rc;
    }
    if (e != hipSuccess) { release(s); return hip_fail(e, "end capture"); }
    s->graph = g;
    e = hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { release(s); return hip_fail(e, "graph instantiate"); }
    *out = s;
    return FWBF_OK;
}

extern "C" int fwbf_sweep_launch(fwbf_sweep *s, void *stream)
{
    if (!s) return fail(FWBF_E_INVALID, "null sweep");
    hipError_t e = hipGraphLaunch(s->exec, (hipStream_t)stream);
    return e == hipSuccess ? FWBF_OK : hip_fail(e, "graph launch");
}

extern "C" int fwbf_sweep_counters(fwbf_sweep *s, int64_t *host, void *stream)
{
    if (!s || !host) return fail(FWBF_E_INVALID, "null argument");
    const size_t bytes = (size_t)s->n_points * (7 + s->max_iter) * 8;
    hipError_t e = hipMemcpyAsync(host, s->counters, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    return e == hipSuccess ? FWBF_OK : hip_fail(e, "counter copy");
}

extern "C" void fwbf_sweep_free(fwbf_sweep *s) { release(s); }
