// Eb/N0 sweep captured in a HIP graph: for every noise level, frame
// generation (channel kernel) -> decoding -> error accounting, recorded once
// on a capture stream and replayed with one launch.  Counters are cleared by
// a fill kernel inside the graph (no memset nodes).  Every point has its own
// frame and output buffers, so after a replay each point's frames and
// decisions can be read back (fwbf_sweep_outputs).
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
    const size_t PF = (size_t)n_points * s->F;
    if (e == hipSuccess) e = hipMalloc(&s->y, PF * code->N * s->esz);
    if (e == hipSuccess) e = hipMalloc((void **)&s->z, PF * NW * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&s->iters, PF * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&s->ok, PF);
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
        const size_t f0 = (size_t)pnt * s->F;
        void *y = (char *)s->y + f0 * code->N * s->esz;
        uint32_t *z = s->z + f0 * NW;
        int32_t *it = s->iters + f0;
        uint8_t *ok = s->ok + f0;
        rc = fwbf_channel(code->N, s->F, 0, pool_dev, pool_n, seed, (uint32_t)pnt, sigma_host[pnt], nullptr, scale,
                          params->dtype, y, code->N, cs);
        if (rc == FWBF_OK) rc = fwbf_decode(code, params, y, s->F, code->N, z, it, ok, cs);
        if (rc == FWBF_OK)
            rc = fwbf_count(code->N, s->F, 0, z, pool_dev, pool_n, it, ok, params->max_iter,
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

extern "C" int fwbf_sweep_outputs(const fwbf_sweep *s, int point, void *y_dev, uint32_t *z_dev, int32_t *iters_dev,
                                  uint8_t *ok_dev, void *stream)
{
    if (!s) return fail(FWBF_E_INVALID, "null sweep");
    if (point < 0 || point >= s->n_points) return fail(FWBF_E_INVALID, "point out of range");
    const size_t f0 = (size_t)point * s->F, F = (size_t)s->F;
    const size_t NW = (size_t)(s->N + 31) / 32;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (y_dev)
        e = hipMemcpyAsync(y_dev, (const char *)s->y + f0 * s->N * s->esz, F * s->N * s->esz, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && z_dev) e = hipMemcpyAsync(z_dev, s->z + f0 * NW, F * NW * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && iters_dev) e = hipMemcpyAsync(iters_dev, s->iters + f0, F * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && ok_dev) e = hipMemcpyAsync(ok_dev, s->ok + f0, F, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? FWBF_OK : hip_fail(e, "sweep output copy");
}

extern "C" void fwbf_sweep_free(fwbf_sweep *s) { release(s); }
