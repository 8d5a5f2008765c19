// Frame generation and error accounting kernels.
//
// Channel (Section II: BPSK s = 1 - 2c; Section V: AWGN of variance N0/2):
// one thread per four consecutive bits of a frame, one Philox4x32-10 block
// (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2,
// 3", SC 2011) per thread, two Box-Muller pairs per block.
//
// Accounting (Section V: bit errors, codeword errors, average iterations):
// one wave per frame; per-block partial sums in LDS, one global atomic per
// counter per block.  Integer sums, so the result does not depend on order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace fwbf {
namespace {

struct Philox {
    uint32_t x[4];
    __device__ __forceinline__ void run(uint32_t k0, uint32_t k1)
    {
        for (int r = 0; r < 10; r++) {
            const uint32_t l0 = 0xD2511F53u * x[0], h0 = __umulhi(0xD2511F53u, x[0]);
            const uint32_t l1 = 0xCD9E8D57u * x[2], h1 = __umulhi(0xCD9E8D57u, x[2]);
            const uint32_t n0 = h1 ^ x[1] ^ k0, n2 = h0 ^ x[3] ^ k1;
            x[0] = n0; x[1] = l1; x[2] = n2; x[3] = l0;
            k0 += 0x9E3779B9u;  // Weyl key schedule
            k1 += 0xBB67AE85u;
        }
    }
};

template <typename Y>
__device__ __forceinline__ Y quantise(float y, float scale);
template <> __device__ __forceinline__ float quantise<float>(float y, float) { return y; }
template <> __device__ __forceinline__ int8_t quantise<int8_t>(float y, float scale)
{
    return (int8_t)fminf(fmaxf(rintf(scale * y), -127.0f), 127.0f);
}
template <> __device__ __forceinline__ int16_t quantise<int16_t>(float y, float scale)
{
    return (int16_t)fminf(fmaxf(rintf(scale * y), -32767.0f), 32767.0f);
}

template <typename Y>
__global__ __launch_bounds__(256) void channel_kernel(int N, int64_t F, int64_t f0, const uint32_t *pool,
                                                      int64_t pool_n, uint32_t k0, uint32_t k1, uint32_t stream_id,
                                                      float sigma, const float *sigma_f, float scale, Y *y,
                                                      int64_t stride)
{
    const int NQ = (N + 3) >> 2;
    const int64_t total = F * NQ;
    const int NW = (N + 31) >> 5;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = idx / NQ;
        const int q = (int)(idx - f * NQ);
        const int64_t fa = f0 + f;
        Philox ph;
        ph.x[0] = (uint32_t)q;
        ph.x[1] = (uint32_t)fa;
        ph.x[2] = (uint32_t)((uint64_t)fa >> 32);
        ph.x[3] = stream_id;
        ph.run(k0, k1);
        const float sg = sigma_f ? sigma_f[f] : sigma;
        const uint32_t *cw = pool ? pool + (size_t)(fa % pool_n) * NW : nullptr;
        float g[4];
        for (int pr = 0; pr < 2; pr++) {
            // u in (0,1): 23 random bits plus one half ulp, exact in float
            const float ua = ((float)(ph.x[2 * pr] >> 9) + 0.5f) * 0x1p-23f;
            const float ub = ((float)(ph.x[2 * pr + 1] >> 9) + 0.5f) * 0x1p-23f;
            const float r = sqrtf(-2.0f * logf(ua));
            float sn, cs;
            sincospif(2.0f * ub, &sn, &cs);
            g[2 * pr] = r * cs;
            g[2 * pr + 1] = r * sn;
        }
        Y *yr = y + f * stride;
        for (int t = 0; t < 4; t++) {
            const int n = 4 * q + t;
            if (n >= N) break;
            const int c = cw ? (cw[n >> 5] >> (n & 31)) & 1 : 0;
            const float yv = __builtin_fmaf(sg, g[t], c ? -1.0f : 1.0f);
            yr[n] = quantise<Y>(yv, scale);
        }
    }
}

__global__ __launch_bounds__(256) void count_kernel(int N, int64_t F, int64_t f0, const uint32_t *z,
                                                    const uint32_t *pool, int64_t pool_n, const int32_t *iters,
                                                    const uint8_t *ok, int max_iter,
                                                    unsigned long long *counters)
{
    // per wavefront: a histogram of rounds (max_iter + 1 bins, 32-bit), then
    // 6 workgroup totals (64-bit)
    extern __shared__ unsigned long long lds_count[];
    const int nbin = max_iter + 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    uint32_t *hist = (uint32_t *)lds_count;
    unsigned long long *tot = lds_count + (nwave * nbin + 1) / 2;
    for (int t = threadIdx.x; t < nwave * nbin; t += blockDim.x) hist[t] = 0;
    for (int t = threadIdx.x; t < 6; t += blockDim.x) tot[t] = 0;
    __syncthreads();
    uint32_t *h = hist + wave * nbin;
    // a wavefront pass covers P frames of NWp lanes each (one word per lane;
    // NWp = 64 and a word loop when a frame has more than 64 words)
    const int NW = (N + 31) >> 5;
    int NWp = 1;
    while (NWp < NW && NWp < 64) NWp <<= 1;
    const int P = 64 / NWp;
    const int sub = lane / NWp, wl = lane % NWp;
    const unsigned long long smask = NWp == 64 ? ~0ull : (((1ull << NWp) - 1) << (sub * NWp));
    unsigned long long bit_err = 0, it_sum = 0, frame_err = 0, undet = 0, nfr = 0, nok = 0;
    for (int64_t fb = ((int64_t)blockIdx.x * nwave + wave) * P; fb < F; fb += (int64_t)gridDim.x * nwave * P) {
        const int64_t f = fb + sub;
        bool err = false;
        if (f < F) {
            const uint32_t *cw = pool ? pool + (size_t)((f0 + f) % pool_n) * NW : nullptr;
            for (int w = wl; w < NW; w += NWp) {
                const uint32_t d = z[f * NW + w] ^ (cw ? cw[w] : 0u);
                bit_err += __popc(d);
                err |= d != 0;
            }
        }
        const bool fe = (__ballot(err) & smask) != 0;  // some word of this lane's frame differs
        if (wl == 0 && f < F) {
            const int it = iters[f];
            const bool okf = ok[f] != 0;
            frame_err += fe;
            undet += fe && okf;
            it_sum += (unsigned long long)(int64_t)it;
            nfr += 1;
            nok += okf;
            if (it >= 0 && it <= max_iter) atomicAdd(&h[it], 1u);
        }
    }
    // totals: wavefront sums, then one LDS atomic per wavefront and counter
    unsigned long long v[6] = {bit_err, frame_err, undet, it_sum, nfr, nok};
#pragma unroll
    for (int c = 0; c < 6; c++) {
        for (int d = 32; d >= 1; d >>= 1) v[c] += __shfl_xor(v[c], d, 64);
        if (lane == 0 && v[c]) atomicAdd(&tot[c], v[c]);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 6; t += blockDim.x)
        if (tot[t]) atomicAdd(&counters[t], tot[t]);
    for (int b = threadIdx.x; b < nbin; b += blockDim.x) {
        unsigned long long sum = 0;
        for (int w = 0; w < nwave; w++) sum += hist[w * nbin + b];
        if (sum) atomicAdd(&counters[6 + b], sum);
    }
}

int grid_for(int64_t work, int block)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int64_t want = (work + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * 16));
}

}  // namespace
}  // namespace fwbf

using namespace fwbf;

extern "C" int fwbf_channel(int N, int64_t F, int64_t f0, const uint32_t *pool_dev, int64_t pool_n, uint64_t seed,
                            uint32_t stream_id, float sigma, const float *sigma_dev, float scale, int dtype,
                            void *y_dev, int64_t y_stride, void *stream)
{
    if (N < 1 || F < 0 || f0 < 0 || y_stride < N) return fail(FWBF_E_INVALID, "invalid size");
    if (pool_dev && pool_n < 1) return fail(FWBF_E_INVALID, "pool_n must be >= 1");
    if (dtype < FWBF_F32 || dtype > FWBF_I16) return fail(FWBF_E_INVALID, "unknown dtype");
    if (!(sigma >= 0.0f) && !sigma_dev) return fail(FWBF_E_INVALID, "sigma must be >= 0");
    if (F == 0) return FWBF_OK;
    if (!y_dev) return fail(FWBF_E_INVALID, "null y");
    const int64_t work = F * ((N + 3) / 4);
    const int grid = grid_for(work, 256);
    hipStream_t st = (hipStream_t)stream;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (dtype == FWBF_F32)
        hipLaunchKernelGGL(channel_kernel<float>, dim3(grid), dim3(256), 0, st, N, F, f0, pool_dev, pool_n, k0, k1,
                           stream_id, sigma, sigma_dev, scale, (float *)y_dev, y_stride);
    else if (dtype == FWBF_I8)
        hipLaunchKernelGGL(channel_kernel<int8_t>, dim3(grid), dim3(256), 0, st, N, F, f0, pool_dev, pool_n, k0, k1,
                           stream_id, sigma, sigma_dev, scale, (int8_t *)y_dev, y_stride);
    else
        hipLaunchKernelGGL(channel_kernel<int16_t>, dim3(grid), dim3(256), 0, st, N, F, f0, pool_dev, pool_n, k0,
                           k1, stream_id, sigma, sigma_dev, scale, (int16_t *)y_dev, y_stride);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FWBF_OK : hip_fail(e, "channel kernel launch");
}

extern "C" int fwbf_count(int N, int64_t F, int64_t f0, const uint32_t *z_dev, const uint32_t *pool_dev,
                          int64_t pool_n, const int32_t *iters_dev, const uint8_t *ok_dev, int max_iter,
                          int64_t *counters_dev, void *stream)
{
    if (N < 1 || F < 0 || f0 < 0 || max_iter < 0 || max_iter > 8192) return fail(FWBF_E_INVALID, "invalid size");
    if (pool_dev && pool_n < 1) return fail(FWBF_E_INVALID, "pool_n must be >= 1");
    if (F == 0) return FWBF_OK;
    if (!z_dev || !iters_dev || !ok_dev || !counters_dev) return fail(FWBF_E_INVALID, "null buffer");
    const int grid = grid_for(F * 64, 256);
    const size_t lds = sizeof(uint32_t) * 4 * (size_t)(max_iter + 1) + 8 + sizeof(unsigned long long) * 6;
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)count_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(count_kernel, dim3(grid), dim3(256), lds, (hipStream_t)stream, N, F, f0, z_dev, pool_dev,
                       pool_n, iters_dev, ok_dev, max_iter, (unsigned long long *)counters_dev);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FWBF_OK : hip_fail(e, "count kernel launch");
}
