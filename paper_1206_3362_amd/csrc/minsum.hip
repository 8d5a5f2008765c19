// Min-sum belief propagation (flooding schedule, float32): the BP reference
// decoder the paper sets FWBF against (Sections I and V).  One workgroup
// decodes one frame at a time (persistent grid).  Per frame in LDS:
//   L, P     channel values and posteriors, one float per bit;
//   check m  min1, min2 of |Q| over N(m), the list position of the first
//            minimum, the sign parity of all Q and one sign bit per member;
//            this compressed state gives every R_{m,n} of the iteration:
//            R = (sign parity xor own sign) * r(n holds the minimum ? min2 : min1),
//            r(x) = c x (normalised) or max(x - c, 0) (offset);
//   z, syndrome count.
// Iteration: check phase (Q = P - R_old member by member, new state), then
// bit phase (P = L + sum of R in ascending check order, z = [P < 0]), then
// the syndrome.  The check state of m is read and rewritten by the thread
// that owns m, so it needs no second copy.  Results equal the oracle's
// literal per-edge computation bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "frames.h"
#include "internal.h"

namespace fwbf {
namespace {

struct MsArgs {
    const float *y;
    int64_t F, stride;
    uint32_t *z;
    int32_t *iters;
    uint8_t *ok;
    const uint32_t *col, *row;
    const uint8_t *coldeg, *rowdeg;
    int N, M, Z, mb, nb, dvmax, dcmax, multi;
    uint32_t magZ, maskZ;
    int offset, max_iter;
    float c;
    int o_L, o_P, o_m1, o_m2, o_pos, o_sp, o_sg, o_z, o_ctl, o_col, o_row, o_cdeg, o_rdeg, lds_bytes;
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t mag, uint32_t mask)
{
    return __umulhi(n, mag) + (n & mask);
}

// R_{m,n} of the member at list position q
__device__ __forceinline__ float msg(const MsArgs &a, float m1, float m2, uint32_t pos, uint32_t neg, uint32_t q)
{
    float mag = q == pos ? m2 : m1;
    if (a.offset) {
        mag = mag - a.c;
        mag = mag > 0.0f ? mag : 0.0f;
    } else {
        mag = a.c * mag;
    }
    return neg ? -mag : mag;
}

template <int T>
__global__ __launch_bounds__(T) void minsum_kernel(MsArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float *L = (float *)(smem + a.o_L);
    float *P = (float *)(smem + a.o_P);
    float *sm1 = (float *)(smem + a.o_m1);
    float *sm2 = (float *)(smem + a.o_m2);
    uint8_t *spos = smem + a.o_pos;
    uint8_t *ssp = smem + a.o_sp;
    unsigned long long *ssg = (unsigned long long *)(smem + a.o_sg);
    uint32_t *zw = (uint32_t *)(smem + a.o_z);
    int *ctl = (int *)(smem + a.o_ctl);
    uint32_t *col = (uint32_t *)(smem + a.o_col);
    uint32_t *row = (uint32_t *)(smem + a.o_row);
    uint8_t *cdeg = smem + a.o_cdeg;
    uint8_t *rdeg = smem + a.o_rdeg;

    const int tid = threadIdx.x, lane = tid & 63;
    const int N = a.N, M = a.M, Z = a.Z;
    for (int t = tid; t < a.nb * a.dvmax; t += T) col[t] = a.col[t];
    for (int t = tid; t < a.mb * a.dcmax; t += T) row[t] = a.row[t];
    for (int t = tid; t < a.nb; t += T) cdeg[t] = a.coldeg[t];
    for (int t = tid; t < a.mb; t += T) rdeg[t] = a.rowdeg[t];
    const int Nr = (N + 63) & ~63, Mr = (M + 63) & ~63, NW = (N + 31) >> 5;

    // parity of check m under the hard decisions in zw
    auto parity = [&](int m) {
        const uint32_t i = fdiv(m, a.magZ, a.maskZ);
        const int r = m - (int)i * Z;
        uint32_t par = 0;
        for (int q = 0; q < rdeg[i]; q++) {
            const uint32_t e = row[i * a.dcmax + q];
            int cc = r + (int)(e & 0xFFFF);
            cc -= cc >= Z ? Z : 0;
            const uint32_t n = (e >> 16) * Z + cc;
            par ^= (zw[n >> 5] >> (n & 31)) & 1;
        }
        return par;
    };
    // unsatisfied checks, left in ctl[0] after the barrier
    auto syndrome_weight = [&]() {
        if (tid == 0) ctl[0] = 0;
        __syncthreads();
        for (int m = tid; m < Mr; m += T) {
            const bool par = m < M && parity(m);
            const unsigned long long b = __ballot(par);
            if (lane == 0 && b) atomicAdd(&ctl[0], __popcll(b));
        }
        __syncthreads();
        return ctl[0];
    };

    const FrameRange fr = xcd_frames(a.F);
    for (int64_t f = fr.first; f < fr.end; f += fr.step) {
        const float *yrow = a.y + f * a.stride;
        __syncthreads();
        for (int n = tid; n < Nr; n += T) {
            float v = 0.0f;
            if (n < N) {
                v = yrow[n];
                L[n] = v;
                P[n] = v;
            }
            const unsigned long long b = __ballot(n < N && v < 0.0f);
            if (lane == 0) { zw[n >> 5] = (uint32_t)b; zw[(n >> 5) + 1] = (uint32_t)(b >> 32); }
        }
        int weight = syndrome_weight();
        int it = 0;
        while (weight != 0 && it < a.max_iter) {
            // ---- check phase: Q = P - R_old, new compressed state ----------
            for (int m = tid; m < M; m += T) {
                const uint32_t i = fdiv(m, a.magZ, a.maskZ);
                const int r = m - (int)i * Z;
                const int deg = rdeg[i];
                const float o1 = sm1[m], o2 = sm2[m];
                const uint32_t opos = spos[m], osp = ssp[m];
                const unsigned long long osg = ssg[m];
                float m1 = __builtin_inff(), m2 = __builtin_inff();
                uint32_t pos = 0, sp = 0;
                unsigned long long sg = 0;
                for (int q = 0; q < deg; q++) {
                    const uint32_t e = row[i * a.dcmax + q];
                    int cc = r + (int)(e & 0xFFFF);
                    cc -= cc >= Z ? Z : 0;
                    const uint32_t n = (e >> 16) * Z + cc;
                    const float rold = it ? msg(a, o1, o2, opos, osp ^ (uint32_t)((osg >> q) & 1), q) : 0.0f;
                    const float Q = P[n] - rold;
                    const float av = fabsf(Q);
                    const uint32_t neg = Q < 0.0f;
                    sp ^= neg;
                    sg |= (unsigned long long)neg << q;
                    if (av < m1) { m2 = m1; m1 = av; pos = q; }
                    else if (av < m2) m2 = av;
                }
                if (deg < 2) m2 = 0.0f;  // empty minimum over N(m)\n
                sm1[m] = m1; sm2[m] = m2; spos[m] = (uint8_t)pos; ssp[m] = (uint8_t)sp; ssg[m] = sg;
            }
            __syncthreads();
            // ---- bit phase: P = L + sum of R in ascending check order -------
            for (int n = tid; n < Nr; n += T) {
                bool neg = false;
                if (n < N) {
                    const uint32_t j = fdiv(n, a.magZ, a.maskZ);
                    const int c = n - (int)j * Z;
                    const int deg = cdeg[j];
                    const uint32_t *ce = col + j * a.dvmax;
                    float s = L[n];
                    auto add = [&](uint32_t e) {
                        int rr = c - (int)(e & 0xFFFF);
                        rr += rr < 0 ? Z : 0;
                        const uint32_t m = (e >> 24) * Z + rr;
                        const uint32_t q = (e >> 16) & 0xFF;
                        s = s + msg(a, sm1[m], sm2[m], spos[m], ssp[m] ^ (uint32_t)((ssg[m] >> q) & 1), q);
                    };
                    if (!a.multi) {
                        for (int t = 0; t < deg; t++) add(ce[t]);
                    } else {
                        // one block row's shifts are listed in descending
                        // order: start at the first shift <= c, then wrap
                        int t0 = 0;
                        while (t0 < deg) {
                            const uint32_t ib = ce[t0] >> 24;
                            int t1 = t0 + 1;
                            while (t1 < deg && (ce[t1] >> 24) == ib) t1++;
                            int u = t0;
                            while (u < t1 && (int)(ce[u] & 0xFFFF) > c) u++;
                            for (int v = 0; v < t1 - t0; v++) {
                                int x = u + v;
                                x -= x >= t1 ? t1 - t0 : 0;
                                add(ce[x]);
                            }
                            t0 = t1;
                        }
                    }
                    P[n] = s;
                    neg = s < 0.0f;
                }
                const unsigned long long b = __ballot(neg);
                if (lane == 0) { zw[n >> 5] = (uint32_t)b; zw[(n >> 5) + 1] = (uint32_t)(b >> 32); }
            }
            it += 1;
            weight = syndrome_weight();
        }
        __syncthreads();
        uint32_t *zo = a.z + f * NW;
        for (int w = tid; w < NW; w += T) zo[w] = zw[w];
        if (tid == 0) {
            a.iters[f] = it;
            a.ok[f] = (uint8_t)(weight == 0);
        }
    }
}

void magic_ms(uint32_t d, uint32_t *mag, uint32_t *mask)
{
    if (d <= 1) { *mag = 0; *mask = 0xFFFFFFFFu; return; }
    *mag = (uint32_t)(((1ULL << 32) + d - 1) / d);
    *mask = 0;
}

template <int T>
hipError_t launch_ms(const MsArgs &a, hipStream_t st)
{
    auto kern = minsum_kernel<T>;
    if (a.lds_bytes > 65536)
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes);
    int blocks = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, T, a.lds_bytes);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (blocks < 1) return hipErrorInvalidConfiguration;
    const int64_t grid = std::min<int64_t>(a.F, (int64_t)blocks * cus);
    hipLaunchKernelGGL(kern, dim3((int)grid), dim3(T), a.lds_bytes, st, a);
    return hipGetLastError();
}

}  // namespace
}  // namespace fwbf

using namespace fwbf;

extern "C" int fwbf_decode_minsum(const fwbf_code *code, const fwbf_minsum_params *p, const float *y_dev,
                                  int64_t F, int64_t y_stride, uint32_t *z_dev, int32_t *iters_dev,
                                  uint8_t *ok_dev, void *stream)
{
    if (!code || !p) return fail(FWBF_E_INVALID, "null code or params");
    if (p->offset != 0 && p->offset != 1) return fail(FWBF_E_INVALID, "offset must be 0 or 1");
    if (!(p->c >= 0.0f) || !(p->c < __builtin_inff())) return fail(FWBF_E_INVALID, "c must be finite and >= 0");
    if (p->max_iter < 0) return fail(FWBF_E_INVALID, "max_iter must be >= 0");
    if (F < 0) return fail(FWBF_E_INVALID, "F must be >= 0");
    if (y_stride < code->N) return fail(FWBF_E_INVALID, "y_stride must be >= N");
    int T = p->threads_per_frame;
    if (T == 0) T = code->N <= 2048 ? 64 : code->N <= 4096 ? 128 : 256;
    if (T != 64 && T != 128 && T != 256 && T != 512 && T != 1024)
        return fail(FWBF_E_INVALID, "threads_per_frame must be 0, 64, 128, 256, 512 or 1024");
    MsArgs a;
    memset(&a, 0, sizeof a);
    a.N = code->N; a.M = code->M; a.Z = code->Z; a.mb = code->mb; a.nb = code->nb;
    a.dvmax = code->dv_max; a.dcmax = code->dc_max; a.multi = code->multi ? 1 : 0;
    a.offset = p->offset; a.c = p->c; a.max_iter = p->max_iter;
    magic_ms(code->Z, &a.magZ, &a.maskZ);
    const int Nr = (code->N + 63) / 64 * 64, M = code->M;
    int off = 0;
    auto take = [&](int bytes, int align) { off = (off + align - 1) / align * align; int o = off; off += bytes; return o; };
    a.o_L = take(4 * code->N, 16);
    a.o_P = take(4 * code->N, 16);
    a.o_m1 = take(4 * M, 4);
    a.o_m2 = take(4 * M, 4);
    a.o_sg = take(8 * M, 8);
    a.o_pos = take(M, 1);
    a.o_sp = take(M, 1);
    a.o_z = take(Nr / 8 + 8, 8);
    a.o_ctl = take(16, 4);
    a.o_col = take(4 * code->nb * code->dv_max, 4);
    a.o_row = take(4 * code->mb * code->dc_max, 4);
    a.o_cdeg = take(code->nb, 1);
    a.o_rdeg = take(code->mb, 1);
    a.lds_bytes = (off + 15) / 16 * 16;
    if (a.lds_bytes > 160 * 1024) return fail(FWBF_E_UNSUPPORTED, "frame state exceeds 160 KiB of LDS");
    if (F == 0) return FWBF_OK;
    if (!y_dev || !z_dev || !iters_dev || !ok_dev) return fail(FWBF_E_INVALID, "null buffer");
    DeviceTables t;
    int rc = device_tables(const_cast<fwbf_code *>(code), &t);
    if (rc) return rc;
    a.y = y_dev; a.F = F; a.stride = y_stride;
    a.z = z_dev; a.iters = iters_dev; a.ok = ok_dev;
    a.col = t.col; a.row = t.row; a.coldeg = t.coldeg; a.rowdeg = t.rowdeg;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    switch (T) {
    case 64: e = launch_ms<64>(a, st); break;
    case 128: e = launch_ms<128>(a, st); break;
    case 256: e = launch_ms<256>(a, st); break;
    case 512: e = launch_ms<512>(a, st); break;
    default: e = launch_ms<1024>(a, st); break;
    }
    if (e != hipSuccess) return hip_fail(e, "min-sum kernel launch");
    return FWBF_OK;
}
