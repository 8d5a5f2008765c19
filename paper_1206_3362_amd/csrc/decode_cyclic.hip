// One-wave-per-frame FWBF kernel for cyclic codes: H is a single N x N
// circulant whose first row has ones at the W shifts s_0 > s_1 > ... (the
// Euclidean-geometry codes of the paper's Section V).  Bit n belongs to the
// checks m = (n - s_t) mod N and check m holds the bits (m + s_t) mod N.
// Same results as the generic kernel in decode.hip.
//
//   - lane l owns bits n = 64 j + l (j < CW): 64 consecutive bits per step
//     gather from 64 consecutive checks, so the LDS reads never conflict;
//   - every round recomputes all metrics of eq. (1) (with W ~ sqrt(N) a
//     round's flips touch nearly every bit anyway);
//   - each check keeps its two smallest reliabilities with the syndrome bit
//     in the entry itself (float inputs: as the sign of both, so a term of
//     eq. (1) is a plain read); a flip toggles its checks with an LDS xor
//     that returns the old entry, which also updates the unsatisfied count;
//   - float sums follow ascending check order as the oracle does: bit n
//     starts at the first shift <= n in a doubled shift table;
//   - the block maximum is a prefix maximum over the 64 lanes of keys
//     (block << 43 | metric << 11 | 2047 - n): the block index in the top
//     bits turns the plain scan into a segmented one, and the last lane of
//     each block segment merges it into the block's LDS slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "frames.h"
#include "internal.h"

namespace fwbf {
namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int WMAX = 64;

struct CycArgs {
    const void *y;
    int64_t F, stride;
    uint32_t *z;
    int32_t *iters;
    uint8_t *ok;
    int N, W, nwin;
    int p, Geff;
    uint32_t magP, maskP;
    int single, imwbf, max_iter, cycle_exit;
    float alpha;
    int aden, anum;
    uint32_t bias, zero_val;
    int o_y, o_ent, o_q, o_z, o_shl, o_gmax, o_prv, lds_bytes;
    uint16_t sh[WMAX];  // descending
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t mag, uint32_t mask)
{
    return __umulhi(n, mag) + (n & mask);
}

__device__ __forceinline__ uint32_t orderable(float e)
{
    uint32_t u = __float_as_uint(e == 0.0f ? 0.0f : e);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWMASK, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWMASK, 0xF, true);
    return ((unsigned long long)hi << 32) | lo;
}

// inclusive prefix maximum over the 64 lanes: row_shr 1, 2, 4, 8 inside
// rows of 16 lanes, then row_bcast:15 and row_bcast:31 carry row maxima up
__device__ __forceinline__ unsigned long long scan_max(unsigned long long v)
{
    unsigned long long o;
    o = dpp64<0x111, 0xF>(v); v = o > v ? o : v;
    o = dpp64<0x112, 0xF>(v); v = o > v ? o : v;
    o = dpp64<0x114, 0xF>(v); v = o > v ? o : v;
    o = dpp64<0x118, 0xF>(v); v = o > v ? o : v;
    o = dpp64<0x142, 0xA>(v); v = o > v ? o : v;
    o = dpp64<0x143, 0xC>(v); v = o > v ? o : v;
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Check entries.  f32: {ws1, ws2} bit patterns, the signed weights of the
// term of eq. (1) (negative = satisfied check), argmin list position in a
// byte array.  i16: {m1 | m2 << 16, q | s << 31}.  i8: m1 | m2 << 8 | q << 16
// | s << 31.
template <int DT> struct CT;
template <> struct CT<FWBF_F32> {
    using Y = float;
    using E = unsigned long long;
    static constexpr E TOGGLE = 0x8000000080000000ull;
    static constexpr bool isf = true;
};
template <> struct CT<FWBF_I16> {
    using Y = int16_t;
    using E = unsigned long long;
    static constexpr E TOGGLE = 1ull << 63;
    static constexpr bool isf = false;
};
template <> struct CT<FWBF_I8> {
    using Y = int8_t;
    using E = uint32_t;
    static constexpr E TOGGLE = 1u << 31;
    static constexpr bool isf = false;
};

// syndrome bit of a check entry (float entries: a clear sign bit)
template <int DT>
__device__ __forceinline__ bool unsat(typename CT<DT>::E e)
{
    if constexpr (DT == FWBF_I8) return e >> 31;
    else if constexpr (DT == FWBF_I16) return e >> 63;
    else return !(e >> 63);
}

template <int DT, int CW>
__global__ __launch_bounds__(64) void cyclic_kernel(CycArgs a)
{
    using T = CT<DT>;
    using Y = typename T::Y;
    using E = typename T::E;
    extern __shared__ __align__(16) unsigned char smem[];
    Y *yv = (Y *)(smem + a.o_y);
    E *ent = (E *)(smem + a.o_ent);
    uint8_t *qa = smem + a.o_q;
    uint32_t *zw = (uint32_t *)(smem + a.o_z);
    uint16_t *shl = (uint16_t *)(smem + a.o_shl);
    unsigned long long *gmax = (unsigned long long *)(smem + a.o_gmax);
    uint32_t *prv = (uint32_t *)(smem + a.o_prv);

    const int lane = threadIdx.x;
    const int N = a.N, W = a.W, nwin = a.nwin;
    for (int t = lane; t < 2 * W; t += 64) shl[t] = a.sh[t < W ? t : t - W];
    // rotation start of every owned bit: the number of shifts above n
    uint32_t ust[CW];
#pragma unroll
    for (int j = 0; j < CW; j++) {
        const int n = 64 * j + lane;
        uint32_t u = 0;
        if constexpr (T::isf)
            for (int t = 0; t < W; t++) u += (int)a.sh[t] > n;
        ust[j] = u;
    }
    const int NW = (N + 31) >> 5;

    const FrameRange fr = xcd_frames(a.F);
    for (int64_t f = fr.first; f < fr.end; f += fr.step) {
        const Y *yrow = (const Y *)a.y + f * a.stride;
        __syncthreads();
        // ---- received values, z_0 = [y < 0] (Section III, Initialization) --
        float yabs[CW];
#pragma unroll
        for (int j = 0; j < CW; j++) {
            const int n = 64 * j + lane;
            Y v = (Y)0;
            if (j < nwin && n < N) v = yrow[n];
            if (j < nwin) {
                if (n < N) yv[n] = v;
                const unsigned long long b = __ballot(v < (Y)0);
                if (lane == 0) { zw[2 * j] = (uint32_t)b; zw[2 * j + 1] = (uint32_t)(b >> 32); }
            }
            if constexpr (T::isf) yabs[j] = fabsf((float)v);
            else yabs[j] = (float)(v < 0 ? -(int)v : (int)v);
        }
        for (int g = lane; g < a.Geff; g += 64) { gmax[g] = 0; prv[g] = NONE; }
        __syncthreads();

        // ---- check minima and the syndrome s_0 ---------------------------
        int weight = 0;
        for (int j = 0; j < nwin; j++) {
            const int m = 64 * j + lane;
            const bool valid = m < N;
            uint32_t par = 0, q = 0;
            if constexpr (T::isf) {
                float m1 = __builtin_inff(), m2 = __builtin_inff();
                if (valid) {
                    for (int t = 0; t < W; t++) {
                        int n = m + (int)a.sh[t];
                        n -= n >= N ? N : 0;
                        const float v = yv[n];
                        const float av = fabsf(v);
                        par ^= (uint32_t)(v < 0.0f);
                        const bool lt = av < m1;
                        m2 = lt ? m1 : fminf(m2, av);
                        q = lt ? (uint32_t)t : q;
                        m1 = lt ? av : m1;
                    }
                    const uint32_t sg = par ? 0u : 0x80000000u;
                    const uint32_t b1 = __float_as_uint(m1) | sg;
                    const uint32_t b2 = a.imwbf ? (__float_as_uint(m2) | sg) : b1;
                    ent[m] = ((unsigned long long)b2 << 32) | b1;
                    qa[m] = (uint8_t)q;
                }
            } else {
                uint32_t m1 = 0xFFFFFFFFu, m2 = 0xFFFFFFFFu;
                if (valid) {
                    for (int t = 0; t < W; t++) {
                        int n = m + (int)a.sh[t];
                        n -= n >= N ? N : 0;
                        const int v = (int)yv[n];
                        const uint32_t av = (uint32_t)(v < 0 ? -v : v);
                        par ^= (uint32_t)(v < 0);
                        const bool lt = av < m1;
                        m2 = lt ? m1 : min(m2, av);
                        q = lt ? (uint32_t)t : q;
                        m1 = lt ? av : m1;
                    }
                    if constexpr (DT == FWBF_I8)
                        ent[m] = m1 | (m2 << 8) | (q << 16) | (par << 31);
                    else
                        ent[m] = ((unsigned long long)(q | (par << 31)) << 32) | (m1 | (m2 << 16));
                }
            }
            weight += __popcll(__ballot(valid && par));
        }
        __syncthreads();

        int k = 0, okf = 0;
        if (weight == 0 || a.max_iter == 0) {
            okf = weight == 0;
        } else {
            for (;;) {
                // ---- Step 2: metrics of eq. (1), block maxima ---------------
#pragma unroll
                for (int j = 0; j < CW; j++) {
                    if (j >= nwin) break;
                    const int n = 64 * j + lane;
                    unsigned long long key = 0;
                    uint32_t g = 0;
                    if (n < N) {
                        uint32_t val;
                        if constexpr (T::isf) {
                            float S = 0.0f;
                            const uint32_t u = ust[j];
                            for (int v = 0; v < W; v++) {
                                const uint32_t idx = u + v;
                                int m = n - (int)shl[idx];
                                m += m < 0 ? N : 0;
                                const E e = ent[m];
                                uint32_t bits = (uint32_t)e;
                                if (a.imwbf) {
                                    const uint32_t t = idx - (idx >= (uint32_t)W ? W : 0);
                                    bits = qa[m] == t ? (uint32_t)(e >> 32) : bits;
                                }
                                const float term = __uint_as_float(bits);
                                S = v == 0 ? term : S + term;
                            }
                            val = orderable(__builtin_fmaf(-a.alpha, yabs[j], S));
                        } else {
                            int S = 0;
                            for (int t = 0; t < W; t++) {
                                int m = n - (int)a.sh[t];
                                m += m < 0 ? N : 0;
                                const E e = ent[m];
                                int w;
                                if constexpr (DT == FWBF_I8) {
                                    const uint32_t qq = (e >> 16) & 0x3F;
                                    w = (int)((a.imwbf && qq == (uint32_t)t) ? (e >> 8) & 0xFF : e & 0xFF);
                                } else {
                                    const uint32_t lo = (uint32_t)e, qq = (uint32_t)(e >> 32) & 0x3F;
                                    w = (int)((a.imwbf && qq == (uint32_t)t) ? lo >> 16 : lo & 0xFFFF);
                                }
                                S += unsat<DT>(e) ? w : -w;
                            }
                            val = (uint32_t)(a.aden * S - a.anum * (int)yabs[j] + (int)a.bias);
                        }
                        g = fdiv(n, a.magP, a.maskP);
                        key = ((unsigned long long)g << 43) | ((unsigned long long)val << 11) | (uint32_t)(2047 - n);
                    }
                    const unsigned long long best = scan_max(key);
                    // last lane of its block segment inside this window
                    const bool last = n < N && (lane == 63 || n + 1 >= N || fdiv(n + 1, a.magP, a.maskP) != g);
                    if (last) atomicMax(&gmax[g], best);
                }
                __syncthreads();

                // ---- choose at most one bit per block ----------------------
                int any = 0, dif = 0;
                for (int g = lane; g < a.Geff; g += 64) {
                    const unsigned long long key = gmax[g];
                    gmax[g] = 0;
                    const uint32_t val = (uint32_t)(key >> 11);
                    const uint32_t n = 2047u - (uint32_t)(key & 2047u);
                    const bool flip = a.single || val > a.zero_val;
                    const uint32_t cur = flip ? n : NONE;
                    dif |= cur != prv[g];
                    any |= flip;
                    prv[g] = cur;
                }
                const bool anyf = __ballot(any) != 0, diff = __ballot(dif) != 0;
                if (a.cycle_exit) {
                    if (!anyf) {  // no flip: fixed point until K_max
                        k = a.max_iter;
                        break;
                    }
                    if (!diff) {
                        // same flips as the round before: the states alternate,
                        // z_{K_max} = z_k if K_max - k is even, else z_k ^ flips
                        if ((a.max_iter - k) & 1)
                            for (int g = lane; g < a.Geff; g += 64) {
                                const uint32_t n = prv[g];
                                if (n != NONE) atomicXor(&zw[n >> 5], 1u << (n & 31));
                            }
                        k = a.max_iter;
                        break;
                    }
                }
                // ---- flip; toggle the checks of every flipped bit -----------
                int delta = 0;
                for (int g = lane; g < a.Geff; g += 64) {
                    const uint32_t n = prv[g];
                    if (n == NONE) continue;
                    atomicXor(&zw[n >> 5], 1u << (n & 31));
                    for (int t = 0; t < W; t++) {
                        int m = (int)n - (int)a.sh[t];
                        m += m < 0 ? N : 0;
                        const E old = atomicXor(&ent[m], T::TOGGLE);
                        delta += unsat<DT>(old) ? -1 : 1;
                    }
                }
                weight += wave_sum(delta);
                k += 1;
                if (weight == 0) { okf = 1; break; }
                if (k == a.max_iter) break;
                __syncthreads();
            }
        }
        __syncthreads();
        uint32_t *zo = a.z + f * NW;
        for (int w = lane; w < NW; w += 64) zo[w] = zw[w];
        if (lane == 0) {
            a.iters[f] = k;
            a.ok[f] = (uint8_t)okf;
        }
    }
}

template <int DT, int CW>
hipError_t launch_cyclic(const CycArgs &a, hipStream_t st)
{
    auto kern = cyclic_kernel<DT, CW>;
    if (a.lds_bytes > 65536)
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes);
    int blocks = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, 64, a.lds_bytes);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (blocks < 1) return hipErrorInvalidConfiguration;
    const int64_t grid = std::min<int64_t>(a.F, (int64_t)blocks * cus);
    hipLaunchKernelGGL(kern, dim3((int)grid), dim3(64), a.lds_bytes, st, a);
    return hipGetLastError();
}

template <int DT>
hipError_t by_cw(int CW, const CycArgs &a, hipStream_t st)
{
    switch (CW) {
    case 4: return launch_cyclic<DT, 4>(a, st);
    case 8: return launch_cyclic<DT, 8>(a, st);
    case 16: return launch_cyclic<DT, 16>(a, st);
    case 32: return launch_cyclic<DT, 32>(a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// Returns 1 if the cyclic kernel was launched, 0 if the code or the
// parameters are not covered (single circulant, 2 <= W <= 64, N <= 2048,
// block choice GROUPS or SINGLE, 64 threads per frame), < 0 on error.
int try_cyclic_decode(const fwbf_code *c, const fwbf_params *p, const void *y, int64_t F, int64_t stride,
                      uint32_t *z, int32_t *iters, uint8_t *ok, hipStream_t st)
{
    if (c->mb != 1 || c->nb != 1 || c->N > 2048) return 0;
    const int W = c->dv_max;
    if (W < 2 || W > WMAX) return 0;
    if (p->select == FWBF_TOPL) return 0;
    if (p->threads_per_frame != 0 && p->threads_per_frame != 64) return 0;
    CycArgs a;
    memset(&a, 0, sizeof a);
    a.N = c->N;
    a.W = W;
    a.nwin = (c->N + 63) / 64;
    const int CW = a.nwin <= 4 ? 4 : a.nwin <= 8 ? 8 : a.nwin <= 16 ? 16 : 32;
    const int G = p->select == FWBF_GROUPS ? p->groups : 1;
    a.p = (c->N + G - 1) / G;
    a.Geff = (c->N + a.p - 1) / a.p;
    if (a.p <= 1) { a.magP = 0; a.maskP = 0xFFFFFFFFu; }
    else { a.magP = (uint32_t)(((1ULL << 32) + a.p - 1) / a.p); a.maskP = 0; }
    a.single = p->select == FWBF_SINGLE;
    a.imwbf = p->weights == FWBF_IMWBF;
    a.max_iter = p->max_iter;
    a.cycle_exit = !(p->flags & FWBF_FLAG_NO_CYCLE_EXIT);
    a.alpha = p->weights == FWBF_WBF ? 0.0f : p->alpha;
    a.aden = p->alpha_den;
    a.anum = p->weights == FWBF_WBF ? 0 : p->alpha_num;
    if (p->dtype == FWBF_F32) {
        a.bias = 0;
        a.zero_val = 0x80000000u;  // orderable(+0)
    } else {
        const int64_t maxmag = p->dtype == FWBF_I8 ? 128 : 32768;
        const int64_t maxE = maxmag * ((int64_t)a.aden * W + a.anum);
        if (maxE >= (1LL << 30)) return 0;
        int vb = 1;
        while ((1LL << (vb - 1)) <= maxE) vb++;
        a.bias = 1u << (vb - 1);
        a.zero_val = a.bias;
    }
    // shifts of the single block, descending
    const auto &cell = c->cells[0];
    for (int t = 0; t < W; t++) a.sh[t] = (uint16_t)cell[t];
    const int esz = p->dtype == FWBF_I8 ? 1 : p->dtype == FWBF_I16 ? 2 : 4;
    const int entsz = p->dtype == FWBF_I8 ? 4 : 8;
    int off = 0;
    auto take = [&](int bytes, int align) { off = (off + align - 1) / align * align; int o = off; off += bytes; return o; };
    a.o_y = take(esz * c->N, 16);
    a.o_ent = take(entsz * c->N, 8);
    a.o_q = take(p->dtype == FWBF_F32 ? c->N : 0, 4);
    a.o_z = take(8 * a.nwin, 8);
    a.o_shl = take(4 * W, 4);
    a.o_gmax = take(8 * a.Geff, 8);
    a.o_prv = take(4 * a.Geff, 4);
    a.lds_bytes = (off + 15) / 16 * 16;
    if (a.lds_bytes > 64 * 1024) return 0;
    a.y = y; a.F = F; a.stride = stride;
    a.z = z; a.iters = iters; a.ok = ok;
    hipError_t e = p->dtype == FWBF_I8 ? by_cw<FWBF_I8>(CW, a, st)
                 : p->dtype == FWBF_I16 ? by_cw<FWBF_I16>(CW, a, st)
                                        : by_cw<FWBF_F32>(CW, a, st);
    if (e != hipSuccess) return hip_fail(e, "cyclic decode kernel launch");
    return 1;
}

}  // namespace fwbf
