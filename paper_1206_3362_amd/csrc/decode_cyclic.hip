// One-wave-per-frame FWBF kernel for cyclic codes: H is a single N x N
// circulant whose first row has ones at the W shifts s_0 > s_1 > ... (the
// Euclidean-geometry codes of the paper's Section V).  Bit n belongs to the
// checks m = (n - s_t) mod N and check m holds the bits (m + s_t) mod N.
// Same results as the generic kernel in decode.hip.
//
//   - lane l owns bits n = 64 j + l (j < CW): 64 consecutive bits per step
//     gather from 64 consecutive checks, so the LDS reads never conflict;
//     the CW bits of a lane advance together, one term of eq. (1) per step;
//   - every round recomputes all metrics (with W ~ sqrt(N) a round's flips
//     touch nearly every bit anyway);
//   - each check keeps its smallest reliability as a float whose sign is the
//     syndrome bit (set = satisfied), so a term of eq. (1) is a plain read
//     and a flip toggles a check with one LDS xor that returns the old
//     entry (which also updates the unsatisfied count);
//   - float inputs: the entry holds the signed first and second minima and
//     the index of the bit holding the minimum; sums follow ascending check
//     order as the oracle does (bit n starts at the first shift <= n, read
//     from a doubled table of signed offsets that also removes the wrap);
//   - integer inputs: magnitudes are small integers, exact as floats in any
//     order, so the IMWBF exclusion becomes a per-bit correction
//     sum over the checks whose minimum the bit holds of sign * (m2 - m1),
//     updated with an LDS add whenever such a check toggles;
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
constexpr uint32_t SIGN = 0x80000000u;
constexpr int WMAX = 64;

struct CycArgs {
    const void *y;
    int64_t F, stride;
    uint32_t *z;
    int32_t *iters;
    uint8_t *ok;
    int N, W, nwin, Nx;  // Nx = N + 64 CW: length of the doubled arrays
    int p, Geff;
    uint32_t magP, maskP, magW, maskW;
    // 32-bit keys (integer metrics): block << (vb + pb) | metric << pb | pmask - pos
    int key32, vb, pb;
    int single, imwbf, max_iter, cycle_exit;
    int exec_rounds;  // report the rounds run before a repeated state (diagnostic)
    float alpha;
    int aden, anum;
    uint32_t bias, zero_val;
    // LDS offsets in bytes (the check entries sit at offset 0)
    int o_am, o_tab, o_info, o_corr, o_y, o_z, o_gmax, o_prv, o_list, o_shl, lds_bytes;
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

__device__ __forceinline__ uint32_t scan_max32(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, true));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, true));
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Y: input type; K: staged value (float: y itself; integer: the check-minimum
// key |y| << 7 | [y < 0] << 6, to which the member position t is or-ed)
template <int DT> struct CY;
template <> struct CY<FWBF_F32> { using Y = float; using K = float; };
template <> struct CY<FWBF_I16> { using Y = int16_t; using K = uint32_t; };
template <> struct CY<FWBF_I8> { using Y = int8_t; using K = uint16_t; };

template <int DT, int CW>
__global__ __launch_bounds__(64) void cyclic_kernel(CycArgs a)
{
    using Y = typename CY<DT>::Y;
    using K = typename CY<DT>::K;
    constexpr bool ISF = DT == FWBF_F32;
    extern __shared__ __align__(16) unsigned char smem[];
    // check entries at offset 0.  float: {ws1, ws2} per check; integer:
    // ws1 per check, stored for every index i < Nx as check i mod N so that
    // n + N - s needs no wrap and step j of a lane is an immediate offset
    unsigned long long *ent = (unsigned long long *)smem;
    uint32_t *ws = (uint32_t *)smem;
    uint16_t *am = (uint16_t *)(smem + a.o_am);      // float: bit holding the minimum
    int32_t *tab = (int32_t *)(smem + a.o_tab);      // float: -s_t, then N - s_t
    uint32_t *info = (uint32_t *)(smem + a.o_info);  // integer IMWBF: bit | (m2 - m1) << 16
    float *corr = (float *)(smem + a.o_corr);        // integer IMWBF: per-bit correction
    K *yv = (K *)(smem + a.o_y);                     // staged y_(i mod N) for i < Nx
    uint32_t *zw = (uint32_t *)(smem + a.o_z);
    unsigned long long *gmax = (unsigned long long *)(smem + a.o_gmax);
    uint32_t *prv = (uint32_t *)(smem + a.o_prv);
    uint32_t *gmax32 = (uint32_t *)gmax;
    uint32_t *list = (uint32_t *)(smem + a.o_list);  // bits flipped this round
    uint16_t *shl = (uint16_t *)(smem + a.o_shl);    // s_t

    const int lane = threadIdx.x;
    const int N = a.N, W = a.W, nwin = a.nwin, Nx = a.Nx;
    const bool icorr = !ISF && a.imwbf;
    const int shv = lane < W ? (int)a.sh[lane] : 0;  // s_t in lane t (read back with readlane)
    if constexpr (ISF)
        for (int t = lane; t < 2 * W; t += 64) tab[t] = t < W ? -(int)a.sh[t] : N - (int)a.sh[t - W];
    // owned bits (tail lanes address bit N - 1 and drop the result), and for
    // float inputs the rotation start: the number of shifts above n
    int nc[CW];
    uint32_t ust[CW];
#pragma unroll
    for (int j = 0; j < CW; j++) {
        nc[j] = min(64 * j + lane, N - 1);
        uint32_t u = 0;
        if constexpr (ISF)
            for (int t = 0; t < W; t++) u += __builtin_amdgcn_readlane(shv, t) > nc[j];
        ust[j] = u;
    }
    for (int t = lane; t < W; t += 64) shl[t] = a.sh[t];
    // frame-independent part of every key, and which lanes end a block
    // segment inside their window (bit j of lastm)
    // (32-bit keys: block << (vb + pb) | pmask - pos; 64-bit keys: the block)
    uint32_t kc[CW];
    uint32_t lastm = 0;
#pragma unroll
    for (int j = 0; j < CW; j++) {
        const int n = 64 * j + lane;
        kc[j] = 0;
        if (j < nwin && n < N) {
            const uint32_t g = fdiv(n, a.magP, a.maskP);
            if (a.key32) kc[j] = ((uint32_t)g << (a.vb + a.pb)) | (((1u << a.pb) - 1) - (n - g * a.p));
            else kc[j] = g;
            const bool last = lane == 63 || n + 1 >= N || fdiv(n + 1, a.magP, a.maskP) != g;
            lastm |= (uint32_t)last << j;
        }
    }
    const int NW = (N + 31) >> 5;

    const FrameRange fr = xcd_frames(a.F);
    // received values of the next frame, loaded while the current one decodes
    Y ynext[CW];
    auto prefetch = [&](int64_t ff) {
        const Y *yr = (const Y *)a.y + ff * a.stride;
#pragma unroll
        for (int j = 0; j < CW; j++) {
            const int n = 64 * j + lane;
            ynext[j] = (j < nwin && n < N) ? yr[n] : (Y)0;
        }
    };
    constexpr bool PF = CW <= 16;  // register budget
    if (PF && fr.first < fr.end) prefetch(fr.first);
    for (int64_t f = fr.first; f < fr.end; f += fr.step) {
        Y ycur[CW];
        if (PF) {
#pragma unroll
            for (int j = 0; j < CW; j++) ycur[j] = ynext[j];
            if (f + fr.step < fr.end) prefetch(f + fr.step);
        } else {
            prefetch(f);
#pragma unroll
            for (int j = 0; j < CW; j++) ycur[j] = ynext[j];
        }
        __syncthreads();
        // ---- received values, z_0 = [y < 0] (Section III, Initialization) --
#pragma unroll
        for (int j = 0; j < CW; j++) {
            const int n = 64 * j + lane;
            const Y v = ycur[j];
            if (j < nwin) {
                K kv;
                if constexpr (ISF) kv = v;
                else kv = (K)(((uint32_t)(v < 0 ? -(int)v : (int)v) << 7) | ((uint32_t)(v < 0) << 6));
                if (n < N)
                    for (int i = n; i < Nx; i += N) yv[i] = kv;
                const unsigned long long b = __ballot(v < (Y)0);
                if (lane == 0) { zw[2 * j] = (uint32_t)b; zw[2 * j + 1] = (uint32_t)(b >> 32); }
            }
        }
        for (int g = lane; g < a.Geff; g += 64) { gmax[g] = 0; prv[g] = NONE; }
        if (icorr)
            for (int n = lane; n < N; n += 64) corr[n] = 0.0f;
        __syncthreads();

        // ---- check minima and the syndrome s_0 ---------------------------
        // check m = 64 j + lane holds bits m + s_t (< Nx, no wrap needed);
        // four windows at a time
        int weight = 0;
        for (int j0 = 0; j0 < nwin; j0 += 4) {
            float m1[4], m2[4];
            uint32_t q[4], par[4];
            if constexpr (ISF) {
                unsigned long long pm[4];
#pragma unroll
                for (int jj = 0; jj < 4; jj++) { m1[jj] = __builtin_inff(); m2[jj] = __builtin_inff(); q[jj] = 0; pm[jj] = 0; }
                for (int t = 0; t < W; t++) {
                    const int base = lane + __builtin_amdgcn_readlane(shv, t) + 64 * j0;
#pragma unroll
                    for (int jj = 0; jj < 4; jj++) {
                        const float v = yv[base + 64 * jj];
                        const float av = fabsf(v);
                        pm[jj] ^= __ballot(v < 0.0f);
                        q[jj] = av < m1[jj] ? (uint32_t)t : q[jj];
                        m2[jj] = __builtin_amdgcn_fmed3f(m1[jj], m2[jj], av);  // m1 <= m2
                        m1[jj] = fminf(m1[jj], av);
                    }
                }
#pragma unroll
                for (int jj = 0; jj < 4; jj++) par[jj] = (uint32_t)(pm[jj] >> lane) & 1u;
            } else {
                // key | t: the minimum key gives m1 and its position; the
                // second smallest key gives m2 (median of m1, m2, key)
                uint32_t k1[4], k2[4], px[4];
#pragma unroll
                for (int jj = 0; jj < 4; jj++) { k1[jj] = 0xFFFFFFFFu; k2[jj] = 0xFFFFFFFFu; px[jj] = 0; }
                for (int t = 0; t < W; t++) {
                    const int base = lane + __builtin_amdgcn_readlane(shv, t) + 64 * j0;
#pragma unroll
                    for (int jj = 0; jj < 4; jj++) {
                        const uint32_t kv = yv[base + 64 * jj];
                        px[jj] ^= kv;
                        const uint32_t key = kv | (uint32_t)t;
                        k2[jj] = max(k1[jj], min(k2[jj], key));
                        k1[jj] = min(k1[jj], key);
                    }
                }
#pragma unroll
                for (int jj = 0; jj < 4; jj++) {
                    m1[jj] = (float)(k1[jj] >> 7);
                    m2[jj] = (float)(k2[jj] >> 7);
                    q[jj] = k1[jj] & 63u;
                    par[jj] = (px[jj] >> 6) & 1u;
                }
            }
#pragma unroll
            for (int jj = 0; jj < 4; jj++) {
                const int j = j0 + jj;
                const int m = 64 * j + lane;
                const bool valid = m < N;
                // bit holding the minimum (the permute runs with every lane active)
                int an = m + __builtin_amdgcn_ds_bpermute(4 * (int)q[jj], shv);
                an -= an >= N ? N : 0;
                if (valid) {
                    const uint32_t sg = par[jj] ? 0u : SIGN;
                    const uint32_t b1 = __float_as_uint(m1[jj]) | sg;
                    if constexpr (ISF) {
                        const uint32_t b2 = a.imwbf ? (__float_as_uint(m2[jj]) | sg) : b1;
                        ent[m] = ((unsigned long long)b2 << 32) | b1;
                        am[m] = (uint16_t)an;
                    } else {
                        for (int i = m; i < Nx; i += N) ws[i] = b1;
                        if (icorr) {
                            const uint32_t d = (uint32_t)(m2[jj] - m1[jj]);
                            info[m] = (uint32_t)an | (d << 16);
                            if (d) atomicAdd(&corr[an], par[jj] ? (float)d : -(float)d);
                        }
                    }
                }
                weight += __popcll(__ballot(valid && par[jj]));
            }
        }
        __syncthreads();

        int k = 0, okf = 0;
        if (weight == 0 || a.max_iter == 0) {
            okf = weight == 0;
        } else {
            for (;;) {
                // ---- Step 2: metrics of eq. (1) of every owned bit -----------
                float S[CW];
                if constexpr (ISF) {
#pragma unroll
                    for (int j = 0; j < CW; j++) S[j] = 0.0f;
                    for (int v = 0; v < W; v++) {
#pragma unroll
                        for (int j = 0; j < CW; j++) {
                            const int m = nc[j] + tab[ust[j] + v];
                            const unsigned long long e = ent[m];
                            const uint32_t bits = am[m] == (uint32_t)nc[j] ? (uint32_t)(e >> 32) : (uint32_t)e;
                            const float term = __uint_as_float(bits);
                            S[j] = v == 0 ? term : S[j] + term;
                        }
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < CW; j++) S[j] = icorr ? corr[nc[j]] : 0.0f;
                    for (int t = 0; t < W; t++) {
                        const int base = lane + N - __builtin_amdgcn_readlane(shv, t);
#pragma unroll
                        for (int j = 0; j < CW; j++) S[j] += __uint_as_float(ws[base + 64 * j]);
                    }
                }
                // ---- block maxima ------------------------------------------
#pragma unroll
                for (int j = 0; j < CW; j++) {
                    const bool valid = 64 * j + lane < N;
                    const K yn = yv[64 * j + lane];  // |y_n| from the staged frame
                    uint32_t val;
                    if constexpr (ISF) val = orderable(__builtin_fmaf(-a.alpha, fabsf(yn), S[j]));
                    else val = (uint32_t)(__mul24(a.aden, (int)S[j]) - __mul24(a.anum, (int)((uint32_t)yn >> 7)) + (int)a.bias);
                    const bool last = (lastm >> j) & 1;
                    if (!ISF && a.key32) {
                        const uint32_t key = valid ? (kc[j] | (val << a.pb)) : 0u;
                        const uint32_t best = scan_max32(key);
                        if (last) atomicMax(&gmax32[kc[j] >> (a.vb + a.pb)], best);
                    } else {
                        const unsigned long long key =
                            valid ? (((unsigned long long)kc[j] << 43) | ((unsigned long long)val << 11) |
                                     (uint32_t)(2047 - 64 * j - lane))
                                  : 0ull;
                        const unsigned long long best = scan_max(key);
                        if (last) atomicMax(&gmax[kc[j]], best);
                    }
                }
                __syncthreads();

                // ---- choose at most one bit per block; list the flips ------
                int any = 0, dif = 0, nflip = 0;
                for (int g0 = 0; g0 < a.Geff; g0 += 64) {
                    const int g = g0 + lane;
                    uint32_t cur = NONE;
                    if (g < a.Geff) {
                        uint32_t val, n;
                        if (!ISF && a.key32) {
                            const uint32_t key = gmax32[g];
                            gmax32[g] = 0;
                            val = (key >> a.pb) & ((1u << a.vb) - 1);
                            n = (uint32_t)g * a.p + (((1u << a.pb) - 1) - (key & ((1u << a.pb) - 1)));
                        } else {
                            const unsigned long long key = gmax[g];
                            gmax[g] = 0;
                            val = (uint32_t)(key >> 11);
                            n = 2047u - (uint32_t)(key & 2047u);
                        }
                        const bool flip = a.single || val > a.zero_val;
                        cur = flip ? n : NONE;
                        dif |= cur != prv[g];
                        any |= flip;
                        prv[g] = cur;
                    }
                    const unsigned long long fm = __ballot(cur != NONE);
                    if (cur != NONE) list[nflip + __popcll(fm & ((1ull << lane) - 1))] = cur;
                    nflip += __popcll(fm);
                }
                const bool anyf = __ballot(any) != 0, diff = __ballot(dif) != 0;
                if (a.cycle_exit) {
                    if (!anyf) {  // no flip: fixed point until K_max
                        k = a.exec_rounds ? k : a.max_iter;
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
                        k = a.exec_rounds ? k : a.max_iter;
                        break;
                    }
                }
                // ---- flip; toggle the checks of every flipped bit -----------
                // (one (bit, check) pair per lane and step)
                __syncthreads();
                for (int i = lane; i < nflip; i += 64) {
                    const uint32_t n = list[i];
                    atomicXor(&zw[n >> 5], 1u << (n & 31));
                }
                int delta = 0;
                const int ntask = nflip * W;
                for (int id = lane; id < ntask; id += 64) {
                    const uint32_t fi = fdiv((uint32_t)id, a.magW, a.maskW);
                    const uint32_t n = list[fi];
                    int m = (int)n - (int)shl[id - (int)fi * W];
                    m += m < 0 ? N : 0;
                    bool was_unsat;
                    if constexpr (ISF) {
                        const unsigned long long old = atomicXor(&ent[m], ((unsigned long long)SIGN << 32) | SIGN);
                        was_unsat = !((uint32_t)old & SIGN);
                    } else {
                        const uint32_t old = atomicXor(&ws[m], SIGN);
                        for (int i = m + N; i < Nx; i += N) atomicXor(&ws[i], SIGN);
                        was_unsat = !(old & SIGN);
                        if (icorr) {
                            const uint32_t inf = info[m];
                            const float d2 = (float)(2u * (inf >> 16));
                            if (inf >> 16) atomicAdd(&corr[inf & 0xFFFFu], was_unsat ? -d2 : d2);
                        }
                    }
                    delta += was_unsat ? -1 : 1;
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
    if (p->select == FWBF_TOPL || p->select == FWBF_STRIDED) return 0;  // contiguous blocks only
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
    a.exec_rounds = (p->flags & FWBF_FLAG_EXECUTED_ROUNDS) != 0;
    a.alpha = p->weights == FWBF_WBF ? 0.0f : p->alpha;
    a.aden = p->alpha_den;
    a.anum = p->weights == FWBF_WBF ? 0 : p->alpha_num;
    if (W <= 1) { a.magW = 0; a.maskW = 0xFFFFFFFFu; }
    else { a.magW = (uint32_t)(((1ULL << 32) + W - 1) / W); a.maskW = 0; }
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
        int gbits = 0, pbits = 0;
        while ((1 << gbits) < a.Geff) gbits++;
        while ((1 << pbits) < a.p) pbits++;
        a.vb = vb;
        a.pb = pbits;
        a.key32 = gbits + vb + pbits <= 32 && vb + pbits < 32;  // the block index is key >> (vb + pb)
    }
    // shifts of the single block, descending
    const auto &cell = c->cells[0];
    for (int t = 0; t < W; t++) a.sh[t] = (uint16_t)cell[t];
    const int esz = p->dtype == FWBF_I8 ? 2 : 4;  // staged value per bit
    const bool isf = p->dtype == FWBF_F32, icorr = !isf && a.imwbf;
    int off = 0;
    auto take = [&](int bytes, int align) { off = (off + align - 1) / align * align; int o = off; off += bytes; return o; };
    a.Nx = c->N + 64 * CW;
    take(isf ? 8 * c->N : 4 * a.Nx, 16);  // check entries at offset 0
    a.o_am = take(isf ? 2 * c->N : 0, 4);
    a.o_tab = take(isf ? 8 * W : 0, 4);
    a.o_info = take(icorr ? 4 * c->N : 0, 4);
    a.o_corr = take(icorr ? 4 * c->N : 0, 4);
    a.o_y = take(esz * a.Nx, 16);
    a.o_z = take(8 * a.nwin, 8);
    a.o_gmax = take(8 * a.Geff, 8);
    a.o_prv = take(4 * a.Geff, 4);
    a.o_list = take(4 * a.Geff, 4);
    a.o_shl = take(2 * W, 4);
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
