// FWBF decoding kernels for gfx950 (eq. (1) and Section III of the paper).
//
// One workgroup decodes one frame at a time and loops over frames
// (persistent grid).  Per-frame state lives in LDS:
//   keys  one 32-bit word per slot: the metric of a bit in order-preserving
//         unsigned form (optionally packed with its position in the block so
//         that an unsigned max picks the largest metric and, among equal
//         metrics, the lowest index);
//   chk   per check: minimum and second minimum of |y| over N(m) and the
//         position of the minimum (the IMWBF weight of bit n in check m is
//         the second minimum when n holds the minimum, else the minimum);
//   syn   syndrome bits, tog per-round toggle parities (integer inputs),
//         zw hard decisions.
// Slots: block g (p = ceil(N/G) bits) is padded to Lc = L*C slots held by L
// consecutive threads with C slots each (L a power of two; lane l of the
// block holds positions l, l + L, ..., so a wavefront's slot accesses fall
// on consecutive words); padding slots
// hold key 0 and never win (the "null" metric padding of the paper's
// footnote to Section V).
//
// Round k (Section III, Step 2 then Step 1):
//   select  each thread takes the max of its C slot keys, an xor-butterfly
//           over the L threads of the block gives the block maximum;
//   apply   winners with a positive metric toggle their hard decision;
//           float inputs also toggle their checks' syndrome bits at once
//           (atomic xors that return the old bit, so each toggle moves the
//           unsatisfied-check count by one), integer inputs toggle a
//           per-round parity of their checks instead;
//   claim   (integer inputs) one winner per net-toggled check flips its
//           syndrome bit and updates the unsatisfied-check count;
//   update  the metrics of the bits of every toggled check change: integer
//           inputs add +-2 a_den w exactly, float inputs recompute the bit's
//           metric from scratch in the fixed check order from the final
//           syndrome (so results equal a full recomputation bit for bit).
// The decoder is a deterministic function of the hard-decision vector; a
// round without flips, or with the same flips as the round before, proves
// the state sequence periodic with period 1 or 2, and the output at K_max
// follows without running the remaining rounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "frames.h"
#include "internal.h"

namespace fwbf {
namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;
// control words: the unsatisfied-check count, and the flags of rounds k even
// and odd (a round's slot is cleared at the start of the round before it)
constexpr int CTL_WEIGHT = 1, CTL_FLAGS0 = 2;
constexpr int F_ANY = 1, F_DIFF = 2;
// task-list entry: check index, with this bit set when the toggle left the
// check unsatisfied (check indices stay below 2^31)
constexpr uint32_t TL_UNSAT = 0x80000000u;

struct DecodeArgs {
    const void *y;
    int64_t F, stride;
    uint32_t *z;
    int32_t *iters;
    uint8_t *ok;
    const uint32_t *col, *row;
    const uint8_t *coldeg, *rowdeg;
    int N, M, Z, mb, nb, dvmax, dcmax;
    uint32_t magZ, maskZ, magP, maskP, magD, maskD;  // exact n/d = umulhi(n, mag) + (n & mask)
    int weights, select, lambda, max_iter;
    float alpha;
    int anum, aden;
    uint32_t flags;
    // slot layout
    int C, L, logL, GP, P, Geff, p, Lc, W;
    int idxb;
    uint32_t idxmask, bias, zero_val;
    // LDS offsets (bytes)
    int o_keys, o_chk, o_chkp, o_mag, o_z, o_syn, o_tog, o_win, o_prv, o_tl, o_gb, o_top, o_ctl,
        o_col, o_row, o_cdeg, o_rdeg, lds_bytes;
    // |y| staged in LDS only while the check minima are computed (it then
    // shares memory with the slots) and read from global memory afterwards
    int mag_alias;
    int multi;    // some block holds several shifts
    int strided;  // block g = {n : n mod G = g}: bit n = pos G + g
    uint32_t magG, maskG;
    // frames with skip[f] != 0 are left alone; the others add their rounds to
    // iters[f] (the plain fallback after the learned pass)
    const uint8_t *skip;
};

// bit of position pos in block g, and block / position of bit n
__device__ __forceinline__ uint32_t bit_of(const DecodeArgs &a, uint32_t g, uint32_t pos)
{
    return a.strided ? pos * (uint32_t)a.Geff + g : g * (uint32_t)a.p + pos;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t mag, uint32_t mask)
{
    return __umulhi(n, mag) + (n & mask);
}

template <int DT> struct Tr;
template <> struct Tr<FWBF_I8> {
    using Y = int8_t;
    using Mag = uint8_t;
    using Chk = uint32_t;  // min1 | min2 << 8 | pos << 16
    static constexpr bool isf = false;
};
template <> struct Tr<FWBF_I16> {
    using Y = int16_t;
    using Mag = uint16_t;
    using Chk = uint32_t;  // min1 | min2 << 16; position in chkp
    static constexpr bool isf = false;
};
template <> struct Tr<FWBF_F32> {
    using Y = float;
    using Mag = float;
    using Chk = uint64_t;  // bits(min1) | bits(min2) << 32; position in chkp
    static constexpr bool isf = true;
};

template <int DT> __device__ __forceinline__ typename Tr<DT>::Chk pack_chk(uint32_t m1, uint32_t m2, uint32_t pos)
{
    if constexpr (DT == FWBF_I8) return m1 | (m2 << 8) | (pos << 16);
    else if constexpr (DT == FWBF_I16) return m1 | (m2 << 16);
    else return (uint64_t)m1 | ((uint64_t)m2 << 32);
}

struct Lds {
    uint32_t *keys;
    void *chk;
    uint8_t *chkp;
    void *mag;
    uint32_t *zw, *syn, *tog, *win, *prv, *tl;
    unsigned long long *gb;
    uint32_t *topn;
    unsigned long long *topk;
    int *ctl;
    uint32_t *col, *row;
    uint8_t *cdeg, *rdeg;
    const void *yrow;  // received values of the current frame (global memory)
};

// weight w_{n,m} of the q-th member of check m (int inputs)
template <int DT>
__device__ __forceinline__ int32_t weight_i(const Lds &s, uint32_t m, uint32_t q, bool imwbf)
{
    const uint32_t c = ((const uint32_t *)s.chk)[m];
    if constexpr (DT == FWBF_I8) {
        const uint32_t m1 = c & 0xFF, m2 = (c >> 8) & 0xFF, pos = (c >> 16) & 0xFF;
        return (int32_t)((imwbf && pos == q) ? m2 : m1);
    } else {
        const uint32_t m1 = c & 0xFFFF, m2 = c >> 16;
        return (int32_t)((imwbf && s.chkp[m] == q) ? m2 : m1);
    }
}
__device__ __forceinline__ float weight_f(uint64_t c, uint32_t pos, uint32_t q, bool imwbf)
{
    uint32_t bits = (imwbf && pos == q) ? (uint32_t)(c >> 32) : (uint32_t)c;
    return __uint_as_float(bits);
}

// order-preserving map of a float to uint32 (-0 canonicalised to +0)
__device__ __forceinline__ uint32_t orderable(float e)
{
    uint32_t u = __float_as_uint(e == 0.0f ? 0.0f : e);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}



// Metric of bit n (eq. (1)) of float inputs from the current syndrome, as an
// order-preserving 32-bit value: fmaf(-alpha, |y_n|, S) with S summed over
// M(n) in ascending check order from the first term.  (Integer inputs keep
// their metrics exact under additions and never recompute them.)
template <int DT>
__device__ __forceinline__ uint32_t metric_val(const DecodeArgs &a, const Lds &s, uint32_t n, bool imwbf)
{
    using T = Tr<DT>;
    static_assert(T::isf, "float inputs only");
    const uint32_t j = fdiv(n, a.magZ, a.maskZ);
    const int c = (int)(n - j * a.Z);
    const int deg = s.cdeg[j];
    const uint32_t *ce = s.col + j * a.dvmax;
    const typename T::Chk *chk = (const typename T::Chk *)s.chk;
    if constexpr (T::isf) {
        // y_n is read first (from global memory where its LDS copy shares the
        // slots' memory) and its magnitude taken only at the end, so that the
        // read's latency overlaps the check terms' LDS reads
        // (a global-memory pointer: a generic load would also count as an LDS
        // access, and the LDS waits below would wait for it)
        typedef const __attribute__((address_space(1))) float gfloat;
        float mg = a.mag_alias ? ((gfloat *)s.yrow)[n] : ((const float *)s.mag)[n];
        float S = 0.0f;
        auto term = [&](uint32_t e) {
            int r = c - (int)(e & 0xFFFF);
            r += (r < 0) ? a.Z : 0;
            const uint32_t m = (e >> 24) * a.Z + r;
            const float w = weight_f(chk[m], s.chkp[m], (e >> 16) & 0xFF, imwbf);
            return ((s.syn[m >> 5] >> (m & 31)) & 1) ? w : -w;
        };
        if (!a.multi) {
            // four terms' reads issued together, then added in list order
            for (int t0 = 0; t0 < deg; t0 += 4) {
                uint32_t e[4], m[4], sw[4], pp[4];
                uint64_t cw[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    e[u] = ce[min(t0 + u, deg - 1)];
                    int r = c - (int)(e[u] & 0xFFFF);
                    r += (r < 0) ? a.Z : 0;
                    m[u] = (e[u] >> 24) * a.Z + r;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    cw[u] = chk[m[u]];
                    pp[u] = s.chkp[m[u]];
                    sw[u] = s.syn[m[u] >> 5];
                }
                // (no branch here: a branch would let the compiler move the
                // reads above into it, one after another)
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const float w = weight_f(cw[u], pp[u], (e[u] >> 16) & 0xFF, imwbf);
                    const float tm = ((sw[u] >> (m[u] & 31)) & 1) ? w : -w;
                    const float nS = (t0 + u == 0) ? tm : S + tm;
                    S = t0 + u < deg ? nS : S;
                }
            }
        } else {
            // the shifts of one block row are listed in descending order:
            // start at the first shift <= c (row c - s), then wrap
            int t0 = 0, cnt = 0;
            while (t0 < deg) {
                const uint32_t i = ce[t0] >> 24;
                int t1 = t0 + 1;
                while (t1 < deg && (ce[t1] >> 24) == i) t1++;
                int u = t0;
                while (u < t1 && (int)(ce[u] & 0xFFFF) > c) u++;
                for (int v = 0; v < t1 - t0; v++, cnt++) {
                    int x = u + v;
                    x -= (x >= t1) ? t1 - t0 : 0;
                    S = (cnt == 0) ? term(ce[x]) : S + term(ce[x]);
                }
                t0 = t1;
            }
        }
        asm volatile("" : "+v"(mg));
        return orderable(__builtin_fmaf(-a.alpha, fabsf(mg), S));
    }
}

template <bool KEY32>
__device__ __forceinline__ unsigned long long widen(uint32_t key, uint32_t pos)
{
    return ((unsigned long long)key << 32) | (0xFFFFFFFFu - pos);
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int d)
{
    uint32_t lo = __shfl_xor((uint32_t)v, d, 64), hi = __shfl_xor((uint32_t)(v >> 32), d, 64);
    return ((unsigned long long)hi << 32) | lo;
}

// maximum over the C slots of one thread, as a 64-bit key
// (value << 32 | ~position) where position is the slot offset in the block.
// Lane l of a block owns positions l, l + L, l + 2L, ...: at every step the
// lanes of a wavefront touch consecutive words (no LDS bank conflicts), and
// the first strict maximum along k is the lowest position.  The slots are
// read KB at a time, all reads of a chunk issued before any is compared.
template <bool KEY32>
__device__ __forceinline__ unsigned long long thread_best(const DecodeArgs &a, const uint32_t *keys, int s0, uint32_t l)
{
    constexpr int KB = 4;
    if constexpr (KEY32) {
        uint32_t best = 0;
        for (int k0 = 0; k0 < a.C; k0 += KB) {
            uint32_t v[KB];
#pragma unroll
            for (int u = 0; u < KB; u++) v[u] = k0 + u < a.C ? keys[s0 + (k0 + u) * a.L] : 0u;
#pragma unroll
            for (int u = 0; u < KB; u++) best = max(best, v[u]);
        }
        // unpack into the common 64-bit form
        return ((unsigned long long)(best >> a.idxb) << 32) | (0xFFFFFFFFu - (a.idxmask - (best & a.idxmask)));
    } else {
        uint32_t best = 0, bk = 0;
        for (int k0 = 0; k0 < a.C; k0 += KB) {
            uint32_t v[KB];
#pragma unroll
            for (int u = 0; u < KB; u++) v[u] = k0 + u < a.C ? keys[s0 + (k0 + u) * a.L] : 0u;
#pragma unroll
            for (int u = 0; u < KB; u++) {
                const bool gt = v[u] > best;
                best = gt ? v[u] : best;
                bk = gt ? (uint32_t)(k0 + u) : bk;
            }
        }
        return ((unsigned long long)best << 32) | (0xFFFFFFFFu - (l + bk * (uint32_t)a.L));
    }
}

// the largest of the C packed keys of one thread (reads KB at a time)
__device__ __forceinline__ uint32_t thread_best32(const DecodeArgs &a, const uint32_t *keys, int s0)
{
    constexpr int KB = 4;
    uint32_t best = 0;
    for (int k0 = 0; k0 < a.C; k0 += KB) {
        uint32_t v[KB];
#pragma unroll
        for (int u = 0; u < KB; u++) v[u] = k0 + u < a.C ? keys[s0 + (k0 + u) * a.L] : 0u;
#pragma unroll
        for (int u = 0; u < KB; u++) best = max(best, v[u]);
    }
    return best;
}

// maximum over aligned groups of w lanes of a 32-bit value (w a power of two
// <= 64, every lane active): DPP row moves fused with the max, then two
// cross-row exchanges; every lane of a group ends with the maximum
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t group_max32(uint32_t v, int w)
{
    if (w > 1) v = max(v, dpp32<0xB1>(v));   // quad_perm [1,0,3,2]
    if (w > 2) v = max(v, dpp32<0x4E>(v));   // quad_perm [2,3,0,1]
    if (w > 4) v = max(v, dpp32<0x141>(v));  // row_half_mirror
    if (w > 8) v = max(v, dpp32<0x140>(v));  // row_mirror
    if (w > 16) v = max(v, (uint32_t)__shfl_xor((int)v, 16, 64));
    if (w > 32) v = max(v, (uint32_t)__shfl_xor((int)v, 32, 64));
    return v;
}

// row-local data movement (DPP) of a 64-bit value: xor 1, xor 2, mirror
// within 8, mirror within 16
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((unsigned long long)hi << 32) | lo;
}

// maximum over aligned groups of w lanes (w a power of two <= 64, every lane
// of the wavefront active); every lane of a group ends with the maximum
__device__ __forceinline__ unsigned long long group_max64(unsigned long long v, int w)
{
    unsigned long long o;
    if (w > 1) { o = dpp64<0xB1>(v); v = o > v ? o : v; }   // quad_perm [1,0,3,2]
    if (w > 2) { o = dpp64<0x4E>(v); v = o > v ? o : v; }   // quad_perm [2,3,0,1]
    if (w > 4) { o = dpp64<0x141>(v); v = o > v ? o : v; }  // row_half_mirror
    if (w > 8) { o = dpp64<0x140>(v); v = o > v ? o : v; }  // row_mirror
    if (w > 16) { o = shfl_xor_u64(v, 16); v = o > v ? o : v; }
    if (w > 32) { o = shfl_xor_u64(v, 32); v = o > v ? o : v; }
    return v;
}

// Barrier of one frame's threads: the workgroup, or (WAVE) the single
// wavefront that decodes the frame alone inside a larger workgroup (LDS
// operations of one wavefront complete in issue order; the wave barrier
// keeps the compiler from moving memory operations across it).
template <bool WAVE>
__device__ __forceinline__ void frame_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Initialisation of integer inputs in 64-wide chunks: a wavefront takes 64
// consecutive checks of one block row (or bits of one block column), so the
// row's (column's) list entries are uniform across it, read once and kept in
// scalar registers, and the lanes' members are consecutive words up to one
// wrap.  The staged row holds the signed values (their magnitudes are taken
// where used).
// ---------------------------------------------------------------------------

// median of three (the second smallest key once a <= c)
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// ORs the 64 bits of b (uniform) into a bit array at bit offset base: lanes
// 0..2 take one word each (LDS atomics), words without set bits untouched
__device__ __forceinline__ void or_bits(uint32_t *w, uint32_t base, unsigned long long b, uint32_t lane)
{
    const uint32_t k = base >> 5, o = base & 31;
    const unsigned long long lo = b << o;
    const uint32_t hi = o ? (uint32_t)(b >> (64 - o)) : 0u;
    const uint32_t v = lane == 0 ? (uint32_t)lo : lane == 1 ? (uint32_t)(lo >> 32) : hi;
    if (lane < 3 && v) atomicOr(&w[k + lane], v);
}

// Keys |y| << 8 | t of the row-list entries t = q0 .. q0 + QL - 1 (entry:
// column block << 16 | shift) for the checks r of one block row (lanes; rm
// = r - Z), all reads issued before any is used, folded into the two
// smallest keys and the parity of the negative members (sign bit of sx).
template <int QL, typename Y>
__device__ __forceinline__ void row_keys(const Y *ys, const uint32_t *re, uint32_t Z, uint32_t r, uint32_t rm, int q0,
                                         uint32_t &k1, uint32_t &k2, int &sx)
{
    uint32_t e[QL];
    int v[QL];
#pragma unroll
    for (int u = 0; u < QL; u++) e[u] = __builtin_amdgcn_readfirstlane(re[q0 + u]);
#pragma unroll
    for (int u = 0; u < QL; u++) {
        const uint32_t sft = e[u] & 0xFFFFu;
        v[u] = (int)ys[(e[u] >> 16) * Z + min(r + sft, rm + sft)];
    }
#pragma unroll
    for (int u = 0; u < QL; u++) {
        sx ^= v[u];
        const uint32_t key = ((uint32_t)(v[u] < 0 ? -v[u] : v[u]) << 8) | (uint32_t)(q0 + u);
        k2 = med3u(k1, key, k2);
        k1 = min(k1, key);
    }
}

// first minimum of check m
template <int DT>
__device__ __forceinline__ int chk_min1(const Lds &s, uint32_t m)
{
    if constexpr (DT == FWBF_I8) return ((const uint8_t *)s.chk)[4 * m];
    else return ((const uint16_t *)s.chk)[2 * m];
}

// Sum over the column-list entries t = t0 .. t0 + QL - 1 (entry: row block
// << 24 | position << 16 | shift) of +-min1 of the bits c (lanes; cz = c + Z)
// of one block column, + for an unsatisfied check; reads issued together.
template <int DT, int QL>
__device__ __forceinline__ int col_terms(const Lds &s, const uint32_t *ce, uint32_t Z, uint32_t c, uint32_t cz, int t0)
{
    uint32_t e[QL], mm[QL], sw[QL];
    int w[QL];
#pragma unroll
    for (int u = 0; u < QL; u++) e[u] = __builtin_amdgcn_readfirstlane(ce[t0 + u]);
#pragma unroll
    for (int u = 0; u < QL; u++) {
        const uint32_t sft = e[u] & 0xFFFFu;
        mm[u] = (e[u] >> 24) * Z + min(c - sft, cz - sft);
    }
#pragma unroll
    for (int u = 0; u < QL; u++) {
        w[u] = chk_min1<DT>(s, mm[u]);
        sw[u] = s.syn[__builtin_amdgcn_ubfe(mm[u], 5, 27)];
    }
    int S = 0;
#pragma unroll
    for (int u = 0; u < QL; u++) S += __builtin_amdgcn_ubfe(sw[u], mm[u], 1) ? w[u] : -w[u];  // offset taken mod 32
    return S;
}

// slot of bit n
__device__ __forceinline__ uint32_t slot_of(const DecodeArgs &a, uint32_t n, uint32_t *pos_out)
{
    uint32_t g, pos;
    if (a.strided) { pos = fdiv(n, a.magG, a.maskG); g = n - pos * a.Geff; }
    else { g = fdiv(n, a.magP, a.maskP); pos = n - g * a.p; }
    *pos_out = pos;
    return g * a.Lc + pos;
}

// Check minima (min1, min2 with multiplicity, position of min1) and the
// syndrome s_0 of integer inputs; the syndrome words start zeroed.
template <int DT, int T>
__device__ __forceinline__ void int_check_minima(const DecodeArgs &a, const Lds &s, int tid, uint32_t lane)
{
    using Tt = Tr<DT>;
    const typename Tt::Y *ys = (const typename Tt::Y *)s.mag;
    const uint32_t Z = a.Z;
    const int NZc = (int)((Z + 63) >> 6);
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int ch = wv; ch < a.mb * NZc; ch += T / 64) {
        const int i = ch / NZc;
        const uint32_t r0 = (uint32_t)(ch - i * NZc) << 6, r = r0 + lane;
        const bool valid = r < Z;
        const uint32_t rr = valid ? r : 0u, rm = rr - Z;  // rm + s wraps below Z
        const int deg = __builtin_amdgcn_readfirstlane(s.rdeg[i]);
        const uint32_t *re = s.row + i * a.dcmax;
        // the two smallest keys: min1 and min2 with multiplicity, the first
        // one's entry the lowest position holding min1
        uint32_t k1 = 0xFFFFFFFFu, k2 = 0xFFFFFFFFu;
        int sx = 0, q0 = 0;
        for (; q0 + 4 <= deg; q0 += 4) row_keys<4>(ys, re, Z, rr, rm, q0, k1, k2, sx);
        if (deg - q0 == 3) row_keys<3>(ys, re, Z, rr, rm, q0, k1, k2, sx);
        else if (deg - q0 == 2) row_keys<2>(ys, re, Z, rr, rm, q0, k1, k2, sx);
        else if (deg - q0 == 1) row_keys<1>(ys, re, Z, rr, rm, q0, k1, k2, sx);
        if (valid) {
            const uint32_t m = (uint32_t)i * Z + rr;
            const uint32_t m1 = deg > 0 ? (k1 >> 8) : 0u, m2 = deg > 1 ? (k2 >> 8) : 0u;  // empty minima: 0
            const uint32_t pos = deg > 0 ? (k1 & 0xFFu) : 0u;
            ((typename Tt::Chk *)s.chk)[m] = pack_chk<DT>(m1, m2, pos);
            if constexpr (DT == FWBF_I16) s.chkp[m] = (uint8_t)pos;
        }
        const unsigned long long b = __ballot(valid && sx < 0);
        if (b) {
            or_bits(s.syn, (uint32_t)i * Z + r0, b, lane);
            if (lane == 0) atomicAdd(&s.ctl[CTL_WEIGHT], __popcll(b));
        }
    }
}

// Float magnitudes of the row-list entries q0 .. q0 + QL - 1 for the checks
// r of one block row (lanes), reads issued together: min1 and min2 (with
// multiplicity) as the bit patterns of non-negative floats, whose unsigned
// order is the float order (a NaN's pattern lies above +inf, so a NaN never
// becomes a minimum, as under float comparisons); pos takes the first entry
// holding min1; neg collects, per member, [y < 0] as a lane mask (xor).
template <int QL>
__device__ __forceinline__ void row_fmins(const float *ys, const uint32_t *re, uint32_t Z, uint32_t r, uint32_t rm, int q0,
                                          uint32_t &m1, uint32_t &m2, uint32_t &pos, unsigned long long &neg)
{
    uint32_t e[QL];
    float v[QL];
#pragma unroll
    for (int u = 0; u < QL; u++) e[u] = __builtin_amdgcn_readfirstlane(re[q0 + u]);
#pragma unroll
    for (int u = 0; u < QL; u++) {
        const uint32_t sft = e[u] & 0xFFFFu;
        v[u] = ys[(e[u] >> 16) * Z + min(r + sft, rm + sft)];
    }
#pragma unroll
    for (int u = 0; u < QL; u++) {
        neg ^= __ballot(v[u] < 0.0f);
        const uint32_t av = __float_as_uint(v[u]) & 0x7FFFFFFFu;
        pos = av < m1 ? (uint32_t)(q0 + u) : pos;
        m2 = med3u(m1, av, m2);
        m1 = min(m1, av);
    }
}

// Check minima and the syndrome s_0 of float inputs (the staged row holds
// the signed values; the syndrome words start zeroed).
template <int T>
__device__ __forceinline__ void f32_check_minima(const DecodeArgs &a, const Lds &s, int tid, uint32_t lane)
{
    const float *ys = (const float *)s.mag;
    const uint32_t Z = a.Z;
    const int NZc = (int)((Z + 63) >> 6);
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr uint32_t INF = 0x7F800000u;
    for (int ch = wv; ch < a.mb * NZc; ch += T / 64) {
        const int i = ch / NZc;
        const uint32_t r0 = (uint32_t)(ch - i * NZc) << 6, r = r0 + lane;
        const bool valid = r < Z;
        const uint32_t rr = valid ? r : 0u, rm = rr - Z;
        const int deg = __builtin_amdgcn_readfirstlane(s.rdeg[i]);
        const uint32_t *re = s.row + i * a.dcmax;
        uint32_t m1 = INF, m2 = INF, pos = 0;
        unsigned long long neg = 0;
        int q0 = 0;
        for (; q0 + 4 <= deg; q0 += 4) row_fmins<4>(ys, re, Z, rr, rm, q0, m1, m2, pos, neg);
        if (deg - q0 == 3) row_fmins<3>(ys, re, Z, rr, rm, q0, m1, m2, pos, neg);
        else if (deg - q0 == 2) row_fmins<2>(ys, re, Z, rr, rm, q0, m1, m2, pos, neg);
        else if (deg - q0 == 1) row_fmins<1>(ys, re, Z, rr, rm, q0, m1, m2, pos, neg);
        if (valid) {
            const uint32_t m = (uint32_t)i * Z + rr;
            ((uint64_t *)s.chk)[m] = (uint64_t)m1 | ((uint64_t)(deg < 2 ? 0u : m2) << 32);  // empty minimum: 0
            s.chkp[m] = (uint8_t)pos;
        }
        const unsigned long long b = neg & __ballot(valid);
        if (b) {
            or_bits(s.syn, (uint32_t)i * Z + r0, b, lane);
            if (lane == 0) atomicAdd(&s.ctl[CTL_WEIGHT], __popcll(b));
        }
    }
}

// Initial keys of integer inputs (eq. (1)): every bit gathers +-min1 of its
// checks; padding slots get key 0; with IMWBF weights each check then moves
// the metric of the member holding its min1 by +-a_den (min2 - min1) (that
// member's weight is min2).  The staged row is dead here (its memory may be
// the slots'), so |y| is read from the frame in global memory.
template <int DT, bool KEY32, int T, bool WAVE>
__device__ __forceinline__ void int_initial_keys(const DecodeArgs &a, const Lds &s, int tid, uint32_t lane,
                                                 const typename Tr<DT>::Y *yrow)
{
    const uint32_t Z = a.Z;
    const int N = a.N;
    const int NZc = (int)((Z + 63) >> 6);
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int pi = 0; pi < a.P; pi++) {
        const int g = pi * a.GP + (tid >> a.logL);
        const int l = tid & (a.L - 1);
        int lim = 0;  // positions below lim hold a bit
        if (g < a.Geff)
            lim = a.strided ? min(a.p, (int)fdiv((uint32_t)(N - g + a.Geff - 1), a.magG, a.maskG)) : min(a.p, N - g * a.p);
        for (int kk = lim > l ? (lim - l + a.L - 1) >> a.logL : 0; kk < a.C; kk++) s.keys[g * a.Lc + l + kk * a.L] = 0;
    }
    for (int ch = wv; ch < a.nb * NZc; ch += T / 64) {
        const int j = ch / NZc;
        const uint32_t c0 = __builtin_amdgcn_readfirstlane((uint32_t)(ch - j * NZc) << 6), c = c0 + lane;
        const bool valid = c < Z;
        const uint32_t cc = valid ? c : 0u, cz = cc + Z;
        const uint32_t n = (uint32_t)j * Z + cc;
        const int x = (int)yrow[n];
        const int deg = __builtin_amdgcn_readfirstlane(s.cdeg[j]);
        const uint32_t *ce = s.col + j * a.dvmax;
        // four entries at a time (entries past the column's degree add nothing)
        int S = 0, t0 = 0;
        for (; t0 + 4 <= deg; t0 += 4) S += col_terms<DT, 4>(s, ce, Z, cc, cz, t0);
        if (t0 + 2 <= deg) { S += col_terms<DT, 2>(s, ce, Z, cc, cz, t0); t0 += 2; }
        if (t0 < deg) S += col_terms<DT, 1>(s, ce, Z, cc, cz, t0);
        const int av = x < 0 ? -x : x;
        const uint32_t v = (uint32_t)(a.aden * S - a.anum * av + (int32_t)a.bias);
        uint32_t pos;
        const uint32_t slot = slot_of(a, n, &pos);
        if (valid) s.keys[slot] = KEY32 ? ((v << a.idxb) | (a.idxmask - pos)) : v;
    }
    if (a.weights != FWBF_IMWBF) return;
    frame_sync<WAVE>();
    for (int ch = wv; ch < a.mb * NZc; ch += T / 64) {
        const int i = ch / NZc;
        const uint32_t r = ((uint32_t)(ch - i * NZc) << 6) + lane;
        if (r >= Z) continue;
        const uint32_t m = (uint32_t)i * Z + r, cw = ((const uint32_t *)s.chk)[m];
        uint32_t m1, m2, q;
        if constexpr (DT == FWBF_I8) { m1 = cw & 0xFF; m2 = (cw >> 8) & 0xFF; q = (cw >> 16) & 0xFF; }
        else { m1 = cw & 0xFFFF; m2 = cw >> 16; q = s.chkp[m]; }
        const int d = (int)m2 - (int)m1;
        if (d == 0 || (int)q >= s.rdeg[i]) continue;  // (an empty row has no member to move)
        const uint32_t e = s.row[i * a.dcmax + q], sft = e & 0xFFFFu;
        const uint32_t nn = (e >> 16) * Z + min(r + sft, r + sft - Z);
        const uint32_t sb = (s.syn[m >> 5] >> (m & 31)) & 1u;
        const int dd = a.aden * (sb ? d : -d);
        uint32_t pos;
        const uint32_t slot = slot_of(a, nn, &pos);
        atomicAdd(&s.keys[slot], KEY32 ? ((uint32_t)dd << a.idxb) : (uint32_t)dd);
    }
}

// Flips bit n of block u (NONE: no flip) and toggles its checks' syndrome
// bits with atomic xors that return the bit replaced: the weight moves by one
// per toggle and each toggle is listed with the check's new bit (a check
// toggled by two winners is listed twice and ends unchanged; integer inputs
// then add +2 a_den w and -2 a_den w to its members).  The round's flags
// record any flip and any block whose choice differs from the previous one.
__device__ __forceinline__ void flip_block(const DecodeArgs &a, const Lds &s, uint32_t u, uint32_t n, int *flags)
{
    const uint32_t pv = s.prv[u];
    s.prv[u] = n;
    uint32_t *tl = s.tl + u * a.dvmax;
    for (int t = 0; t < a.dvmax; t++) tl[t] = NONE;
    int fl = (n != pv) ? F_DIFF : 0;
    if (n != NONE) {
        fl |= F_ANY;
        atomicXor(&s.zw[n >> 5], 1u << (n & 31));
        const uint32_t j = fdiv(n, a.magZ, a.maskZ);
        const int c = (int)(n - j * a.Z);
        const int deg = s.cdeg[j];
        int dw = 0;
        // four checks at a time, their toggles issued together
        for (int t0 = 0; t0 < deg; t0 += 4) {
            uint32_t mq[4], so[4];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const uint32_t e = s.col[j * a.dvmax + min(t0 + v, deg - 1)];
                int r = c - (int)(e & 0xFFFF);
                r += (r < 0) ? a.Z : 0;
                mq[v] = (e >> 24) * a.Z + r;
            }
#pragma unroll
            for (int v = 0; v < 4; v++)
                so[v] = t0 + v < deg ? atomicXor(&s.syn[mq[v] >> 5], 1u << (mq[v] & 31)) : 0u;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                if (t0 + v < deg) {
                    const uint32_t bit = 1u << (mq[v] & 31);
                    dw += (so[v] & bit) ? -1 : 1;
                    tl[t0 + v] = (so[v] & bit) ? mq[v] : (mq[v] | TL_UNSAT);
                }
            }
        }
        if (dw) atomicAdd(&s.ctl[CTL_WEIGHT], dw);
    }
    if (fl) atomicOr(flags, fl);
}

template <int DT, bool KEY32, int T, bool WAVE = false>
__device__ void decode_frame(const DecodeArgs &a, Lds s, int64_t f)
{
    static_assert(!WAVE || T == 64, "a frame decoded by one wavefront has 64 threads");
    using Tt = Tr<DT>;
    using Y = typename Tt::Y;
    using Mag = typename Tt::Mag;
    const int tid = WAVE ? (int)(threadIdx.x & 63) : (int)threadIdx.x, lane = tid & 63;
    const bool imwbf = a.weights == FWBF_IMWBF;
    const int N = a.N, M = a.M;
    Mag *mag = (Mag *)s.mag;
    if (a.skip && a.skip[f]) return;  // the same answer for every thread of the frame

    // ---- Initialization: |y|, z_0 = [y < 0] (Section III) ----------------
    const Y *yrow = (const Y *)a.y + f * a.stride;
    s.yrow = yrow;
    const int Nr = (N + 63) & ~63, Mr = (M + 63) & ~63;
    // eight loads in flight per thread before any is used (n < Nr is
    // uniform across a wavefront: Nr is a multiple of 64)
    constexpr int UNR = 8;
    for (int n0 = tid; n0 < Nr; n0 += UNR * T) {
        Y v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const int n = n0 + u * T;
            v[u] = n < N ? yrow[n] : (Y)0;
        }
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const int n = n0 + u * T;
            if (n >= Nr) break;
            const bool neg = n < N && v[u] < (Y)0;
            if (n < N) {
                mag[n] = (Mag)v[u];  // the signed value (magnitudes taken where used)
            }
            const unsigned long long b = __ballot(neg);
            if (lane == 0) {
                s.zw[(n >> 5)] = (uint32_t)b;
                s.zw[(n >> 5) + 1] = (uint32_t)(b >> 32);
            }
        }
    }
    for (int w = tid; w < (Mr >> 5); w += T) s.tog[w] = 0;
    for (int w = tid; w < (Mr >> 5); w += T) s.syn[w] = 0;
    if (tid == 0) { s.ctl[CTL_FLAGS0] = 0; s.ctl[CTL_FLAGS0 + 1] = 0; s.ctl[CTL_WEIGHT] = 0; }
    frame_sync<WAVE>();

    // ---- check minima (weights) and the syndrome s_0 (Step 1 at k=0) -----
    if constexpr (!Tt::isf) int_check_minima<DT, T>(a, s, tid, (uint32_t)lane);
    else f32_check_minima<T>(a, s, tid, (uint32_t)lane);
    frame_sync<WAVE>();

    int k = 0, okf = 0;
    const int weight0 = s.ctl[CTL_WEIGHT];
    if (weight0 == 0 || a.max_iter == 0) {
        okf = weight0 == 0;
    } else {
        // ---- initial metrics (eq. (1)) into the slots ---------------------
        if constexpr (!Tt::isf) int_initial_keys<DT, KEY32, T, WAVE>(a, s, tid, (uint32_t)lane, yrow);
        else for (int pi = 0; pi < a.P; pi++) {
            const int g = pi * a.GP + (tid >> a.logL);
            const int l = tid & (a.L - 1);
            for (int kk = 0; kk < a.C; kk++) {
                const int pos = l + kk * a.L;
                const int n = (int)bit_of(a, g, pos);
                uint32_t key = 0;
                if (g < a.Geff && pos < a.p && n < N) {
                    const uint32_t v = metric_val<DT>(a, s, n, imwbf);
                    key = KEY32 ? ((v << a.idxb) | (a.idxmask - pos)) : v;
                }
                s.keys[g * a.Lc + pos] = key;
            }
        }
        for (int u = tid; u < a.W; u += T) s.prv[u] = NONE;
        if (tid < 2) s.gb[tid] = 0;
        for (int u = tid; u < a.Geff && a.L > 64; u += T) s.gb[u] = 0;
        frame_sync<WAVE>();

        // the flips of a block follow its choice at once (no barrier between)
        // where one wavefront holds the block and the flip pass is the one
        // that lists every toggle
        const bool merged = (Tt::isf || T > 64) && a.select != FWBF_TOPL && a.L <= 64;
        for (;;) {
            // this round's flags; the next round's slot was last read in the
            // round before this one, so it is cleared here
            const int fi = CTL_FLAGS0 + (k & 1);
            if (tid == 0) s.ctl[CTL_FLAGS0 + ((k + 1) & 1)] = 0;
            // ---- Step 2: choose at most one bit per block ------------------
            if (a.select != FWBF_TOPL) {
                for (int pi = 0; pi < a.P; pi++) {
                    const int g = pi * a.GP + (tid >> a.logL);
                    const int l = tid & (a.L - 1);
                    unsigned long long best;
                    if constexpr (KEY32) {
                        // packed keys: the maximum runs on 32 bits, then unpacks
                        const uint32_t b32 = group_max32(thread_best32(a, s.keys, g * a.Lc + l), a.L < 64 ? a.L : 64);
                        best = ((unsigned long long)(b32 >> a.idxb) << 32) | (0xFFFFFFFFu - (a.idxmask - (b32 & a.idxmask)));
                    } else {
                        best = thread_best<KEY32>(a, s.keys, g * a.Lc + l, l);
                        best = group_max64(best, a.L < 64 ? a.L : 64);
                    }
                    if (a.L <= 64) {
                        if ((tid & (a.L - 1)) == 0 && g < a.Geff) {
                            const uint32_t val = (uint32_t)(best >> 32);
                            const uint32_t pos = 0xFFFFFFFFu - (uint32_t)best;
                            const bool flip = (a.select == FWBF_SINGLE) || val > a.zero_val;
                            const uint32_t n = flip ? bit_of(a, g, pos) : NONE;
                            s.win[g] = n;
                            if (merged) flip_block(a, s, (uint32_t)g, n, &s.ctl[fi]);
                        }
                    } else if (lane == 0 && g < a.Geff) {
                        atomicMax(&s.gb[g], best);
                    }
                }
                if (a.L > 64) {
                    frame_sync<WAVE>();
                    for (int g = tid; g < a.Geff; g += T) {
                        const unsigned long long best = s.gb[g];
                        s.gb[g] = 0;
                        const uint32_t val = (uint32_t)(best >> 32);
                        const uint32_t pos = 0xFFFFFFFFu - (uint32_t)best;
                        const bool flip = (a.select == FWBF_SINGLE) || val > a.zero_val;
                        s.win[g] = flip ? bit_of(a, g, pos) : NONE;
                    }
                }
            } else {
                // top-lambda: lambda sequential maxima over the whole frame
                // (single block layout), each excluded before the next
                int cnt = 0;
                for (int t = 0; t < a.lambda; t++) {
                    unsigned long long best = thread_best<KEY32>(a, s.keys, (tid >> a.logL) * a.Lc + (tid & (a.L - 1)),
                                                                  tid & (a.L - 1));
                    best = group_max64(best, 64);
                    if (lane == 0) atomicMax(&s.gb[t & 1], best);
                    frame_sync<WAVE>();
                    best = s.gb[t & 1];
                    const uint32_t val = (uint32_t)(best >> 32);
                    const uint32_t pos = 0xFFFFFFFFu - (uint32_t)best;
                    if (val <= a.zero_val) break;  // uniform: every thread read the same value
                    if (tid == 0) {
                        s.gb[(t + 1) & 1] = 0;
                        s.topn[t] = pos;
                        s.topk[t] = s.keys[pos];
                        s.keys[pos] = 0;
                    }
                    cnt = t + 1;
                    frame_sync<WAVE>();
                }
                frame_sync<WAVE>();
                if (tid == 0) {
                    s.gb[0] = 0;
                    s.gb[1] = 0;
                    // restore, then list the chosen bits in ascending order
                    for (int t = 0; t < cnt; t++) s.keys[s.topn[t]] = (uint32_t)s.topk[t];
                    for (int t = 1; t < cnt; t++) {
                        const uint32_t v = s.topn[t];
                        int u = t - 1;
                        while (u >= 0 && s.topn[u] > v) { s.topn[u + 1] = s.topn[u]; u--; }
                        s.topn[u + 1] = v;
                    }
                    for (int t = 0; t < a.W; t++) s.win[t] = t < cnt ? s.topn[t] : NONE;
                }
            }
            frame_sync<WAVE>();

            if constexpr (Tt::isf || T > 64) {
                // ---- flip the chosen bits and toggle their checks' syndrome -----
                // (flip_block; done above, with the choice, when merged)
                if (!merged) {
                    for (int u = tid; u < a.W; u += T) flip_block(a, s, (uint32_t)u, s.win[u], &s.ctl[fi]);
                    frame_sync<WAVE>();
                }
                const int flags = s.ctl[fi];
                if (!(a.flags & FWBF_FLAG_NO_CYCLE_EXIT)) {
                    if (!(flags & F_ANY)) {  // no flip: fixed point until K_max
                        k = (a.flags & FWBF_FLAG_EXECUTED_ROUNDS) ? k : a.max_iter;
                        break;
                    }
                    if (!(flags & F_DIFF)) {
                        // same flips as the previous round: z_{k+1} = z_{k-1}, the
                        // states alternate; z_{K_max} = z_k iff K_max - k is even
                        if (((a.max_iter - k) & 1) == 0)
                            for (int u = tid; u < a.W; u += T) {
                                const uint32_t n = s.win[u];
                                if (n != NONE) atomicXor(&s.zw[n >> 5], 1u << (n & 31));
                            }
                        k = (a.flags & FWBF_FLAG_EXECUTED_ROUNDS) ? k : a.max_iter;
                        break;
                    }
                }
                const int weight = s.ctl[CTL_WEIGHT];
                k += 1;
                if (weight == 0) { okf = 1; break; }
                if (k == a.max_iter) break;
            } else {
                // ---- flip the chosen bits; toggle parity of their checks -------
                for (int u = tid; u < a.W; u += T) {
                    const uint32_t n = s.win[u];
                    const uint32_t pv = s.prv[u];
                    s.prv[u] = n;
                    int fl = (n != pv) ? F_DIFF : 0;
                    if (n != NONE) {
                        fl |= F_ANY;
                        atomicXor(&s.zw[n >> 5], 1u << (n & 31));
                        const uint32_t j = fdiv(n, a.magZ, a.maskZ);
                        const int c = (int)(n - j * a.Z);
                        for (int t = 0; t < s.cdeg[j]; t++) {
                            const uint32_t e = s.col[j * a.dvmax + t];
                            int r = c - (int)(e & 0xFFFF);
                            r += (r < 0) ? a.Z : 0;
                            const uint32_t m = (e >> 24) * a.Z + r;
                            atomicXor(&s.tog[m >> 5], 1u << (m & 31));
                        }
                    }
                    if (fl) atomicOr(&s.ctl[fi], fl);
                }
                frame_sync<WAVE>();
                const int flags = s.ctl[fi];
                if (!(a.flags & FWBF_FLAG_NO_CYCLE_EXIT)) {
                    if (!(flags & F_ANY)) {  // no flip: fixed point until K_max
                        k = (a.flags & FWBF_FLAG_EXECUTED_ROUNDS) ? k : a.max_iter;
                        break;
                    }
                    if (!(flags & F_DIFF)) {
                        // same flips as the previous round: z_{k+1} = z_{k-1}, the
                        // states alternate; z_{K_max} = z_k iff K_max - k is even
                        if (((a.max_iter - k) & 1) == 0)
                            for (int u = tid; u < a.W; u += T) {
                                const uint32_t n = s.win[u];
                                if (n != NONE) atomicXor(&s.zw[n >> 5], 1u << (n & 31));
                            }
                        k = (a.flags & FWBF_FLAG_EXECUTED_ROUNDS) ? k : a.max_iter;
                        break;
                    }
                }

                // ---- claim net-toggled checks; update syndrome and its weight --
                for (int u = tid; u < a.W; u += T) {
                    const uint32_t n = s.win[u];
                    uint32_t *tl = s.tl + u * a.dvmax;
                    for (int t = 0; t < a.dvmax; t++) tl[t] = NONE;
                    if (n == NONE) continue;
                    if constexpr (T > 64) {
                        const uint32_t j = fdiv(n, a.magZ, a.maskZ);
                        const int c = (int)(n - j * a.Z);
                        const int deg = s.cdeg[j];
                        int dw = 0;
                        // two checks at a time: their claims, then their syndrome
                        // toggles, each issued together (measured faster in
                        // workgroups wider than one wavefront, slower in one)
                        for (int t0 = 0; t0 < deg; t0 += 2) {
                            uint32_t mq[2], old[2], so[2];
#pragma unroll
                            for (int v = 0; v < 2; v++) {
                                const uint32_t e = s.col[j * a.dvmax + min(t0 + v, deg - 1)];
                                int r = c - (int)(e & 0xFFFF);
                                r += (r < 0) ? a.Z : 0;
                                mq[v] = (e >> 24) * a.Z + r;
                            }
#pragma unroll
                            for (int v = 0; v < 2; v++)
                                old[v] = t0 + v < deg ? atomicAnd(&s.tog[mq[v] >> 5], ~(1u << (mq[v] & 31))) : 0u;
#pragma unroll
                            for (int v = 0; v < 2; v++) {
                                const uint32_t bit = 1u << (mq[v] & 31);
                                so[v] = (old[v] & bit) ? atomicXor(&s.syn[mq[v] >> 5], bit) : 0u;
                            }
#pragma unroll
                            for (int v = 0; v < 2; v++) {
                                const uint32_t bit = 1u << (mq[v] & 31);
                                if (old[v] & bit) {
                                    dw += (so[v] & bit) ? -1 : 1;
                                    tl[t0 + v] = (so[v] & bit) ? mq[v] : (mq[v] | TL_UNSAT);
                                }
                            }
                        }
                        if (dw) atomicAdd(&s.ctl[CTL_WEIGHT], dw);
                    } else {
                        const uint32_t j = fdiv(n, a.magZ, a.maskZ);
                        const int c = (int)(n - j * a.Z);
                        for (int t = 0; t < s.cdeg[j]; t++) {
                            const uint32_t e = s.col[j * a.dvmax + t];
                            int r = c - (int)(e & 0xFFFF);
                            r += (r < 0) ? a.Z : 0;
                            const uint32_t m = (e >> 24) * a.Z + r;
                            const uint32_t bit = 1u << (m & 31);
                            const uint32_t old = atomicAnd(&s.tog[m >> 5], ~bit);
                            if (old & bit) {
                                const uint32_t so = atomicXor(&s.syn[m >> 5], bit);
                                atomicAdd(&s.ctl[CTL_WEIGHT], (so & bit) ? -1 : 1);
                                tl[t] = (so & bit) ? m : (m | TL_UNSAT);
                            }
                        }
                    }
                }
                frame_sync<WAVE>();
                const int weight = s.ctl[CTL_WEIGHT];
                k += 1;
                if (weight == 0) { okf = 1; break; }
                if (k == a.max_iter) break;
            }

            // ---- update the metrics of every bit of a toggled check --------
            const int ntask = a.W * a.dvmax * a.dcmax;
            for (int id = tid; id < ntask; id += T) {
                const uint32_t e0 = fdiv(id, a.magD, a.maskD);
                const uint32_t q = id - e0 * a.dcmax;
                const uint32_t ent = s.tl[e0];
                if (ent == NONE) continue;
                const uint32_t m = ent & ~TL_UNSAT;
                // float: a check toggled by several winners is listed once per
                // toggle; recompute its members for the entries whose new bit
                // is the final one (the last toggle among them)
                if constexpr (Tt::isf)
                    if (((s.syn[m >> 5] >> (m & 31)) & 1) != (ent >> 31)) continue;
                const uint32_t i = fdiv(m, a.magZ, a.maskZ);
                if ((int)q >= s.rdeg[i]) continue;
                const int r = (int)(m - i * a.Z);
                const uint32_t e = s.row[i * a.dcmax + q];
                int cc = r + (int)(e & 0xFFFF);
                cc -= (cc >= a.Z) ? a.Z : 0;
                const uint32_t n = (e >> 16) * a.Z + cc;
                uint32_t g, pos;
                if (a.strided) { pos = fdiv(n, a.magG, a.maskG); g = n - pos * a.Geff; }
                else { g = fdiv(n, a.magP, a.maskP); pos = n - g * a.p; }
                const uint32_t slot = g * a.Lc + pos;
                if constexpr (Tt::isf) {
                    s.keys[slot] = metric_val<DT>(a, s, n, imwbf);  // KEY32 is never used for float
                } else {
                    const int32_t w = weight_i<DT>(s, m, q, imwbf);
                    const int32_t d = (ent & TL_UNSAT) ? 2 * a.aden * w : -2 * a.aden * w;
                    atomicAdd(&s.keys[slot], KEY32 ? ((uint32_t)d << a.idxb) : (uint32_t)d);
                }
            }
            frame_sync<WAVE>();
        }
    }
    frame_sync<WAVE>();

    // ---- output z_k, rounds, syndrome flag --------------------------------
    const int NW = (N + 31) >> 5;
    uint32_t *zo = a.z + f * NW;
    for (int w = tid; w < NW; w += T) zo[w] = s.zw[w];
    if (tid == 0) {
        a.iters[f] = k + (a.skip ? a.iters[f] : 0);
        a.ok[f] = (uint8_t)okf;
    }
    frame_sync<WAVE>();
}

template <int DT, bool KEY32, int T>
__global__ __launch_bounds__(T) void decode_kernel(DecodeArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Lds s;
    s.keys = (uint32_t *)(smem + a.o_keys);
    s.chk = smem + a.o_chk;
    s.chkp = smem + a.o_chkp;
    s.mag = smem + a.o_mag;
    s.zw = (uint32_t *)(smem + a.o_z);
    s.syn = (uint32_t *)(smem + a.o_syn);
    s.tog = (uint32_t *)(smem + a.o_tog);
    s.win = (uint32_t *)(smem + a.o_win);
    s.prv = (uint32_t *)(smem + a.o_prv);
    s.tl = (uint32_t *)(smem + a.o_tl);
    s.gb = (unsigned long long *)(smem + a.o_gb);
    s.topk = (unsigned long long *)(smem + a.o_top);
    s.topn = (uint32_t *)(smem + a.o_top + 8 * a.lambda);
    s.ctl = (int *)(smem + a.o_ctl);
    s.col = (uint32_t *)(smem + a.o_col);
    s.row = (uint32_t *)(smem + a.o_row);
    s.cdeg = smem + a.o_cdeg;
    s.rdeg = smem + a.o_rdeg;
    for (int t = threadIdx.x; t < a.nb * a.dvmax; t += T) s.col[t] = a.col[t];
    for (int t = threadIdx.x; t < a.mb * a.dcmax; t += T) s.row[t] = a.row[t];
    for (int t = threadIdx.x; t < a.nb; t += T) s.cdeg[t] = a.coldeg[t];
    for (int t = threadIdx.x; t < a.mb; t += T) s.rdeg[t] = a.rowdeg[t];
    __syncthreads();
    const FrameRange fr = xcd_frames(a.F);
    for (int64_t f = fr.first; f < fr.end; f += fr.step) decode_frame<DT, KEY32, T>(a, s, f);
}

// ---------------------------------------------------------------------------
// Mixed-code persistent launch: frames of up to 8 decode jobs (each its own
// code, parameters and buffers) are claimed one at a time from a global
// ticket counter, so a workgroup whose frame ends early takes the next
// unclaimed frame of any job.  Job descriptors travel as kernel arguments.
// ---------------------------------------------------------------------------
constexpr int MAX_JOBS = 8;

// A ticket is a chunk of consecutive frames of one job.  Jobs whose frames
// need one wavefront (wave[j]) are decoded one frame per wavefront, each
// wavefront in its own LDS region of lds_job[j] bytes; the others by the
// whole workgroup.
struct BatchArgs {
    DecodeArgs job[MAX_JOBS];
    int64_t cbase[MAX_JOBS + 1];  // first ticket of each job; cbase[njobs] = number of tickets
    int chunk[MAX_JOBS];
    int wave[MAX_JOBS];
    int lds_job[MAX_JOBS];
    int njobs;
    unsigned long long *counter;
};
static_assert(sizeof(BatchArgs) <= 4096, "batch descriptors must fit the kernel argument segment");

__device__ __forceinline__ Lds lds_of(unsigned char *smem, const DecodeArgs &a)
{
    Lds s;
    s.keys = (uint32_t *)(smem + a.o_keys);
    s.chk = smem + a.o_chk;
    s.chkp = smem + a.o_chkp;
    s.mag = smem + a.o_mag;
    s.zw = (uint32_t *)(smem + a.o_z);
    s.syn = (uint32_t *)(smem + a.o_syn);
    s.tog = (uint32_t *)(smem + a.o_tog);
    s.win = (uint32_t *)(smem + a.o_win);
    s.prv = (uint32_t *)(smem + a.o_prv);
    s.tl = (uint32_t *)(smem + a.o_tl);
    s.gb = (unsigned long long *)(smem + a.o_gb);
    s.topk = (unsigned long long *)(smem + a.o_top);
    s.topn = (uint32_t *)(smem + a.o_top + 8 * a.lambda);
    s.ctl = (int *)(smem + a.o_ctl);
    s.col = (uint32_t *)(smem + a.o_col);
    s.row = (uint32_t *)(smem + a.o_row);
    s.cdeg = smem + a.o_cdeg;
    s.rdeg = smem + a.o_rdeg;
    s.yrow = nullptr;
    return s;
}

template <int DT, bool KEY32, int T>
__global__ __launch_bounds__(T) void batched_kernel(BatchArgs b)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_ticket;
    for (;;) {
        if (threadIdx.x == 0) s_ticket = (long long)atomicAdd(b.counter, 1ull);
        __syncthreads();
        const long long tk = s_ticket;
        __syncthreads();  // every thread has read the ticket before it is overwritten
        if (tk >= b.cbase[b.njobs]) break;
        int j = 0;
        while (j + 1 < b.njobs && b.cbase[j + 1] <= tk) j++;
        const DecodeArgs &a = b.job[j];
        const int64_t f0 = (tk - b.cbase[j]) * b.chunk[j];
        const int64_t f1 = f0 + b.chunk[j] < a.F ? f0 + b.chunk[j] : a.F;
        bool done = false;
        if constexpr (T > 64) {
            if (b.wave[j]) {
                const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
                Lds s = lds_of(smem + w * b.lds_job[j], a);
                for (int t = lane; t < a.nb * a.dvmax; t += 64) s.col[t] = a.col[t];
                for (int t = lane; t < a.mb * a.dcmax; t += 64) s.row[t] = a.row[t];
                for (int t = lane; t < a.nb; t += 64) s.cdeg[t] = a.coldeg[t];
                for (int t = lane; t < a.mb; t += 64) s.rdeg[t] = a.rowdeg[t];
                frame_sync<true>();
                for (int64_t f = f0 + w; f < f1; f += T / 64) decode_frame<DT, KEY32, 64, true>(a, s, f);
                __syncthreads();  // the regions are reused by the next ticket
                done = true;
            }
        }
        if (!done) {
            Lds s = lds_of(smem, a);
            for (int t = threadIdx.x; t < a.nb * a.dvmax; t += T) s.col[t] = a.col[t];
            for (int t = threadIdx.x; t < a.mb * a.dcmax; t += T) s.row[t] = a.row[t];
            for (int t = threadIdx.x; t < a.nb; t += T) s.cdeg[t] = a.coldeg[t];
            for (int t = threadIdx.x; t < a.mb; t += T) s.rdeg[t] = a.rowdeg[t];
            __syncthreads();
            for (int64_t f = f0; f < f1; f++) decode_frame<DT, KEY32, T>(a, s, f);
        }
    }
}

__global__ void reset_counter(unsigned long long *c) { *c = 0ull; }

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void magic(uint32_t d, uint32_t *mag, uint32_t *mask)
{
    if (d <= 1) { *mag = 0; *mask = 0xFFFFFFFFu; return; }
    *mag = (uint32_t)(((1ULL << 32) + d - 1) / d);  // ceil(2^32 / d), exact for n*d < 2^32
    *mask = 0;
}

int ilog2(uint32_t v) { int r = 0; while ((1u << r) < v) r++; return r; }

struct Plan {
    int C, L, P;
    long cost;
};

// choose C (slots per thread) and L (threads per block, a power of two)
Plan plan_layout(int Geff, int p, int T)
{
    Plan best{0, 0, 0, -1};
    for (int C = 1; C <= 64; C++) {
        const int need = (p + C - 1) / C;
        const int L = 1 << ilog2(need);
        if (L > T) continue;
        const int GP = T / L;
        const int P = (Geff + GP - 1) / GP;
        const long cost = (long)P * C + 2L * P * std::min(ilog2(L), 6) + (L > 64 ? 8 : 0);
        if (best.cost < 0 || cost < best.cost) best = Plan{C, L, P, cost};
    }
    return best;
}

template <int DT, bool KEY32>
hipError_t launch_t(int T, const DecodeArgs &a, int grid, hipStream_t st)
{
    switch (T) {
#define FWBF_CASE(TT)                                                                                 \
    case TT:                                                                                          \
        if (a.lds_bytes > 65536)                                                                      \
            (void)hipFuncSetAttribute((const void *)decode_kernel<DT, KEY32, TT>,                     \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes);       \
        hipLaunchKernelGGL((decode_kernel<DT, KEY32, TT>), dim3(grid), dim3(TT), a.lds_bytes, st, a); \
        return hipGetLastError();
        FWBF_CASE(64)
        FWBF_CASE(128)
        FWBF_CASE(256)
        FWBF_CASE(512)
        FWBF_CASE(1024)
#undef FWBF_CASE
    }
    return hipErrorInvalidValue;
}

template <int DT, bool KEY32>
int occupancy_t(int T, int lds, int *blocks)
{
    hipError_t e = hipErrorInvalidValue;
    switch (T) {
#define FWBF_CASE(TT)                                                                               \
    case TT:                                                                                        \
        if (lds > 65536)                                                                            \
            (void)hipFuncSetAttribute((const void *)decode_kernel<DT, KEY32, TT>,                   \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);             \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, decode_kernel<DT, KEY32, TT>, TT, lds); \
        break;
        FWBF_CASE(64)
        FWBF_CASE(128)
        FWBF_CASE(256)
        FWBF_CASE(512)
        FWBF_CASE(1024)
#undef FWBF_CASE
    }
    return e == hipSuccess ? FWBF_OK : hip_fail(e, "occupancy query");
}

int dispatch(int DT, bool key32, int T, const DecodeArgs &a, int grid, hipStream_t st)
{
    hipError_t e;
    if (DT == FWBF_I8) e = key32 ? launch_t<FWBF_I8, true>(T, a, grid, st) : launch_t<FWBF_I8, false>(T, a, grid, st);
    else if (DT == FWBF_I16) e = key32 ? launch_t<FWBF_I16, true>(T, a, grid, st) : launch_t<FWBF_I16, false>(T, a, grid, st);
    else e = launch_t<FWBF_F32, false>(T, a, grid, st);
    return e == hipSuccess ? FWBF_OK : hip_fail(e, "decode kernel launch");
}

int occupancy(int DT, bool key32, int T, int lds, int *blocks)
{
    if (DT == FWBF_I8) return key32 ? occupancy_t<FWBF_I8, true>(T, lds, blocks) : occupancy_t<FWBF_I8, false>(T, lds, blocks);
    if (DT == FWBF_I16) return key32 ? occupancy_t<FWBF_I16, true>(T, lds, blocks) : occupancy_t<FWBF_I16, false>(T, lds, blocks);
    return occupancy_t<FWBF_F32, false>(T, lds, blocks);
}

}  // namespace

// Validates parameters and fills the kernel arguments (everything but the
// data pointers).  Shared by the plain decoder and the batched launch.
int prepare_decode(const fwbf_code *c, const fwbf_params *p, DecodeArgs *out, int *T_out, bool force_key64 = false,
                   bool force_alias = false);
int try_fast_decode(const fwbf_code *c, const fwbf_params *p, const void *y, int64_t F, int64_t stride,
                    uint32_t *z, int32_t *iters, uint8_t *ok, hipStream_t st, const uint32_t *shift_dev,
                    const uint8_t *skip, int iters_add);
int try_cyclic_decode(const fwbf_code *c, const fwbf_params *p, const void *y, int64_t F, int64_t stride,
                      uint32_t *z, int32_t *iters, uint8_t *ok, hipStream_t st);
// The general kernel (any code, dtype and selection); with a skip list, only
// frames with skip[f] == 0 are decoded and their rounds add to iters[f].
int decode_general(const fwbf_code *code, const fwbf_params *params, const void *y_dev, int64_t F, int64_t y_stride,
                   uint32_t *z_dev, int32_t *iters_dev, uint8_t *ok_dev, hipStream_t stream, const uint8_t *skip);

int prepare_decode(const fwbf_code *c, const fwbf_params *p, DecodeArgs *out, int *T_out, bool force_key64,
                   bool force_alias)
{
    if (!c || !p) return fail(FWBF_E_INVALID, "null code or params");
    if (p->dtype < FWBF_F32 || p->dtype > FWBF_I16) return fail(FWBF_E_INVALID, "unknown dtype");
    if (p->weights < FWBF_WBF || p->weights > FWBF_IMWBF) return fail(FWBF_E_INVALID, "unknown weights");
    if (p->select < FWBF_GROUPS || p->select > FWBF_STRIDED) return fail(FWBF_E_INVALID, "unknown select");
    if ((p->select == FWBF_GROUPS || p->select == FWBF_STRIDED) && (p->groups < 1 || p->groups > c->N))
        return fail(FWBF_E_INVALID, "groups must be in [1, N]");
    if (p->select == FWBF_TOPL && (p->lambda < 1 || p->lambda > 64))
        return fail(FWBF_E_INVALID, "lambda must be in [1, 64]");
    if (p->max_iter < 0) return fail(FWBF_E_INVALID, "max_iter must be >= 0");
    if (p->dtype != FWBF_F32 && (p->alpha_den < 1 || p->alpha_num < 0))
        return fail(FWBF_E_INVALID, "alpha_num must be >= 0 and alpha_den >= 1");
    if (p->dtype == FWBF_F32 && !(p->alpha == p->alpha)) return fail(FWBF_E_INVALID, "alpha is NaN");

    DecodeArgs a;
    memset(&a, 0, sizeof a);
    a.N = c->N; a.M = c->M; a.Z = c->Z; a.mb = c->mb; a.nb = c->nb;
    a.dvmax = c->dv_max; a.dcmax = c->dc_max;
    a.weights = p->weights; a.select = p->select; a.max_iter = p->max_iter;
    a.lambda = p->select == FWBF_TOPL ? p->lambda : 1;
    a.alpha = p->weights == FWBF_WBF ? 0.0f : p->alpha;
    a.anum = p->weights == FWBF_WBF ? 0 : p->alpha_num;
    a.aden = p->alpha_den;
    a.flags = p->flags;
    a.multi = c->multi ? 1 : 0;

    int T = p->threads_per_frame;
    if (T == 0) T = c->N <= 2048 ? 64 : c->N <= 4096 ? 128 : c->N <= 16384 ? 256 : 1024;
    if (T != 64 && T != 128 && T != 256 && T != 512 && T != 1024)
        return fail(FWBF_E_INVALID, "threads_per_frame must be 0, 64, 128, 256, 512 or 1024");

    const int G = (p->select == FWBF_GROUPS || p->select == FWBF_STRIDED) ? p->groups : 1;
    a.p = (c->N + G - 1) / G;
    a.strided = p->select == FWBF_STRIDED;
    a.Geff = a.strided ? G : (c->N + a.p - 1) / a.p;  // strided: every residue class is nonempty
    Plan pl = plan_layout(a.Geff, a.p, T);
    if (pl.cost < 0) return fail(FWBF_E_UNSUPPORTED, "block too long for threads_per_frame (use more threads)");
    if (p->select == FWBF_TOPL && pl.P != 1) return fail(FWBF_E_UNSUPPORTED, "top-lambda layout");
    a.C = pl.C; a.L = pl.L; a.logL = ilog2(pl.L); a.GP = T / pl.L; a.P = pl.P; a.Lc = pl.L * pl.C;
    a.W = p->select == FWBF_TOPL ? p->lambda : a.Geff;
    // the update phase divides task ids < W*dv*dc by dc with a 32-bit magic
    if ((int64_t)a.W * c->dv_max * c->dc_max * c->dc_max >= (1LL << 32))
        return fail(FWBF_E_UNSUPPORTED, "too many blocks for this code's degrees");

    // value range of the metric
    bool key32 = false;
    if (p->dtype == FWBF_F32) {
        a.bias = 0;
        a.zero_val = 0x80000000u;  // orderable(+0)
    } else {
        const int64_t maxmag = p->dtype == FWBF_I8 ? 128 : 32768;
        const int64_t maxE = maxmag * ((int64_t)a.aden * c->dv_max + a.anum);
        if (maxE >= (1LL << 30)) return fail(FWBF_E_UNSUPPORTED, "alpha_num/alpha_den too large for 32-bit metrics");
        int vb = 1;
        while ((1LL << (vb - 1)) <= maxE) vb++;
        a.bias = 1u << (vb - 1);
        a.zero_val = a.bias;
        a.idxb = ilog2((uint32_t)a.Lc);
        if (vb + a.idxb <= 32 && !force_key64) key32 = true;
        a.idxmask = key32 ? (a.idxb ? ((1u << a.idxb) - 1) : 0) : 0;
    }
    magic(a.Z, &a.magZ, &a.maskZ);
    magic(a.p, &a.magP, &a.maskP);
    magic(a.Geff, &a.magG, &a.maskG);
    magic(a.dcmax, &a.magD, &a.maskD);

    // LDS layout; |y| gets its own array when everything fits, else it
    // overlays the slots during initialisation only
    const int slots = a.P * T * a.C;
    const int Nr = (c->N + 63) / 64 * 64, Mr = (c->M + 63) / 64 * 64;
    const int chk_sz = p->dtype == FWBF_F32 ? 8 : 4;
    const int mag_sz = p->dtype == FWBF_I8 ? 1 : p->dtype == FWBF_I16 ? 2 : 4;
    auto layout = [&](bool alias) {
        int off = 0;
        auto take = [&](int bytes, int align) { off = (off + align - 1) / align * align; int o = off; off += bytes; return o; };
        a.o_keys = take(4 * slots, 16);
        a.o_chk = take(chk_sz * c->M, 8);
        a.o_chkp = take(p->dtype == FWBF_I8 ? 0 : c->M, 4);
        a.o_mag = alias ? a.o_keys : take(mag_sz * c->N, 4);
        a.o_z = take(Nr / 8, 8);
        a.o_syn = take(Mr / 8, 8);
        a.o_tog = take(Mr / 8, 8);
        a.o_win = take(4 * a.W, 4);
        a.o_prv = take(4 * a.W, 4);
        a.o_tl = take(4 * a.W * a.dvmax, 4);
        a.o_gb = take(8 * std::max(a.Geff, 2), 8);
        a.o_top = take(12 * a.lambda, 8);
        a.o_ctl = take(16, 4);
        a.o_col = take(4 * c->nb * c->dv_max, 4);
        a.o_row = take(4 * c->mb * c->dc_max, 4);
        a.o_cdeg = take(c->nb, 1);
        a.o_rdeg = take(c->mb, 1);
        a.lds_bytes = (off + 15) / 16 * 16;
        a.mag_alias = alias ? 1 : 0;
    };
    layout(force_alias);
    if (a.lds_bytes > 160 * 1024) layout(true);
    if (a.lds_bytes > 160 * 1024) return fail(FWBF_E_UNSUPPORTED, "frame state exceeds 160 KiB of LDS");
    a.idxb = key32 ? a.idxb : 0;
    *out = a;
    *T_out = T;
    return key32 ? 1 : 0;
}

}  // namespace fwbf

using namespace fwbf;

extern "C" int fwbf_decode(const fwbf_code *code, const fwbf_params *params, const void *y_dev, int64_t F,
                           int64_t y_stride, uint32_t *z_dev, int32_t *iters_dev, uint8_t *ok_dev,
                           void *stream)
{
    DecodeArgs a;
    int T = 0;
    const int k = prepare_decode(code, params, &a, &T);
    if (k < 0) return k;
    if (F < 0) return fail(FWBF_E_INVALID, "F must be >= 0");
    if (y_stride < code->N) return fail(FWBF_E_INVALID, "y_stride must be >= N");
    if (F == 0) return FWBF_OK;
    if (!y_dev || !z_dev || !iters_dev || !ok_dev) return fail(FWBF_E_INVALID, "null buffer");
    DeviceTables t;
    int rc = device_tables(const_cast<fwbf_code *>(code), &t);
    if (rc) return rc;
    if (!(params->flags & FWBF_FLAG_GENERIC_KERNEL)) {
        rc = try_cyclic_decode(code, params, y_dev, F, y_stride, z_dev, iters_dev, ok_dev, (hipStream_t)stream);
        if (rc != 0) return rc < 0 ? rc : FWBF_OK;
        rc = try_fast_decode(code, params, y_dev, F, y_stride, z_dev, iters_dev, ok_dev, (hipStream_t)stream,
                             t.shift, nullptr, 0);
        if (rc != 0) return rc < 0 ? rc : FWBF_OK;
    }
    if (params->flags & FWBF_FLAG_SPECIALISED_ONLY)
        return fail(FWBF_E_UNSUPPORTED, "no specialised kernel takes these parameters");
    return decode_general(code, params, y_dev, F, y_stride, z_dev, iters_dev, ok_dev, (hipStream_t)stream, nullptr);
}

namespace fwbf {
int decode_general(const fwbf_code *code, const fwbf_params *params, const void *y_dev, int64_t F, int64_t y_stride,
                   uint32_t *z_dev, int32_t *iters_dev, uint8_t *ok_dev, hipStream_t stream, const uint8_t *skip)
{
    DecodeArgs a;
    int T = 0;
    const int k = prepare_decode(code, params, &a, &T);
    if (k < 0) return k;
    DeviceTables t;
    int rc = device_tables(const_cast<fwbf_code *>(code), &t);
    if (rc) return rc;
    int dev = 0, cus = 0, blocks = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    // the layout for parameters pp and how many of its workgroups fit on a
    // compute unit; returns prepare_decode's key mode or an error code
    auto choose = [&](const fwbf_params *pp, DecodeArgs &out, int &Tout, int &bl) -> int {
        const int kk = prepare_decode(code, pp, &out, &Tout);
        if (kk < 0) return kk;
        int r = occupancy(pp->dtype, kk == 1, Tout, out.lds_bytes, &bl);
        if (r) return r;
        if (!out.mag_alias) {
            // staging |y| over the slots shrinks the frame's LDS; take that
            // layout when it lets more frames share a compute unit
            DecodeArgs b;
            int Tb = 0, bb = 0;
            if (prepare_decode(code, pp, &b, &Tb, false, true) == kk) {
                r = occupancy(pp->dtype, kk == 1, Tout, b.lds_bytes, &bb);
                if (r) return r;
                if (bb > bl) {
                    out = b;
                    bl = bb;
                }
            }
        }
        return kk;
    };
    int kc = choose(params, a, T, blocks);
    if (kc < 0) return kc;
    if (params->threads_per_frame == 0 && T < 1024) {
        // a batch that the wider launch holds at once (every frame gets its
        // own workgroup immediately) is bound by the time of one frame, and
        // twice the threads per frame shortens each frame's phases
        fwbf_params p2 = *params;
        p2.threads_per_frame = 2 * T;
        DecodeArgs a2;
        int T2 = 0, blocks2 = 0;
        const int k2 = choose(&p2, a2, T2, blocks2);
        if (k2 >= 0 && blocks2 >= 1 && F <= (int64_t)blocks2 * cus) {
            a = a2;
            T = T2;
            blocks = blocks2;
            kc = k2;
        }
    }
    const bool key32 = kc == 1;
    if (blocks < 1) return fail(FWBF_E_UNSUPPORTED, "decode kernel does not fit on a compute unit");
    a.y = y_dev; a.F = F; a.stride = y_stride;
    a.z = z_dev; a.iters = iters_dev; a.ok = ok_dev;
    a.col = t.col; a.row = t.row; a.coldeg = t.coldeg; a.rowdeg = t.rowdeg;
    a.skip = skip;
    const int64_t grid = std::min<int64_t>(F, (int64_t)blocks * cus);
    return dispatch(params->dtype, key32, T, a, (int)grid, stream);
}
}  // namespace fwbf

// ---------------------------------------------------------------------------
// mixed-code batch
// ---------------------------------------------------------------------------
namespace fwbf {
namespace {
template <int DT>
hipError_t launch_batched(int T, const BatchArgs &b, int lds, int grid, hipStream_t st)
{
    switch (T) {
#define FWBF_CASE(TT)                                                                                \
    case TT:                                                                                         \
        if (lds > 65536)                                                                             \
            (void)hipFuncSetAttribute((const void *)batched_kernel<DT, false, TT>,                   \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);              \
        hipLaunchKernelGGL((batched_kernel<DT, false, TT>), dim3(grid), dim3(TT), lds, st, b);       \
        return hipGetLastError();
        FWBF_CASE(64)
        FWBF_CASE(128)
        FWBF_CASE(256)
        FWBF_CASE(512)
        FWBF_CASE(1024)
#undef FWBF_CASE
    }
    return hipErrorInvalidValue;
}
template <int DT>
hipError_t occupancy_batched(int T, int lds, int *blocks)
{
    switch (T) {
#define FWBF_CASE(TT)                                                                                \
    case TT:                                                                                         \
        if (lds > 65536)                                                                             \
            (void)hipFuncSetAttribute((const void *)batched_kernel<DT, false, TT>,                   \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);              \
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, batched_kernel<DT, false, TT>, TT, lds);
        FWBF_CASE(64)
        FWBF_CASE(128)
        FWBF_CASE(256)
        FWBF_CASE(512)
        FWBF_CASE(1024)
#undef FWBF_CASE
    }
    return hipErrorInvalidValue;
}
}  // namespace
}  // namespace fwbf

// Scratch of the no-allocation entry point: the ticket counter lives here
// instead of in a caller workspace.  Each device holds its own copy until
// the process ends.  In host code `scratch` only stands for the symbol; its
// device address comes from hipGetSymbolAddress, looked up once per device.
constexpr size_t SCRATCH_BYTES = 256;
constexpr size_t SCRATCH_NEED = sizeof(unsigned long long);  // one counter, whatever the batch
static_assert(SCRATCH_NEED <= SCRATCH_BYTES, "scratch too small for the ticket counter");
static __device__ __align__(256) unsigned long long scratch[SCRATCH_BYTES / sizeof(unsigned long long)];

namespace fwbf {
namespace {
// The batched launch behind both entry points.  `counter` is the ticket
// counter (device memory, cleared here by a kernel).  With resident_only,
// the code tables must already be on the device (nothing is allocated).
int batched_impl(const fwbf_batch_item *items, int n_items, int threads_per_frame, int blocks_per_cu,
                 unsigned long long *counter, void *stream, bool resident_only)
{
    if (!items || n_items < 1 || n_items > MAX_JOBS)
        return fail(FWBF_E_INVALID, "n_items must be in [1, 8]");
    if (blocks_per_cu < 0) return fail(FWBF_E_INVALID, "blocks_per_cu must be >= 0");
    const int dtype = items[0].params ? items[0].params->dtype : -1;
    int T = threads_per_frame;
    for (int i = 0; i < n_items; i++) {
        const fwbf_batch_item &it = items[i];
        if (!it.code || !it.params) return fail(FWBF_E_INVALID, "null code or params in a batch item");
        if (it.params->dtype != dtype) return fail(FWBF_E_UNSUPPORTED, "all batch items must share the dtype");
        if (it.F < 0 || it.y_stride < it.code->N) return fail(FWBF_E_INVALID, "invalid size in a batch item");
        if (it.F > 0 && (!it.y_dev || !it.z_dev || !it.iters_dev || !it.ok_dev))
            return fail(FWBF_E_INVALID, "null buffer in a batch item");
        if (threads_per_frame == 0) {
            const int N = it.code->N;
            const int t = N <= 2048 ? 64 : N <= 4096 ? 128 : N <= 16384 ? 256 : 1024;
            T = std::max(T, t);
        }
    }
    // builds the job table for one LDS layout; returns the dynamic LDS the
    // launch needs (the largest job's), or an error code
    int64_t total = 0;
    for (int i = 0; i < n_items; i++) total += items[i].F;
    auto build = [&](bool alias, BatchArgs &b) -> int {
        memset(&b, 0, sizeof b);
        b.njobs = n_items;
        int lds = 0;
        int64_t tickets = 0;
        for (int i = 0; i < n_items; i++) {
            const fwbf_batch_item &it = items[i];
            fwbf_params p = *it.params;
            // frames that take 64 threads on their own are decoded one per
            // wavefront when the launch is wider (automatic width only)
            const int N = it.code->N;
            const bool wave = threads_per_frame == 0 && T > 64 && N <= 2048;
            p.threads_per_frame = wave ? 64 : T;
            int Ti = 0;
            int k = prepare_decode(it.code, &p, &b.job[i], &Ti, true, alias);
            if (k < 0) return k;
            b.wave[i] = wave && (int64_t)(T / 64) * b.job[i].lds_bytes <= 160 * 1024;
            if (wave && !b.wave[i]) {
                p.threads_per_frame = T;
                k = prepare_decode(it.code, &p, &b.job[i], &Ti, true, alias);
                if (k < 0) return k;
            }
            b.lds_job[i] = b.job[i].lds_bytes;
            b.chunk[i] = b.wave[i] ? 4 * (T / 64) : 2;
            DeviceTables tb;
            const int rc = resident_only ? device_tables_resident(it.code, &tb)
                                         : device_tables(const_cast<fwbf_code *>(it.code), &tb);
            if (rc) return rc;
            DecodeArgs &a = b.job[i];
            a.y = it.y_dev; a.F = it.F; a.stride = it.y_stride;
            a.z = it.z_dev; a.iters = it.iters_dev; a.ok = it.ok_dev;
            a.col = tb.col; a.row = tb.row; a.coldeg = tb.coldeg; a.rowdeg = tb.rowdeg;
            b.cbase[i] = tickets;
            tickets += (it.F + b.chunk[i] - 1) / b.chunk[i];
            lds = std::max(lds, b.wave[i] ? (T / 64) * a.lds_bytes : a.lds_bytes);
        }
        b.cbase[n_items] = tickets;
        return lds;
    };
    auto blocks_for = [&](int lds, int *blocks) {
        return dtype == FWBF_F32 ? occupancy_batched<FWBF_F32>(T, lds, blocks)
               : dtype == FWBF_I8 ? occupancy_batched<FWBF_I8>(T, lds, blocks)
                                  : occupancy_batched<FWBF_I16>(T, lds, blocks);
    };
    BatchArgs b;
    int lds = build(false, b);
    if (lds < 0) return lds;
    if (total == 0) return FWBF_OK;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, cus = 0, blocks = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = blocks_for(lds, &blocks);
    if (e != hipSuccess) return hip_fail(e, "batched occupancy");
    {
        // staging |y| over the slots shrinks every job's LDS (and lets more
        // jobs take the one-frame-per-wavefront form); take that layout when
        // it lets more workgroups share a compute unit
        BatchArgs b2;
        const int lds2 = build(true, b2);
        if (lds2 < 0) return lds2;
        int blocks2 = 0;
        e = blocks_for(lds2, &blocks2);
        if (e != hipSuccess) return hip_fail(e, "batched occupancy");
        if (blocks2 > blocks) {
            b = b2;
            lds = lds2;
            blocks = blocks2;
        }
    }
    b.counter = counter;
    if (blocks < 1) return fail(FWBF_E_UNSUPPORTED, "batched kernel does not fit on a compute unit");
    if (blocks_per_cu > 0) blocks = std::min(blocks, blocks_per_cu);
    const int64_t grid = std::min<int64_t>(b.cbase[n_items], (int64_t)blocks * cus);
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, st, b.counter);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = dtype == FWBF_F32 ? launch_batched<FWBF_F32>(T, b, lds, (int)grid, st)
            : dtype == FWBF_I8 ? launch_batched<FWBF_I8>(T, b, lds, (int)grid, st)
                               : launch_batched<FWBF_I16>(T, b, lds, (int)grid, st);
    return e == hipSuccess ? FWBF_OK : hip_fail(e, "batched decode launch");
}

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[MAX_DEVICES];  // per device: address of that device's copy

int scratch_ptr(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(FWBF_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(FWBF_E_HIP, "hipGetSymbolAddress(scratch) returned null");
        scratch_dev[dev] = ptr;
    }
    *out = scratch_dev[dev];
    return FWBF_OK;
}
}  // namespace
}  // namespace fwbf

extern "C" int fwbf_decode_batched(const fwbf_batch_item *items, int n_items, int threads_per_frame,
                                   int blocks_per_cu, void *workspace_dev, size_t workspace_bytes, void *stream)
{
    if (!workspace_dev || workspace_bytes < 256) return fail(FWBF_E_INVALID, "workspace must hold 256 bytes");
    return batched_impl(items, n_items, threads_per_frame, blocks_per_cu, (unsigned long long *)workspace_dev,
                        stream, false);
}

extern "C" int fwbf_decode_batched_noalloc(const fwbf_batch_item *items, int n_items, int threads_per_frame,
                                           int blocks_per_cu, void *stream)
{
    void *ptr = nullptr;
    const int rc = scratch_ptr(&ptr);
    if (rc) return rc;
    return batched_impl(items, n_items, threads_per_frame, blocks_per_cu, (unsigned long long *)ptr, stream, true);
}
