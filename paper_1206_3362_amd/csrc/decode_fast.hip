// One-wave-per-frame FWBF kernel for fixed-point inputs on regular QC codes
// (every base entry a circulant permutation, column weight DV, row weight
// DC known at compile time).  Same results as the generic kernel in
// decode.hip, with fewer instructions per round:
//   - the block maximum is an xor-butterfly over L lanes of packed 32-bit
//     keys (metric << idxb | ~position), C keys per lane read as 16-byte
//     vectors from an interleaved slot layout (lane-consecutive 16-byte
//     chunks, no bank conflicts);
//   - the flip, the syndrome toggle and the metric update are one pass:
//     every lane of a block holds the block's winner after the butterfly,
//     and the block's own lanes take its DV checks (a lane pair per check,
//     three members each, where a block has at least 2 DV lanes), toggling
//     each with an LDS xor that returns the old word; the new syndrome bit
//     fixes the sign of the change +-2 a_den w of every member metric.
//     The syndrome bit is bit 7 of the check's min1-position byte, so the
//     one xor also returns the position and the check phase stores both
//     with one byte write.
//     Toggles of one check by two winners in the same round are serialised
//     by the LDS atomics and their changes cancel exactly, so no separate
//     parity pass is needed;
//   - the initial metrics are pushed from the check side while the check
//     minima are computed (each check adds its signed reliability to its
//     members; the first check of a column also adds -a_num |y_n|);
//   - winner bookkeeping (previous flips, flip masks, the unsatisfied-check
//     count) stays in registers and wave ballots;
//   - a workgroup holds FAST_WAVES independent wavefronts, each decoding its
//     own frames with wavefront-scope barriers; the frame-independent tables
//     (shifts, the slot of every bit with each block column stored twice)
//     are stored once per workgroup, which with at most 96 VGPRs gives 5
//     wavefronts per SIMD;
//   - tests of kernel arguments inside the loops use copies taken there
//     (fresh()), so they stay scalar compares rather than loop-long lane
//     masks that would spill.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "frames.h"
#include "internal.h"

namespace fwbf {
namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int FAST_WAVES = 4;  // independent wavefronts (frames) per workgroup

struct FastArgs {
    const void *y;
    int64_t F, stride;
    uint32_t *z;
    int32_t *iters;
    uint8_t *ok;
    const uint32_t *shift;  // DV x nb shifts (block row-major)
    const uint8_t *skip;    // optional: frames with skip[f] != 0 are left untouched
    int iters_add;          // add the rounds to iters[f] instead of storing them
    int N, M, Z, nb;
    uint32_t magP, maskP, magG, maskG;
    uint32_t rZ24;  // n / Z = (n * rZ24) >> 20 for every bit n
    int strided;  // block g = {n : n mod G = g}: bit n = pos G + g
    int p, L, logL, Geff, Lc;
    int single, imwbf, max_iter, cycle_exit, vec_ok;
    int exec_rounds;  // report the rounds run before a repeated state (diagnostic)
    int aden, anum, idxb;
    // a_den << idxb and 2 a_den << idxb (24-bit multiplicands of the check
    // weights), -(a_num << idxb) (signed 24-bit multiplicand of |y|)
    uint32_t kden, kden2;
    int nknum;
    uint32_t idxmask, bias, zero_val;
    // LDS offsets in bytes
    // LDS: tables shared by the workgroup (o_sh, o_slot), then one region of
    // wave_bytes per wavefront (offsets relative to the region; keys at 0)
    int o_chk, o_chkp, o_y, o_z, o_sh, o_slot, o_wave0, wave_bytes, lds_bytes;
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t mag, uint32_t mask)
{
    return __umulhi(n, mag) + (n & mask);
}

// (a - b) mod Z for a, b in [0, Z)
__device__ __forceinline__ uint32_t submod(uint32_t a, uint32_t b, uint32_t Z)
{
    const uint32_t s = a - b;
    return min(s, s + Z);
}

// Slot layout: the kk-th 16-byte chunk of lane l sits at chunk index
// kk*64 + (l ^ 4*(kk mod 16)).  For a fixed kk the lanes read 64 distinct
// consecutive chunks (conflict-free vector reads in the block maximum), and
// 64 consecutive bits (4 lanes x 16 slots) land in 64 distinct banks
// (conflict-free atomics when a check pushes to its members).
__device__ __forceinline__ uint32_t chunk_of(uint32_t lane, uint32_t kk)
{
    return (kk << 6) + (lane ^ ((kk & 15) << 2));
}
__device__ __forceinline__ uint32_t slot_addr(uint32_t lane, uint32_t k)
{
    return chunk_of(lane, k >> 2) * 4 + (k & 3);
}

// row-local data movement (DPP): xor 1, xor 2, mirror within 8, mirror within 16
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// maximum over aligned groups of L lanes (L a power of two <= 64); every
// lane of a group ends with the group maximum
__device__ __forceinline__ uint32_t group_max(uint32_t v, int L)
{
    if (L > 1) v = max(v, dpp<0xB1>(v));   // quad_perm [1,0,3,2]
    if (L > 2) v = max(v, dpp<0x4E>(v));   // quad_perm [2,3,0,1]
    if (L > 4) v = max(v, dpp<0x141>(v));  // row_half_mirror
    if (L > 8) v = max(v, dpp<0x140>(v));  // row_mirror
    if (L > 16) v = max(v, (uint32_t)__shfl_xor((int)v, 16, 64));
    if (L > 32) v = max(v, (uint32_t)__shfl_xor((int)v, 32, 64));
    return v;
}

template <int DT> struct FT;
template <> struct FT<FWBF_I8> {
    using Y = int8_t;
};
template <> struct FT<FWBF_I16> {
    using Y = int16_t;
};

// Ordering of one wavefront's LDS operations across its lanes: a frame
// belongs to one wavefront, whose LDS operations complete in issue order;
// the fences and the wave barrier keep the compiler from moving memory
// operations across this point.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Initialisation of check m = i Z + r (block row i; member q is bit
// q Z + ((r + js[q]) mod Z)): its two smallest |y| into chk (16-bit
// min1 | min2 << 8 for int8, 32-bit min1 | min2 << 16 for int16) and the
// position of the first into chkp, its term of eq. (1) pushed to the slots of
// its members (the first block row also adds -a_num |y_n|, once per bit);
// returns the check's syndrome bit.
template <int DT, int DC>
__device__ __forceinline__ uint32_t check_init(const FastArgs &a, int i, int imwbf, uint32_t r, const uint32_t (&js)[DC],
                                               const typename FT<DT>::Y *ys, const uint16_t *slotof,
                                               uint32_t *keys, uint32_t *chk, uint8_t *chkp)
{
    constexpr int QB = DC <= 2 ? 1 : DC <= 4 ? 2 : DC <= 8 ? 3 : DC <= 16 ? 4 : DC <= 32 ? 5 : 6;  // bits of q
    const uint32_t Z = a.Z;
    uint32_t av[DC], sl[DC];
    int yq[DC];
    uint32_t par = 0;
    // member q is bit q Z + ((r + js[q]) mod Z); its slot comes from the
    // doubled slot table without the reduction, and its received value from
    // the slot-ordered copy (every read of the check before its pushes)
#pragma unroll
    for (int q = 0; q < DC; q++) sl[q] = (slotof + 2 * q * Z)[r + js[q]];
#pragma unroll
    for (int q = 0; q < DC; q++) yq[q] = (int)ys[sl[q]];
    // the two smallest keys |y| << QB | q: their magnitudes are
    // min1 and min2 (with multiplicity), the first one's q is
    // the lowest position holding min1
    uint32_t k1 = 0xFFFFFFFFu, k2 = 0xFFFFFFFFu;
    if constexpr (DT == FWBF_I8 && DC == 6) {
        // int8 keys fit 16 bits (|y| <= 128): three pairs of
        // members in packed 16-bit lanes; per half the
        // smallest and second smallest of three, then the two
        // halves merged (second smallest of six = the smaller
        // of the larger first minimum and the smaller second
        // minimum)
        typedef short s16x2 __attribute__((ext_vector_type(2)));
        typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
        u16x2 P[3];
        uint32_t px = 0;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const s16x2 v = {(short)yq[2 * j], (short)yq[2 * j + 1]};
            px ^= __builtin_bit_cast(uint32_t, v);
            const s16x2 av2 = __builtin_elementwise_max(v, -v);
            const u16x2 qq = {(unsigned short)(2 * j), (unsigned short)(2 * j + 1)};
            P[j] = (__builtin_bit_cast(u16x2, av2) << (unsigned short)QB) | qq;
            av[2 * j] = (uint32_t)av2.x;
            av[2 * j + 1] = (uint32_t)av2.y;
        }
        const u16x2 A = __builtin_elementwise_min(P[0], P[1]), B = __builtin_elementwise_max(P[0], P[1]);
        const u16x2 S1 = __builtin_elementwise_min(A, P[2]);
        const u16x2 S2 = __builtin_elementwise_min(B, __builtin_elementwise_max(A, P[2]));
        k1 = min((uint32_t)S1.x, (uint32_t)S1.y);
        k2 = min(max((uint32_t)S1.x, (uint32_t)S1.y), min((uint32_t)S2.x, (uint32_t)S2.y));
        par = ((px >> 15) ^ (px >> 31)) & 1u;  // parity of the negative members
    } else {
        uint32_t sx = 0;
#pragma unroll
        for (int q = 0; q < DC; q++) {
            const int v = yq[q];
            const uint32_t av_ = (uint32_t)(v < 0 ? -v : v);
            av[q] = av_;
            sx ^= (uint32_t)v;  // bit 31: parity of the negative members
            const uint32_t key = (av_ << QB) | (uint32_t)q;
            k2 = min(k2, max(k1, key));
            k1 = min(k1, key);
        }
        par = sx >> 31;
    }
    const uint32_t m1 = k1 >> QB, pos = k1 & ((1u << QB) - 1);
    const uint32_t m2 = DC < 2 ? 0u : (k2 >> QB);
    const uint32_t m = i * Z + r;
    if constexpr (DT == FWBF_I8) {
        ((uint16_t *)chk)[m] = (uint16_t)(m1 | (m2 << 8));
        chkp[m] = (uint8_t)(pos | (par << 7));
    } else {
        chk[m] = m1 | (m2 << 16);
        chkp[m] = (uint8_t)(pos | (par << 7));
    }
    // push this check's term of eq. (1) to its members: the
    // two signed values (a_den w << idxb) are formed once
    // (minima are at most 32768: 16 bits)
    const uint32_t e1 = mul24(a.kden, m1 & 0xFFFFu);
    const uint32_t e2 = imwbf ? mul24(a.kden, m2 & 0xFFFFu) : e1;
    const uint32_t d1 = par ? e1 : 0u - e1, d2 = par ? e2 : 0u - e2;
#pragma unroll
    for (int q = 0; q < DC; q++) {
        uint32_t d = pos == (uint32_t)q ? d2 : d1;
        if (i == 0) d += (uint32_t)__mul24((int)av[q], a.nknum);  // - a_num |y| << idxb
        atomicAdd(&keys[sl[q]], d);
    }
    return par;
}

// Round update of check t of the flipped bit nf: toggles the check's
// syndrome bit (an LDS xor returning the old word) and adds +-2 a_den w to
// the metrics of its members, the sign given by the new bit; returns the new
// bit (1: the check is now unsatisfied).
template <int DT, int DC>
__device__ __forceinline__ uint32_t toggle_check(const FastArgs &a, int imwbf, uint32_t nf, uint32_t t, const uint32_t *sh,
                                                 const uint16_t *slotof, const uint32_t *chk, uint8_t *chkp,
                                                 uint32_t *keys)
{
    const uint32_t Z = a.Z;
    const uint32_t j = mul24(nf, a.rZ24) >> 20;  // block column: nf / Z
    const uint32_t c = nf - mul24(j, Z);
    const uint32_t *st = sh + mul24(t, (uint32_t)a.nb);
    const uint32_t rr = submod(c, st[j], Z);
    const uint32_t m = mul24(t, Z) + rr;
    // the syndrome bit is bit 7 of the check's position byte: toggled with
    // an xor on its 32-bit word, which also returns the position
    const uint32_t sb = 8u * (m & 3u);
    const uint32_t ob = atomicXor(&((uint32_t *)chkp)[m >> 2], 0x80u << sb) >> sb;
    const uint32_t nb1 = ((ob >> 7) & 1u) ^ 1u;
    const uint32_t pos = ob & 7u;
    // the check's two weights
    uint32_t w1, w2;
    if constexpr (DT == FWBF_I8) {
        const uint32_t cw = ((const uint16_t *)chk)[m];
        w1 = cw & 0xFF; w2 = cw >> 8;
    } else {
        const uint32_t cw = chk[m];
        w1 = cw & 0xFFFF; w2 = cw >> 16;
    }
    const uint32_t e1 = mul24(a.kden2, w1);
    const uint32_t e2 = imwbf ? mul24(a.kden2, w2) : e1;
    const uint32_t d1 = nb1 ? e1 : 0u - e1, d2 = nb1 ? e2 : 0u - e2;
    // every member's slot first, then the adds
    uint32_t sl[DC];
#pragma unroll
    for (int q = 0; q < DC; q++) sl[q] = slotof[mul24((uint32_t)q, 2 * Z) + rr + st[q]];
#pragma unroll
    for (int q = 0; q < DC; q++) atomicAdd(&keys[sl[q]], pos == (uint32_t)q ? d2 : d1);
    return nb1;
}

// The same update split over a pair of lanes (u = 0, 1), each taking half
// of the check's members (q = u DC/2 .. u DC/2 + DC/2 - 1); the even lane
// toggles the syndrome bit and its partner takes the new bit from it (DPP
// within the quad). sbq[k] = slotof + 2 q Z + s_{t,q} for this lane's
// members q = u DC/2 + k (fixed per lane): the slot of member q of check
// t Z + rr is sbq[k][rr] in the doubled slot table (below). Returns the new bit on the even lane, 0 on the
// odd one.
template <int DT, int DC>
__device__ __forceinline__ uint32_t toggle_half(const FastArgs &a, int imwbf, uint32_t nf, uint32_t t, uint32_t u,
                                                const uint16_t *const (&sbq)[DC / 2],
                                                const uint32_t *sh, const uint32_t *chk, uint8_t *chkp,
                                                uint32_t *keys)
{
    constexpr int H = DC / 2;
    const uint32_t Z = a.Z;
    const uint32_t j = mul24(nf, a.rZ24) >> 20;  // block column: nf / Z
    const uint32_t c = nf - mul24(j, Z);
    const uint32_t rr = submod(c, sh[mul24(t, (uint32_t)a.nb) + j], Z);
    const uint32_t m = mul24(t, Z) + rr;
    // syndrome bit 7 of the position byte; the odd lane xors 0 and only
    // takes the (unchanged) position from the word it reads
    const uint32_t sb = 8u * (m & 3u);
    const uint32_t ob = atomicXor(&((uint32_t *)chkp)[m >> 2], u == 0 ? 0x80u << sb : 0u) >> sb;
    const uint32_t nb1 = dpp<0xA0>(((ob >> 7) & 1u) ^ 1u);  // quad_perm [0,0,2,2]: the even lane's bit
    const uint32_t pos = ob & 7u;
    uint32_t w1, w2;
    if constexpr (DT == FWBF_I8) {
        const uint32_t cw = ((const uint16_t *)chk)[m];
        w1 = cw & 0xFF; w2 = cw >> 8;
    } else {
        const uint32_t cw = chk[m];
        w1 = cw & 0xFFFF; w2 = cw >> 16;
    }
    const uint32_t e1 = mul24(a.kden2, w1);
    const uint32_t e2 = imwbf ? mul24(a.kden2, w2) : e1;
    const uint32_t d1 = nb1 ? e1 : 0u - e1, d2 = nb1 ? e2 : 0u - e2;
    const uint32_t pk = pos - u * (uint32_t)H;  // the minimum's index among this lane's members
    uint32_t sl[H];
#pragma unroll
    for (int k = 0; k < H; k++) sl[k] = sbq[k][rr];
#pragma unroll
    for (int k = 0; k < H; k++) atomicAdd(&keys[sl[k]], pk == (uint32_t)k ? d2 : d1);
    return u == 0 ? nb1 : 0u;
}

template <int DT, int DV, int DC, int C>
__global__ __launch_bounds__(64 * FAST_WAVES) __attribute__((amdgpu_waves_per_eu(5))) void fast_kernel(FastArgs a)
{
    using Y = typename FT<DT>::Y;
    extern __shared__ __align__(16) unsigned char smem[];
    // the wavefront index is uniform across the wavefront: in a scalar
    // register, so LDS base addresses derived from it are scalar too
    const uint32_t lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned char *wbase = smem + a.o_wave0 + wv * a.wave_bytes;
    uint32_t *keys = (uint32_t *)wbase;
    uint32_t *chk = (uint32_t *)(wbase + a.o_chk);
    uint8_t *chkp = wbase + a.o_chkp;
    Y *yv = (Y *)(wbase + a.o_y);
    uint32_t *zw = (uint32_t *)(wbase + a.o_z);
    uint32_t *flips = (uint32_t *)(wbase + a.o_y);  // the rounds' winners (over the received values)
    uint32_t *sh = (uint32_t *)(smem + a.o_sh);
    uint16_t *slotof = (uint16_t *)(smem + a.o_slot);  // slot word of every bit, doubled (frame-independent)

    const uint32_t Z = a.Z;
    const int N = a.N, M = a.M;
    for (int t = threadIdx.x; t < DV * a.nb; t += 64 * FAST_WAVES) sh[t] = a.shift[t];
    // the slot of every bit, each block column stored twice in a row
    // (entry q 2Z + x holds bit q Z + (x mod Z)), so that the member of a
    // check at rotation r + s (r, s < Z) needs no reduction mod Z
    for (int e = threadIdx.x; e < 2 * a.N; e += 64 * FAST_WAVES) {
        const uint32_t q = (uint32_t)e / (2 * Z);  // once per workgroup: a plain division
        const uint32_t x = (uint32_t)e - 2 * q * Z;
        const uint32_t n = q * Z + (x < Z ? x : x - Z);
        uint32_t gg, pp;
        if (a.strided) { pp = fdiv(n, a.magG, a.maskG); gg = n - pp * a.Geff; }
        else { gg = fdiv(n, a.magP, a.maskP); pp = n - gg * a.p; }
        slotof[e] = (uint16_t)slot_addr(gg * a.L + pp / C, pp & (C - 1));
    }
    __syncthreads();  // the only workgroup barrier: the wavefronts run independently from here

    // lane -> block layout
    const uint32_t g = lane >> a.logL;
    const bool lead = ((lane & (a.L - 1)) == 0) && (int)g < a.Geff;
    const uint32_t pos0 = (lane & (a.L - 1)) * C;
    const uint32_t gp = g * a.p;
    const int NW = (N + 31) >> 5;
    // this lane's slots that hold a bit are its first nreal (positions pos0,
    // pos0 + 1, ...), and the initial key of position pos0 + j is key0 - j:
    // the bias (metric 0) above the reversed position (bias << idxb | idxmask - pos)
    int nreal = 0;
    if ((int)g < a.Geff) {
        const int lim = min(a.p, a.strided ? (N - (int)g + a.Geff - 1) / a.Geff : N - (int)gp);
        nreal = max(0, min(C, lim - (int)pos0));
    }
    const uint32_t key0 = (a.bias << a.idxb) | (a.idxmask - pos0);
    // the bit of this lane's slot j is ybase + j ystep (lanes without a block
    // read from 0: their slots hold no bit)
    const uint32_t ystep = a.strided ? (uint32_t)a.Geff : 1u;
    const uint32_t ybase = (int)g < a.Geff ? (a.strided ? mul24(pos0, (uint32_t)a.Geff) + g : gp + pos0) : 0u;
    // blocks of at least 2 dv lanes: lanes 2t, 2t + 1 (t < dv) of a block
    // share check t of the block's winner, half of its members each
    const uint32_t tl = lane & (uint32_t)(a.L - 1), tt = tl >> 1, tu = tl & 1;
    const uint16_t *sbq[DC / 2];
#pragma unroll
    for (int k = 0; k < DC / 2; k++) {
        const uint32_t q = tu * (DC / 2) + k;
        sbq[k] = slotof + 2 * q * Z + (tt < (uint32_t)DV ? sh[tt * a.nb + q] : 0u);
    }

    const FrameRange fr = xcd_frames_waves(a.F, FAST_WAVES, (int)wv);
    for (int64_t f = fr.first; f < fr.end; f += fr.step) {
        const uint8_t *skip = a.skip;
        asm volatile("" : "+s"(skip));
        if (skip && skip[f]) continue;  // uniform across the wave
        const Y *yrow = (const Y *)a.y + f * a.stride;
        wave_sync();
        for (int w = lane; w < ((N + 63) >> 6) * 2; w += 64) zw[w] = 0;
        // ---- received values -> LDS ---------------------------------------
        constexpr int E = 16 / (int)sizeof(Y);  // values per 16-byte chunk
        const int nchunk = fresh(a.vec_ok) ? min(N / E, 128) : 0;
        uint32_t zmask[2] = {0, 0};
        for (int it = 0; it < 2; it++) {
            const int cidx = lane + 64 * it;
            if (cidx < nchunk) {
                const uint4 v = ((const uint4 *)yrow)[cidx];
                ((uint4 *)yv)[cidx] = v;
                // sign bits of the chunk (z_0 = [y < 0]), E bits
                uint32_t msk = 0;
                const uint32_t xs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    uint32_t nib;
                    if constexpr (sizeof(Y) == 1) nib = ((((xs[u] >> 7) & 0x01010101u) * 0x01020408u) >> 24) & 0xFu;
                    else nib = ((xs[u] >> 15) & 1u) | ((xs[u] >> 30) & 2u);
                    msk |= nib << (u * (sizeof(Y) == 1 ? 4 : 2));
                }
                zmask[it] = msk;
            }
        }
        for (int n = nchunk * E + lane; n < N; n += 64) yv[n] = yrow[n];
        // initial keys: bias (metric 0) packed with the position in the block
#pragma unroll
        for (int kk = 0; kk < C; kk += 4) {
            uint4 v;
            uint32_t *vp = (uint32_t *)&v;
#pragma unroll
            for (int u = 0; u < 4; u++) vp[u] = kk + u < nreal ? key0 - (uint32_t)(kk + u) : 0u;
            ((uint4 *)keys)[chunk_of(lane, kk >> 2)] = v;
        }
        wave_sync();
        // hard decisions z_0 = [y < 0] (Section III, Initialization)
        for (int it = 0; it < 2; it++) {
            const int cidx = lane + 64 * it;
            if (cidx < nchunk && zmask[it]) {
                const int b0 = cidx * E;
                atomicOr(&zw[b0 >> 5], zmask[it] << (b0 & 31));
            }
        }
        for (int n0 = nchunk * E; n0 < N; n0 += 64) {
            const int n = n0 + lane;
            const bool neg = n < N && yv[n] < (Y)0;
            if (neg) atomicOr(&zw[n >> 5], 1u << (n & 31));
        }
        // the received values in slot order, in place: the check phase reaches
        // a member through its slot (no reduction mod Z for the value). Every
        // lane reads the values of its C slots, then (the wavefront's LDS
        // operations complete in order) writes them at its slots; a padding
        // slot gets whatever follows its block (never read).
        {
            Y vals[C];
            if (fresh(a.strided)) {
#pragma unroll
                for (int j = 0; j < C; j++) vals[j] = yv[ybase + (uint32_t)j * ystep];
            } else {
#pragma unroll
                for (int j = 0; j < C; j++) vals[j] = yv[ybase + j];
            }
            wave_sync();
#pragma unroll
            for (int kk = 0; kk < C; kk += 4) {
                if constexpr (sizeof(Y) == 1) {
                    const uint32_t w = (uint32_t)(uint8_t)vals[kk] | ((uint32_t)(uint8_t)vals[kk + 1] << 8) |
                                       ((uint32_t)(uint8_t)vals[kk + 2] << 16) | ((uint32_t)(uint8_t)vals[kk + 3] << 24);
                    ((uint32_t *)yv)[chunk_of(lane, kk >> 2)] = w;
                } else {
                    const uint2 w = make_uint2((uint32_t)(uint16_t)vals[kk] | ((uint32_t)(uint16_t)vals[kk + 1] << 16),
                                               (uint32_t)(uint16_t)vals[kk + 2] | ((uint32_t)(uint16_t)vals[kk + 3] << 16));
                    ((uint2 *)yv)[chunk_of(lane, kk >> 2)] = w;
                }
            }
            wave_sync();
        }

        // ---- check minima, syndrome s_0 and check-side initial metrics ----
        int weight = 0;
        for (int i = 0; i < DV; i++) {
            uint32_t js[DC];
#pragma unroll
            for (int q = 0; q < DC; q++) js[q] = sh[i * a.nb + q];
            for (uint32_t r0 = 0; r0 < Z; r0 += 64) {
                const int imwbf = fresh(a.imwbf);
                // the addresses of this pass are the lane offset plus scalar
                // sums (an opaque r0 keeps them from becoming per-member
                // induction registers)
                const uint32_t r = (uint32_t)fresh((int)r0) + lane;
                const bool valid = r < Z;
                const uint32_t par = valid ? check_init<DT, DC>(a, i, imwbf, r, js, yv, slotof, keys, chk, chkp) : 0u;
                const unsigned long long b = __ballot(valid && par);
                weight += __popcll(b);
            }
        }
        wave_sync();

        int k = 0, okf = 0;
        uint32_t prv = NONE;
        if (weight == 0 || a.max_iter == 0) {
            okf = weight == 0;
        } else {
            for (;;) {
                // this round's copies of the launch's switches
                const int Lr = fresh(a.L), single = fresh(a.single), strided = fresh(a.strided);
                const int imwbf = fresh(a.imwbf), cycle_exit = fresh(a.cycle_exit), exec_rounds = fresh(a.exec_rounds);
                // ---- Step 2: block maxima ----------------------------------
                // every chunk read is issued before any is compared
                uint4 kv[C / 4];
#pragma unroll
                for (int kk = 0; kk < C; kk += 4) kv[kk >> 2] = ((const uint4 *)keys)[chunk_of(lane, kk >> 2)];
                uint32_t best = 0;
#pragma unroll
                for (int kk = 0; kk < C / 4; kk++) best = max(best, max(max(kv[kk].x, kv[kk].y), max(kv[kk].z, kv[kk].w)));
                best = group_max(best, Lr);
                const uint32_t val = best >> a.idxb;
                const uint32_t bp = a.idxmask - (best & a.idxmask);
                const uint32_t n = strided ? mul24(bp, (uint32_t)a.Geff) + g : gp + bp;
                const bool flip = lead && (single || val > a.zero_val);
                const uint32_t cur = flip ? n : NONE;
                const unsigned long long fmask = __ballot(flip);
                const unsigned long long dmask = __ballot(lead && cur != prv);
                prv = lead ? cur : prv;
                if (cycle_exit) {
                    if (fmask == 0) {  // no flip: fixed point until K_max
                        k = exec_rounds ? k : a.max_iter;
                        break;
                    }
                    if (dmask == 0) {
                        // same flips as the round before: states alternate,
                        // z_{K_max} = z_k if K_max - k is even, else z_k ^ flips
                        if (((a.max_iter - k) & 1) && flip) atomicXor(&zw[n >> 5], 1u << (n & 31));
                        k = exec_rounds ? k : a.max_iter;
                        break;
                    }
                }
                // ---- flip, toggle the syndrome, update the member metrics --
                // the winners flip their bits; one lane per (winner, check)
                // pair toggles the check and adds +-2 a_den w to the metrics
                // of the check's members, the sign given by the check's new
                // bit (two winners toggling one check are serialised by the
                // atomics: their changes cancel exactly)
                const int nflip = __popcll(fmask);
                int sum_ones = 0;  // toggles that leave their check unsatisfied
                if (Lr >= 2 * DV) {
                    // lanes 2t, 2t + 1 of the block share check t of its
                    // winner (three members each), the lead lane flips the bit
                    if (flip) atomicXor(&zw[n >> 5], 1u << (n & 31));
                    const bool tog = tt < (uint32_t)DV && (int)g < a.Geff && (single || val > a.zero_val);
                    uint32_t nb1 = 0;
                    if (tog) nb1 = toggle_half<DT, DC>(a, imwbf, n, tt, tu, sbq, sh, chk, chkp, keys);
                    sum_ones = __popcll(__ballot(nb1));
                } else if (Lr >= DV) {
                    // every lane of a block holds the block's winner after the
                    // butterfly: lane t < DV of the block takes check t, and
                    // the lead lane flips the bit
                    if (flip) atomicXor(&zw[n >> 5], 1u << (n & 31));
                    const uint32_t t = lane & (uint32_t)(Lr - 1);
                    const bool tog = t < (uint32_t)DV && (int)g < a.Geff && (single || val > a.zero_val);
                    uint32_t nb1 = 0;
                    if (tog) nb1 = toggle_check<DT, DC>(a, imwbf, n, t, sh, slotof, chk, chkp, keys);
                    sum_ones = __popcll(__ballot(nb1));
                } else {
                    // fewer lanes than checks per block: the winners are
                    // listed and one lane per (winner, check) pair takes it
                    const int rank = __popcll(fmask & ((1ull << lane) - 1));
                    if (flip) {
                        atomicXor(&zw[n >> 5], 1u << (n & 31));
                        flips[rank] = n;
                    }
                    wave_sync();
                    const int ntog = nflip * DV;
                    constexpr uint32_t DVM = ((1u << 16) + DV - 1) / DV;  // i / DV = (i * DVM) >> 16 for i < 2^12
                    for (int base = 0; base < ntog; base += 64) {
                        const int i = base + (int)lane;
                        uint32_t nb1 = 0;
                        if (i < ntog) {
                            const uint32_t u = mul24((uint32_t)i, DVM) >> 16;
                            const uint32_t t = (uint32_t)i - mul24(u, (uint32_t)DV);
                            nb1 = toggle_check<DT, DC>(a, imwbf, flips[u], t, sh, slotof, chk, chkp, keys);
                        }
                        sum_ones += __popcll(__ballot(nb1));
                    }
                }
                weight += 2 * sum_ones - DV * nflip;
                k += 1;
                if (weight == 0) { okf = 1; break; }
                if (k == a.max_iter) break;
                wave_sync();
            }
        }
        wave_sync();
        uint32_t *zo = a.z + f * NW;
        for (int w = lane; w < NW; w += 64) zo[w] = zw[w];
        if (lane == 0) {
            a.iters[f] = fresh(a.iters_add) ? a.iters[f] + k : k;
            a.ok[f] = (uint8_t)okf;
        }
    }
}


}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

int ilog2c(uint32_t v) { int r = 0; while ((1u << r) < v) r++; return r; }

void magic_c(uint32_t d, uint32_t *mag, uint32_t *mask)
{
    if (d <= 1) { *mag = 0; *mask = 0xFFFFFFFFu; return; }
    *mag = (uint32_t)(((1ULL << 32) + d - 1) / d);
    *mask = 0;
}

template <int DT, int DV, int DC, int C>
hipError_t launch_fast(const FastArgs &a, hipStream_t st, int *grid_out, bool query)
{
    auto kern = fast_kernel<DT, DV, DC, C>;
    if (a.lds_bytes > 65536)
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes);
    int blocks = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, 64 * FAST_WAVES, a.lds_bytes);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (blocks < 1) return hipErrorInvalidConfiguration;
    const int64_t grid = std::min<int64_t>((a.F + FAST_WAVES - 1) / FAST_WAVES, (int64_t)blocks * cus);
    *grid_out = (int)grid;
    if (query) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3((int)grid), dim3(64 * FAST_WAVES), a.lds_bytes, st, a);
    return hipGetLastError();
}

template <int DT, int DV, int DC>
hipError_t by_c(int C, const FastArgs &a, hipStream_t st, int *grid, bool query)
{
    switch (C) {
    case 4: return launch_fast<DT, DV, DC, 4>(a, st, grid, query);
    case 8: return launch_fast<DT, DV, DC, 8>(a, st, grid, query);
    case 16: return launch_fast<DT, DV, DC, 16>(a, st, grid, query);
    case 32: return launch_fast<DT, DV, DC, 32>(a, st, grid, query);
    case 64: return launch_fast<DT, DV, DC, 64>(a, st, grid, query);
    }
    return hipErrorInvalidValue;
}

template <int DT>
hipError_t by_deg(int dv, int dc, int C, const FastArgs &a, hipStream_t st, int *grid, bool query)
{
    if (dv == 3 && dc == 6) return by_c<DT, 3, 6>(C, a, st, grid, query);
    return hipErrorInvalidValue;
}

}  // namespace

// Returns 1 if the fast kernel was launched, 0 if the configuration is not
// covered (the caller then uses the generic kernel), < 0 on error.
int try_fast_decode(const fwbf_code *c, const fwbf_params *p, const void *y, int64_t F, int64_t stride,
                    uint32_t *z, int32_t *iters, uint8_t *ok, hipStream_t st, const uint32_t *shift_dev,
                    const uint8_t *skip, int iters_add)
{
    if (p->dtype != FWBF_I8 && p->dtype != FWBF_I16) return 0;
    if (p->select == FWBF_TOPL) return 0;
    if (p->threads_per_frame != 0 && p->threads_per_frame != 64) return 0;
    const int dv = c->mb, dc = c->nb;
    if (c->multi || !(dv == 3 && dc == 6)) return 0;
    for (int v : c->shift)
        if (v < 0) return 0;
    FastArgs a;
    memset(&a, 0, sizeof a);
    const int G = (p->select == FWBF_GROUPS || p->select == FWBF_STRIDED) ? p->groups : 1;
    a.p = (c->N + G - 1) / G;
    a.strided = p->select == FWBF_STRIDED;
    a.Geff = a.strided ? G : (c->N + a.p - 1) / a.p;
    // smallest C with Geff * L <= 64 lanes, L = 2^ceil(log2(ceil(p / C)))
    int C = 0, L = 0;
    for (int cc : {4, 8, 16, 32, 64}) {
        const int l = 1 << ilog2c((a.p + cc - 1) / cc);
        if ((int64_t)a.Geff * l <= 64) { C = cc; L = l; break; }
    }
    if (!C) return 0;
    a.L = L;
    a.logL = ilog2c(L);
    a.Lc = L * C;
    a.N = c->N; a.M = c->M; a.Z = c->Z; a.nb = c->nb;
    // a 24-bit reciprocal of Z that divides every bit index exactly (always
    // so for the codes taken here: Z <= 341); otherwise the general kernel
    // (exact for every n < N when (N - 1) (rZ24 Z - 2^20) < 2^20: the error
    // n (rZ24 Z - 2^20) / (Z 2^20) then stays below 1 / Z)
    a.rZ24 = (uint32_t)(((1u << 20) + c->Z - 1) / c->Z);
    if ((uint64_t)(c->N - 1) * ((uint64_t)a.rZ24 * c->Z - (1u << 20)) >= (1u << 20) ||
        (uint64_t)c->N * a.rZ24 >= (1ull << 32))
        return 0;
    magic_c(a.p, &a.magP, &a.maskP);
    magic_c(a.Geff, &a.magG, &a.maskG);
    a.single = p->select == FWBF_SINGLE;
    a.imwbf = p->weights == FWBF_IMWBF;
    a.max_iter = p->max_iter;
    a.cycle_exit = !(p->flags & FWBF_FLAG_NO_CYCLE_EXIT);
    a.exec_rounds = (p->flags & FWBF_FLAG_EXECUTED_ROUNDS) != 0;
    a.aden = p->alpha_den;
    a.anum = p->weights == FWBF_WBF ? 0 : p->alpha_num;
    const int64_t maxmag = p->dtype == FWBF_I8 ? 128 : 32768;
    const int64_t maxE = maxmag * ((int64_t)a.aden * dv + a.anum);
    int vb = 1;
    while ((1LL << (vb - 1)) <= maxE) vb++;
    a.bias = 1u << (vb - 1);
    a.zero_val = a.bias;
    a.idxb = ilog2c((uint32_t)a.Lc);
    if (vb + a.idxb > 32) return 0;
    a.idxmask = a.idxb ? (1u << a.idxb) - 1 : 0;
    if (((int64_t)2 * a.aden << a.idxb) >= (1 << 24) || ((int64_t)a.anum << a.idxb) >= (1 << 23)) return 0;
    a.kden = (uint32_t)a.aden << a.idxb;
    a.kden2 = 2u * (uint32_t)a.aden << a.idxb;
    a.nknum = -(a.anum << a.idxb);
    const int esz = p->dtype == FWBF_I8 ? 1 : 2;
    a.vec_ok = (((uintptr_t)y & 15) == 0) && ((stride * esz) % 16 == 0);
    // LDS layout
    int off = 0;
    auto take = [&](int bytes, int align) { off = (off + align - 1) / align * align; int o = off; off += bytes; return o; };
    a.o_sh = take(4 * dv * c->nb, 4);
    a.o_slot = take(2 * 2 * c->N, 4);
    a.o_wave0 = (off + 15) / 16 * 16;
    off = 64 * C * 4;  // keys, then the rest of one wavefront's frame state
    a.o_chk = take((p->dtype == FWBF_I16 ? 4 : 2) * c->M, 4);  // min1 | min2 << 16 (int16), << 8 (int8)
    a.o_chkp = take((c->M + 3) / 4 * 4, 4);  // position of min1 | syndrome bit << 7 (whole words: atomics)
    // the received values, needed only while initialising; in the rounds the
    // same bytes hold the flipped bits (Geff words)
    // received values: bit order while loading, then slot order (64 C slots;
    // a lane's reads run up to N + L C in bit order)
    a.o_y = take(std::max({esz * ((c->N + 15) / 16 * 16), esz * (c->N + a.L * C), esz * 64 * C, 4 * a.Geff}), 16);
    a.o_z = take(((c->N + 63) / 64) * 8, 8);
    a.wave_bytes = (off + 15) / 16 * 16;
    a.lds_bytes = a.o_wave0 + FAST_WAVES * a.wave_bytes;
    if (a.lds_bytes > 160 * 1024) return 0;
    a.y = y; a.F = F; a.stride = stride;
    a.z = z; a.iters = iters; a.ok = ok;
    a.shift = shift_dev;
    a.skip = skip;
    a.iters_add = iters_add;
    int grid = 0;
    hipError_t e = p->dtype == FWBF_I8 ? by_deg<FWBF_I8>(dv, dc, C, a, st, &grid, false)
                                       : by_deg<FWBF_I16>(dv, dc, C, a, st, &grid, false);
    if (e != hipSuccess) return hip_fail(e, "fast decode kernel launch");
    return 1;
}

}  // namespace fwbf
