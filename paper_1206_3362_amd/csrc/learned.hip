// Learned flip scorer for FWBF: a per-round metric E_t = beta_t S - alpha_t |y|
// proposes the k best bits of each block (the paper's partially parallel
// choice, Section III), and a 4 -> 32 -> 32 -> 1 ReLU network scores the
// proposals; in each block the best-scoring proposal is flipped if its score
// is positive.  Frames whose syndrome is still nonzero after the learned pass
// are decoded again from the original y by plain FWBF (the fast kernel with
// a skip list).  Training kernels (forward, backward, deterministic
// reduction, Adam) run on records the learned pass emits.
//
// The network runs on MFMA v_mfma_f32_32x32x8_bf16 in transposed form: a
// tile holds 32 candidates, activations are (hidden x candidate) with the
// candidate on lane % 32, so the accumulator of one layer is already laid out
// as the B operand of the next (items 4c..4c+3 of lane l hold rows
// 8c + 4(l/32) + 0..3 of column l % 32), and the weights are per-lane
// constant A operands.  Operands are bfloat16 (round to nearest even), sums
// single precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "frames.h"
#include "internal.h"

namespace fwbf {

int try_fast_decode(const fwbf_code *c, const fwbf_params *p, const void *y, int64_t F, int64_t stride,
                    uint32_t *z, int32_t *iters, uint8_t *ok, hipStream_t st, const uint32_t *shift_dev,
                    const uint8_t *skip, int iters_add);
int decode_general(const fwbf_code *code, const fwbf_params *params, const void *y_dev, int64_t F, int64_t y_stride,
                   uint32_t *z_dev, int32_t *iters_dev, uint8_t *ok_dev, hipStream_t stream, const uint8_t *skip);

namespace {

constexpr int H = 32;
constexpr uint32_t NONE = 0xFFFFFFFFu;
// slot word of a bit: S << 16 (S signed, |S| <= dv * 128) + |y| << 8 + u (u <= dv);
// adds to S and u never carry or borrow across the fields

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8h __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// parameter vector offsets (float32): W1[32][4] b1 W2[32][32] b2 W3 b3 alpha[T] beta[T]
constexpr int O_W1 = 0, O_B1 = 128, O_W2 = 160, O_B2 = 1184, O_W3 = 1216, O_B3 = 1248, O_AL = 1249;

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Four floats rounded to bfloat16 (to nearest, ties to even) and packed: two
// hardware pair conversions, which give bf16_rne's result for every float
// that is not a NaN (checked over all 2^32 bit patterns).
typedef __bf16 bf16x2h __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d)
{
    const f32x2 ab = {a, b}, cd = {c, d};
    const uint32_t lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(ab, bf16x2h));
    const uint32_t hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(cd, bf16x2h));
    return __builtin_bit_cast(bf16x4, ((uint64_t)hi << 32) | lo);
}

// row (hidden unit) held by accumulator item q of lane l
__device__ __forceinline__ int row_of(int q, int lane) { return 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3); }

struct Net {
    bf16x4 w1;      // W1[l%32][4(l/32) + 0..3] (zero for the upper half: only 4 inputs)
    bf16x4 w2[4];   // W2[l%32][8c + 4(l/32) + 0..3]
    float b1[16], b2[16], w3[16];
    float b3;
};

__device__ void load_net(Net &n, const float *p)
{
    const int l = threadIdx.x & 63, i = l & 31, hi = l >> 5;
    if (hi == 0) n.w1 = pack4(p[O_W1 + i * 4 + 0], p[O_W1 + i * 4 + 1], p[O_W1 + i * 4 + 2], p[O_W1 + i * 4 + 3]);
    else n.w1 = pack4(0.f, 0.f, 0.f, 0.f);
    for (int c = 0; c < 4; c++) {
        const float *r = p + O_W2 + i * H + 8 * c + 4 * hi;
        n.w2[c] = pack4(r[0], r[1], r[2], r[3]);
    }
    for (int q = 0; q < 16; q++) {
        const int row = row_of(q, l);
        n.b1[q] = p[O_B1 + row];
        n.b2[q] = p[O_B2 + row];
        n.w3[q] = p[O_W3 + row];
    }
    n.b3 = p[O_B3];
}

// decode-side network: everything in LDS (the MFMA weight operands per lane,
// biases and W3 per row), read at each scoring, to keep the kernel's register
// count low
struct NetL {
    const bf16x4 *wq;           // lane l: W1 operand at wq[5l], W2 operands at wq[5l + 1 + c]
    const float *b1, *b2, *w3;  // LDS copies
    float b3;
};

__device__ __forceinline__ float net_score(const NetL &n, bf16x4 x)
{
    const int l = threadIdx.x & 63;
    const bf16x4 *wl = n.wq + 5 * l;
    f32x16 acc = {};
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(wl[0], x, acc, 0, 0, 0);
    bf16x4 h1[4];
    for (int c = 0; c < 4; c++) {
        float h[4];
        for (int u = 0; u < 4; u++) h[u] = fmaxf(acc[4 * c + u] + n.b1[row_of(4 * c + u, l)], 0.0f);
        h1[c] = pack4(h[0], h[1], h[2], h[3]);
    }
    // layer 2 as two 16-deep products: the A and B operands of chunks 2c and
    // 2c + 1 side by side hold the same hidden units at the same (lane half,
    // element) positions, so each product sums over 16 of the 32 units
    f32x16 acc2 = {};
    for (int c = 0; c < 2; c++) {
        const bf16x8h a8 = __builtin_bit_cast(bf16x8h, __builtin_shufflevector(wl[1 + 2 * c], wl[2 + 2 * c], 0, 1, 2, 3, 4, 5, 6, 7));
        const bf16x8h b8 = __builtin_bit_cast(bf16x8h, __builtin_shufflevector(h1[2 * c], h1[2 * c + 1], 0, 1, 2, 3, 4, 5, 6, 7));
        acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, b8, acc2, 0, 0, 0);
    }
    float part = 0.0f;
    for (int q = 0; q < 16; q++) {
        const int row = row_of(q, l);
        part = __builtin_fmaf(n.w3[row], fmaxf(acc2[q] + n.b2[row], 0.0f), part);
    }
    return part + __shfl_xor(part, 32, 64) + n.b3;
}

struct Act {
    f32x16 pre1, pre2;
    bf16x4 h1[4];
};

// Scores the 32 candidates of a tile.  x: the four features of candidate
// l % 32 in lanes 0..31 (rounded to bfloat16), zero in lanes 32..63.
// Returns the score of candidate l % 32 (in both halves of the wave).
__device__ __forceinline__ float net_forward(const Net &n, bf16x4 x, Act &a)
{
    const int l = threadIdx.x & 63;
    f32x16 acc = {};
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(n.w1, x, acc, 0, 0, 0);
    float h[16];
    for (int q = 0; q < 16; q++) {
        a.pre1[q] = acc[q] + n.b1[q];
        h[q] = fmaxf(a.pre1[q], 0.0f);
    }
    for (int c = 0; c < 4; c++) a.h1[c] = pack4(h[4 * c], h[4 * c + 1], h[4 * c + 2], h[4 * c + 3]);
    f32x16 acc2 = {};
    for (int c = 0; c < 4; c++) acc2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(n.w2[c], a.h1[c], acc2, 0, 0, 0);
    float part = 0.0f;
    for (int q = 0; q < 16; q++) {
        a.pre2[q] = acc2[q] + n.b2[q];
        part = __builtin_fmaf(n.w3[q], fmaxf(a.pre2[q], 0.0f), part);
    }
    (void)l;
    return part + __shfl_xor(part, 32, 64) + n.b3;
}

__device__ __forceinline__ uint32_t orderable(float e)
{
    uint32_t u = __float_as_uint(e == 0.0f ? 0.0f : e);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t mag, uint32_t mask) { return __umulhi(n, mag) + (n & mask); }
__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t Z) { const uint32_t s = a + b; return min(s, s - Z); }
__device__ __forceinline__ uint32_t submod(uint32_t a, uint32_t b, uint32_t Z) { const uint32_t s = a - b; return min(s, s + Z); }

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) { return a > b ? a : b; }
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v)
{
    return ((unsigned long long)dpp<CTRL>((uint32_t)(v >> 32)) << 32) | dpp<CTRL>((uint32_t)v);
}
// maximum over aligned groups of L lanes, L a power of two <= 64
__device__ __forceinline__ unsigned long long group_max64(unsigned long long v, int L)
{
    if (L > 1) v = umax64(v, dpp64<0xB1>(v));
    if (L > 2) v = umax64(v, dpp64<0x4E>(v));
    if (L > 4) v = umax64(v, dpp64<0x141>(v));
    if (L > 8) v = umax64(v, dpp64<0x140>(v));
    for (int d = 16; d < L; d <<= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, d, 64), hi = __shfl_xor((uint32_t)(v >> 32), d, 64);
        v = umax64(v, ((unsigned long long)hi << 32) | lo);
    }
    return v;
}

struct LearnArgs {
    const int8_t *y;
    int64_t F, stride;
    uint32_t *z;
    int32_t *iters;
    uint8_t *ok;
    uint8_t *learned_ok;  // optional
    fwbf_record *rec;     // optional [F][T][32] (one tile per round)
    const uint32_t *pool; // labels for records (pool row f % pool_n, NULL: all-zero)
    int64_t pool_n, f0;
    const float *params;
    const uint32_t *shift;
    int N, M, Z, nb;
    uint32_t rZ24, magP, maskP;  // n / Z = (n * rZ24) >> 22 for every bit n
    int p, L, logL, Geff, k, T;
    int vec_ok;  // y and its row stride allow 16-byte loads
    float A, dv;
    float invA;   // 1/A when A is a power of two (then x * invA == x / A), else 0
    // LDS: tables shared by the workgroup (o_sh, o_slot, o_net, o_netw), then one
    // region of wave_bytes per wavefront (offsets relative to it; slots at 0)
    int o_chk, o_y, o_z, o_list, o_sh, o_cand, o_slot, o_net, o_netw, o_wave0, wave_bytes, lds_bytes;
};

// independent wavefronts (frames) per workgroup; the tables (shifts, slot
// of every bit, scorer biases) are stored once per workgroup.  The kernel is
// compiled for four wavefronts per SIMD (128 VGPRs, a few spilled), which
// measured faster than three without spills.
constexpr int LEARN_WAVES = 4;

// barrier of the one wavefront that owns a frame (its LDS operations
// complete in issue order; the fences keep the compiler from moving memory
// operations across this point)
__device__ __forceinline__ void lwave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t slot_chunk(uint32_t lane, uint32_t kk) { return (kk << 6) + (lane ^ ((kk & 15) << 2)); }
__device__ __forceinline__ uint32_t slot_word(uint32_t lane, uint32_t k) { return slot_chunk(lane, k >> 2) * 4 + (k & 3); }

template <int DV, int DC, int C>
__global__ __launch_bounds__(64 * LEARN_WAVES) __attribute__((amdgpu_waves_per_eu(4))) void learned_kernel(LearnArgs a)
{
    static_assert(DC <= 8, "check positions are packed in 3 bits");
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned char *wbase = smem + a.o_wave0 + wv * a.wave_bytes;
    uint32_t *slots = (uint32_t *)wbase;  // slot words
    uint32_t *chk = (uint32_t *)(wbase + a.o_chk);
    int8_t *yv = (int8_t *)(wbase + a.o_y);
    uint32_t *zw = (uint32_t *)(wbase + a.o_z);
    uint32_t *list = (uint32_t *)(wbase + a.o_list);  // the bits flipped in a round
    uint4 *cand = (uint4 *)(wbase + a.o_cand);  // 32 proposals: n, slot word
    uint32_t *sh = (uint32_t *)(smem + a.o_sh);
    uint16_t *slotof = (uint16_t *)(smem + a.o_slot);  // slot word of every bit (each block column twice)
    float *nbias = (float *)(smem + a.o_net);               // b1[32], b2[32], W3[32]
    bf16x4 *nw = (bf16x4 *)(smem + a.o_netw);               // MFMA weight operands, 5 per lane

    const uint32_t Z = a.Z;
    const int N = a.N, M = a.M;
    for (int t = threadIdx.x; t < DV * a.nb; t += 64 * LEARN_WAVES) sh[t] = a.shift[t];
    // entry q 2Z + x holds the slot of bit q Z + (x mod Z): a check member at
    // rotation r + s (r, s < Z) needs no reduction mod Z
    for (int e = threadIdx.x; e < 2 * a.N; e += 64 * LEARN_WAVES) {
        const uint32_t q = (uint32_t)e / (2 * Z);  // once per workgroup: a plain division
        const uint32_t x = (uint32_t)e - 2 * q * Z;
        const uint32_t n = q * Z + (x < Z ? x : x - Z);
        const uint32_t gg = fdiv(n, a.magP, a.maskP);
        const uint32_t pp = n - gg * a.p;
        slotof[e] = (uint16_t)slot_word(gg * a.L + pp / C, pp & (C - 1));
    }
    for (int t = threadIdx.x; t < 32; t += 64 * LEARN_WAVES) {
        nbias[t] = a.params[O_B1 + t];
        nbias[32 + t] = a.params[O_B2 + t];
        nbias[64 + t] = a.params[O_W3 + t];
    }
    // the round feature t / T for every round (divided once here)
    for (int t = threadIdx.x; t < a.T; t += 64 * LEARN_WAVES) nbias[96 + t] = (float)t / (float)a.T;
    if (threadIdx.x < 64) {
        // MFMA operands of lane l: W1[l%32][4(l/32) + 0..3] (zero for the
        // upper half: only 4 inputs), W2[l%32][8c + 4(l/32) + 0..3]
        const int i = lane & 31, hi = lane >> 5;
        const float *p = a.params;
        nw[5 * lane] = hi == 0 ? pack4(p[O_W1 + i * 4 + 0], p[O_W1 + i * 4 + 1], p[O_W1 + i * 4 + 2], p[O_W1 + i * 4 + 3])
                               : pack4(0.f, 0.f, 0.f, 0.f);
        for (int c = 0; c < 4; c++) {
            const float *r = p + O_W2 + i * H + 8 * c + 4 * hi;
            nw[5 * lane + 1 + c] = pack4(r[0], r[1], r[2], r[3]);
        }
    }
    __syncthreads();  // the only workgroup barrier: the wavefronts run independently from here
    NetL net;
    {
        const float *p = a.params;
        net.wq = nw;
        net.b1 = nbias;
        net.b2 = nbias + 32;
        net.w3 = nbias + 64;
        net.b3 = p[O_B3];
    }

    const float qu1 = 1.0f / a.dv, qu2 = 2.0f / a.dv, qu3 = 3.0f / a.dv;  // u / dv feature values
    const uint32_t g = lane >> a.logL;
    const bool lead = ((lane & (a.L - 1)) == 0) && (int)g < a.Geff;
    const uint32_t pos0 = (lane & (a.L - 1)) * C;
    const uint32_t gp = g * a.p;
    const int NW = (N + 31) >> 5;
    const int NC = a.Geff * a.k;  // proposals per round (<= 32)

    const FrameRange fr = xcd_frames_waves(a.F, LEARN_WAVES, (int)wv);
    // the 16-byte pieces of a frame (up to two per lane; every lane loads,
    // idle lanes a copy of the last piece, so the loads need no lane mask)
    auto fetch = [&](int64_t ff, uint4 *x) {
        const int nchunk = fresh(a.vec_ok) ? min(N >> 4, 128) : 0;
        if (nchunk == 0) return;
        const uint4 *src = (const uint4 *)(a.y + ff * a.stride);
        x[0] = src[min((int)lane, nchunk - 1)];
        if (nchunk > 64) x[1] = src[min((int)lane + 64, nchunk - 1)];
    };
    // the next frame's pieces are loaded while the current frame decodes
    uint4 nxt[2] = {make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0)};
    if (fr.first < fr.end) fetch(fr.first, nxt);
    for (int64_t f = fr.first; f < fr.end; f += fr.step) {
        const int nchunk = fresh(a.vec_ok) ? min(N >> 4, 128) : 0;
        const int8_t *yrow = a.y + f * a.stride;
        const uint4 vc[2] = {nxt[0], nxt[1]};
        if (f + fr.step < fr.end) fetch(f + fr.step, nxt);
        lwave_sync();
        for (int w = lane; w < ((N + 63) >> 6) * 2; w += 64) zw[w] = 0;
        {
            // the frame's pieces to LDS; z_0 = [y < 0] from their sign bits
#pragma unroll
            for (int it = 0; it < 2; it++) {
                const int cidx = (int)lane + 64 * it;
                if (cidx < nchunk) {
                    ((uint4 *)yv)[cidx] = vc[it];
                    const uint32_t xs[4] = {vc[it].x, vc[it].y, vc[it].z, vc[it].w};
                    uint32_t msk = 0;
#pragma unroll
                    for (int u = 0; u < 4; u++)
                        msk |= (((((xs[u] >> 7) & 0x01010101u) * 0x01020408u) >> 24) & 0xFu) << (4 * u);
                    if (msk) atomicOr(&zw[cidx >> 1], msk << (16 * (cidx & 1)));
                }
            }
            for (int n = nchunk * 16 + (int)lane; n < N; n += 64) {
                const int8_t v = yrow[n];
                yv[n] = v;
                if (v < 0) atomicOr(&zw[n >> 5], 1u << (n & 31));
            }
        }
        lwave_sync();
        // slot words: S = 0, u = 0, |y| of the slot's bit and its sign (bit 7,
        // above u <= 3: the check phase reads a member's value from its slot
        // word, whose |y| and sign the pushes of other checks leave alone);
        // when every lane's slots are 16 aligned consecutive bits, |y| comes
        // from one 16-byte read per 16 slots
        const bool a16 = (C % 16 == 0) && (a.p % 16 == 0);
        uint64_t realm = 0;
        uint4 y16 = make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int kk = 0; kk < C; kk += 4) {
            if (a16 && (kk & 15) == 0) {
                const uint32_t n0 = gp + pos0 + kk;
                y16 = (int)g < a.Geff && (int)n0 < N ? ((const uint4 *)yv)[n0 >> 4] : make_uint4(0, 0, 0, 0);
            }
            const uint32_t yw = ((kk & 15) >> 2) == 0 ? y16.x : ((kk & 15) >> 2) == 1 ? y16.y
                              : ((kk & 15) >> 2) == 2 ? y16.z : y16.w;
            uint4 v;
            uint32_t *vp = (uint32_t *)&v;
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t pos = pos0 + kk + u;
                const uint32_t n = gp + pos;
                const bool real = (int)g < a.Geff && (int)pos < a.p && (int)n < N;
                int yn = a16 ? (int)(int8_t)(yw >> (8 * u)) : (real ? (int)yv[n] : 0);
                yn = real ? yn : 0;
                vp[u] = ((uint32_t)(yn < 0 ? -yn : yn) << 8) | ((uint32_t)(yn < 0) << 7);
                realm |= (uint64_t)real << (kk + u);
            }
            ((uint4 *)slots)[slot_chunk(lane, kk >> 2)] = v;
        }
        lwave_sync();
        // check minima, syndrome, initial S and u pushed from the check side
        int weight = 0;
        for (int i = 0; i < DV; i++) {
            uint32_t js[DC];
#pragma unroll
            for (int q = 0; q < DC; q++) js[q] = sh[i * a.nb + q];
            for (uint32_t r0 = 0; r0 < Z; r0 += 64) {
                // an opaque r0: the pass's addresses are the lane offset plus
                // scalar sums, not one induction register per member
                const uint32_t r = (uint32_t)fresh((int)r0) + lane;
                const bool valid = r < Z;
                uint32_t par = 0;
                if (valid) {
                    // the two smallest keys |y| << 3 | q (q < 8): min1, min2 (with
                    // multiplicity) and the lowest position holding min1.
                    // Member q's slot comes from the doubled slot table (no
                    // reduction mod Z) and its |y| and sign from its slot word
                    // (every LDS read of the check is issued before its pushes)
                    uint32_t sl[DC], wq[DC];
#pragma unroll
                    for (int q = 0; q < DC; q++) sl[q] = (slotof + 2 * q * Z)[r + js[q]];
#pragma unroll
                    for (int q = 0; q < DC; q++) wq[q] = slots[sl[q]];
                    uint32_t k1 = 0xFFFFFFFFu, k2 = 0xFFFFFFFFu, sx = 0;
#pragma unroll
                    for (int q = 0; q < DC; q++) {
                        const uint32_t av = (wq[q] >> 8) & 0xFFu;
                        sx ^= wq[q];  // bit 7: parity of the negative members
                        const uint32_t key = (av << 3) | (uint32_t)q;
                        k2 = min(k2, max(k1, key));
                        k1 = min(k1, key);
                    }
                    par = (sx >> 7) & 1u;
                    const uint32_t m1 = k1 >> 3, m2 = k2 >> 3, pos = k1 & 7u;
                    chk[i * Z + r] = m1 | (m2 << 8) | (pos << 16) | (par << 24);  // bit 24: syndrome
                    // the check's two signed terms, formed once
                    const uint32_t d1 = ((uint32_t)(par ? (int)m1 : -(int)m1) << 16) + par;
                    const uint32_t d2 = ((uint32_t)(par ? (int)m2 : -(int)m2) << 16) + par;
#pragma unroll
                    for (int q = 0; q < DC; q++) atomicAdd(&slots[sl[q]], pos == (uint32_t)q ? d2 : d1);
                }
                const unsigned long long b = __ballot(valid && par);
                weight += __popcll(b);
            }
        }
        lwave_sync();

        int t = 0, okf = 0, rec_end = 0;
        uint32_t prv = NONE;
        const uint32_t *cw = a.pool ? a.pool + (size_t)((a.f0 + f) % a.pool_n) * NW : nullptr;
        for (;;) {
            // this round's copies of the launch's switches
            const int Lr = fresh(a.L), kr = fresh(a.k);
            fwbf_record *const rec = fresh(a.rec);
            const bool pool = fresh(a.pool) != nullptr;
            const float invA = fresh(a.invA);
            if (weight == 0) { okf = 1; break; }
            if (t == a.T) break;
            const float al = a.params[O_AL + t], be = a.params[O_AL + a.T + t];
            // k best per block by E_t (ties: lower index); each chosen slot is
            // excluded before the next pass
            uint64_t excl = 0;
            for (int rk = 0; rk < kr; rk++) {
                // the lane's best live slot, scanned in ascending position with
                // a strict comparison (ties keep the lower position; -0 == +0)
                const uint64_t livem = realm & ~excl;
                float bE = -__builtin_huge_valf();  // E is finite: a live slot always beats it
                uint32_t bi = NONE;                  // no live slot yet
                // every chunk read is issued before any is scanned
                uint4 cv[C / 4];
#pragma unroll
                for (int kk = 0; kk < C; kk += 4) cv[kk >> 2] = ((const uint4 *)slots)[slot_chunk(lane, kk >> 2)];
#pragma unroll
                for (int kk = 0; kk < C; kk += 4) {
                    const uint4 v = cv[kk >> 2];
                    const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const float S = (float)((int32_t)vv[u] >> 16);
                        const float E = __builtin_fmaf(-al, (float)((vv[u] >> 8) & 0xFFu), be * S);
                        const uint32_t lm = kk + u < 32 ? (uint32_t)livem : (uint32_t)(livem >> 32);
                        const bool live = (lm >> ((kk + u) & 31)) & 1;
                        const bool take = live && E > bE;
                        bE = take ? E : bE;
                        bi = take ? (uint32_t)(kk + u) : bi;
                    }
                }
                unsigned long long best = bi == NONE ? 0ull
                                                     : (((unsigned long long)orderable(bE) << 32) |
                                                        (0xFFFFFFFFu - (pos0 + bi)));
                best = group_max64(best, Lr);
                const uint32_t bpos = 0xFFFFFFFFu - (uint32_t)best;
                const bool real = (best >> 32) != 0;
                if (real && (int)g < a.Geff && bpos / C == (lane & (a.L - 1))) excl |= 1ull << (bpos & (C - 1));
                if (lead) {
                    const uint32_t word = real ? slots[slot_word(g * a.L + bpos / C, bpos & (C - 1))] : 0u;
                    cand[g * a.k + rk] = make_uint4(real ? gp + bpos : NONE, word, 0, 0);
                }
            }
            lwave_sync();
            // features of proposal lane % 32, score
            const uint32_t j = lane & 31;
            const uint4 cj = j < (uint32_t)NC ? cand[j] : make_uint4(NONE, 0, 0, 0);
            const bool realc = cj.x != NONE;
            const int cS = (int32_t)cj.y >> 16;
            const uint32_t ca = (cj.y >> 8) & 0xFFu, cu = cj.y & 0x7Fu;  // bit 7: the sign of y
            bf16x4 x = pack4(0.f, 0.f, 0.f, 0.f);
            if (lane < 32 && realc) {
                const float E = __builtin_fmaf(-al, (float)ca, be * (float)cS);
                // the same quotients as dividing: a power-of-two scale is a
                // multiply by its reciprocal, u / dv takes one of dv + 1 values
                float fa, fe;
                if (invA != 0.0f) { fa = (float)ca * invA; fe = E * invA; }
                else { fa = (float)ca / a.A; fe = E / a.A; }
                const float fu = cu == 0 ? 0.0f : cu == 1 ? qu1 : cu == 2 ? qu2 : cu == 3 ? qu3 : (float)cu / a.dv;
                x = pack4(fa, fe, fu, nbias[96 + t]);
            }
            const float score = net_score(net, x);
            // every one of the 32 slots is written in each round run; slots
            // j >= NC (no proposal) get valid = 0
            if (rec && lane < 32) {
                fwbf_record r;
                r.S = cS;
                r.a = (uint16_t)ca;
                r.u = (uint8_t)cu;
                r.pad = 0;
                uint32_t lab = 0;
                if (realc) {
                    const uint32_t zb = (zw[cj.x >> 5] >> (cj.x & 31)) & 1u;
                    const uint32_t cb = pool ? (cw[cj.x >> 5] >> (cj.x & 31)) & 1u : 0u;
                    lab = zb ^ cb;
                }
                r.label = (uint8_t)lab;
                r.valid = realc ? 1 : 0;
                r.n = (uint16_t)(realc ? cj.x : 0xFFFF);
                rec[((size_t)f * a.T + t) * 32 + j] = r;
            }
            rec_end = t + 1;
            // best score among the k proposals of each block (ties: lower index)
            unsigned long long sk = realc ? (((unsigned long long)orderable(score) << 32) | (0xFFFFFFFFu - cj.x)) : 0ull;
            if (kr > 1) sk = group_max64(sk, kr);
            const bool blead = lane < 32 && (j % kr) == 0 && j < (uint32_t)NC;
            const uint32_t nsel = 0xFFFFFFFFu - (uint32_t)sk;
            const bool flip = blead && (sk >> 32) > orderable(0.0f) && sk != 0;
            const uint32_t cur = flip ? nsel : NONE;
            const unsigned long long fmask = __ballot(flip);
            const unsigned long long dmask = __ballot(blead && cur != prv);
            prv = blead ? cur : prv;
            if (fmask == 0 || dmask == 0) break;  // no flip, or the previous round's flips: stop
            // the winners flip their bits and list them; then one lane per
            // (winner, check) pair toggles the check and adds +-(2w, 1) to S
            // and u of the check's members, the sign given by the check's new
            // bit (toggles of one check by two winners cancel exactly)
            const int rank = __popcll(fmask & ((1ull << lane) - 1));
            if (flip) {
                atomicXor(&zw[nsel >> 5], 1u << (nsel & 31));
                list[rank] = nsel;
            }
            lwave_sync();
            const int nflip = __popcll(fmask);
            const int ntog = nflip * DV;
            int sum_ones = 0;  // toggles that leave their check unsatisfied
            constexpr uint32_t DVM = ((1u << 16) + DV - 1) / DV;  // i / DV = (i * DVM) >> 16 for i < 2^12
            for (int base = 0; base < ntog; base += 64) {
                const int i = base + (int)lane;
                uint32_t nb1 = 0;
                if (i < ntog) {
                    const uint32_t u = mul24((uint32_t)i, DVM) >> 16;
                    const uint32_t tt = (uint32_t)i - mul24(u, (uint32_t)DV);
                    const uint32_t n = list[u];
                    const uint32_t jb = mul24(n, a.rZ24) >> 22;  // block column: n / Z
                    const uint32_t c = n - mul24(jb, Z);
                    const uint32_t *st = sh + mul24(tt, (uint32_t)a.nb);
                    const uint32_t rr = submod(c, st[jb], Z);
                    const uint32_t m = mul24(tt, Z) + rr;
                    // toggles the syndrome bit (bit 24) and returns the minima
                    const uint32_t cwd = atomicXor(&chk[m], 1u << 24);
                    nb1 = ((cwd >> 24) & 1u) ^ 1u;
                    const uint32_t e1 = ((2u * (cwd & 0xFFu)) << 16) + 1u, e2 = ((2u * ((cwd >> 8) & 0xFFu)) << 16) + 1u;
                    const uint32_t d1 = nb1 ? e1 : 0u - e1, d2 = nb1 ? e2 : 0u - e2;
                    const uint32_t pos = (cwd >> 16) & 0xFFu;
                    uint32_t sl[DC];
#pragma unroll
                    for (int q = 0; q < DC; q++) sl[q] = slotof[mul24((uint32_t)q, 2 * Z) + rr + st[q]];
#pragma unroll
                    for (int q = 0; q < DC; q++) atomicAdd(&slots[sl[q]], pos == (uint32_t)q ? d2 : d1);
                }
                sum_ones += __popcll(__ballot(nb1));
            }
            weight += 2 * sum_ones - DV * nflip;
            t += 1;
            lwave_sync();
        }
        lwave_sync();
        // records of the rounds not run are marked invalid
        if (fresh(a.rec))
            for (int s = rec_end; s < a.T; s++)
                if (lane < 32) a.rec[((size_t)f * a.T + s) * 32 + lane].valid = 0;
        uint32_t *zo = a.z + f * NW;
        for (int w = lane; w < NW; w += 64) zo[w] = zw[w];
        if (lane == 0) {
            a.iters[f] = t;
            a.ok[f] = (uint8_t)okf;
            if (fresh(a.learned_ok)) a.learned_ok[f] = (uint8_t)okf;
        }
    }
}

// ---------------------------------------------------------------------------
// Learned pass with one frame per workgroup (larger codes, int8 or int16)
// ---------------------------------------------------------------------------
// The same rounds as learned_kernel for any full base of single shifts with
// three block rows.  Slot word of bit n: S << 14 | min(|y_n|, 4095) << 2 | u
// (S signed, |S| <= 3 * 32768 < 2^17; u <= 3): adds to S and u never carry
// across the fields, and a saturated magnitude field means that |y_n| is read
// from the frame's row in global memory.  Block g (p bits) is padded to
// Lc = L*C slots: thread (g, l) holds positions l, l + L, ..., and the column
// kk = pos / L is XORed with g mod B (B = 64/L blocks per wavefront) so that a
// wavefront's slot reads use distinct LDS banks.  Proposal c = block * k +
// rank is scored by lane c % 32 of wavefront c / 32.
constexpr int WIDE_T = 1024;
constexpr uint32_t WSAT = 4095;
constexpr int CW_WEIGHT = 0, CW_FLAGS = 1, CW_NTOG = 2, CW_SAT = 3;

struct WideArgs {
    const void *y;
    int64_t F, stride;
    uint32_t *z;
    int32_t *iters;
    uint8_t *ok;
    uint8_t *learned_ok;  // optional
    fwbf_record *rec;     // optional [F][T][32 tpr]
    const uint32_t *pool; // labels for records (pool row f % pool_n, NULL: all-zero)
    int64_t pool_n, f0;
    const float *params;
    int N, M, Z, nb;
    // quotients by Z, p and nb as 24-bit multiplies: x / d = (x * r) >> s for
    // every x below the kernel's bound (checked exhaustively on the host)
    uint32_t rZ, sZ, rP, sP, rD, sD;
    uint16_t shv[3 * 32];  // the shifts (3 x nb), staged in LDS
    int p, L, logL, Lc, B, Geff, k, T, NC, tpr;
    int pref;   // rows are whole 4-byte words: loaded as words, the next one ahead
    float A, invA, dv;
    int o_chk, o_chkp, o_z, o_syn, o_cand, o_list, o_ctl, o_sh, o_net, o_netw, lds_bytes;
};

__device__ __forceinline__ uint32_t wide_slot(const WideArgs &a, uint32_t n)
{
    const uint32_t g = mul24(n, a.rP) >> a.sP, pos = n - mul24(g, (uint32_t)a.p);
    return mul24(g, (uint32_t)a.Lc) + (pos ^ ((g & (uint32_t)(a.B - 1)) << a.logL));
}

template <int DT>
__device__ __forceinline__ uint32_t wide_mag(const void *yrow, uint32_t n)
{
    if constexpr (DT == FWBF_I8) {
        const int v = ((const int8_t *)yrow)[n];
        return (uint32_t)(v < 0 ? -v : v);
    } else {
        const int v = ((const int16_t *)yrow)[n];
        return (uint32_t)(v < 0 ? -v : v);
    }
}

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

// Member keys |y| << 5 | q of QL consecutive block columns q0.. of the
// checks r (lanes) of one block row whose shifts are si[]: all reads issued
// before any is used. Folds them into the two smallest keys and the parity
// of the negative members (the sign bit of sx).
template <int QL, typename Y>
__device__ __forceinline__ void member_keys(const Y *sty, const uint32_t *si, uint32_t Z, uint32_t r, uint32_t rm,
                                            int q0, uint32_t &k1, uint32_t &k2, int &sx)
{
    uint32_t s[QL];
    int v[QL];
#pragma unroll
    for (int u = 0; u < QL; u++) s[u] = si[q0 + u];
#pragma unroll
    for (int u = 0; u < QL; u++) v[u] = sty[(uint32_t)(q0 + u) * Z + min(r + s[u], rm + s[u])];
#pragma unroll
    for (int u = 0; u < QL; u++) {
        sx ^= v[u];
        const uint32_t key = ((uint32_t)(v[u] < 0 ? -v[u] : v[u]) << 5) | (uint32_t)(q0 + u);
        k2 = med3u(k1, key, k2);
        k1 = min(k1, key);
    }
}

template <int DT, int C>
__global__ __launch_bounds__(WIDE_T) void learned_wide_kernel(WideArgs a)
{
    using Y = typename std::conditional<DT == FWBF_I8, int8_t, int16_t>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *slots = (uint32_t *)smem;
    uint32_t *chk = (uint32_t *)(smem + a.o_chk);    // min1 | min2 << 16
    uint8_t *chkp = smem + a.o_chkp;                  // lowest position holding min1
    uint32_t *zw = (uint32_t *)(smem + a.o_z);
    uint32_t *syn = (uint32_t *)(smem + a.o_syn);
    uint32_t *cand = (uint32_t *)(smem + a.o_cand);  // proposals: bit index or NONE
    uint32_t *list = (uint32_t *)(smem + a.o_list);  // toggles: check | new bit << 31
    int *ctl = (int *)(smem + a.o_ctl);
    uint32_t *sh = (uint32_t *)(smem + a.o_sh);
    float *nbias = (float *)(smem + a.o_net);
    bf16x4 *nw = (bf16x4 *)(smem + a.o_netw);
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t Z = a.Z;
    const int N = a.N, M = a.M, dc = a.nb;

    for (int t = tid; t < 3 * dc; t += WIDE_T) sh[t] = a.shv[t];
    for (int t = tid; t < 32; t += WIDE_T) {
        nbias[t] = a.params[O_B1 + t];
        nbias[32 + t] = a.params[O_B2 + t];
        nbias[64 + t] = a.params[O_W3 + t];
    }
    for (int t = tid; t < a.T; t += WIDE_T) nbias[96 + t] = (float)t / (float)a.T;
    if (tid < 64) {
        const int i = lane & 31, hi = lane >> 5;
        const float *p = a.params;
        nw[5 * lane] = hi == 0 ? pack4(p[O_W1 + i * 4 + 0], p[O_W1 + i * 4 + 1], p[O_W1 + i * 4 + 2], p[O_W1 + i * 4 + 3])
                               : pack4(0.f, 0.f, 0.f, 0.f);
        for (int c = 0; c < 4; c++) {
            const float *r = p + O_W2 + i * H + 8 * c + 4 * hi;
            nw[5 * lane + 1 + c] = pack4(r[0], r[1], r[2], r[3]);
        }
    }
    __syncthreads();
    NetL net;
    net.wq = nw;
    net.b1 = nbias;
    net.b2 = nbias + 32;
    net.w3 = nbias + 64;
    net.b3 = a.params[O_B3];

    const float qu1 = 1.0f / a.dv, qu2 = 2.0f / a.dv, qu3 = 3.0f / a.dv;
    const uint32_t g = tid >> a.logL, l = tid & (uint32_t)(a.L - 1);
    const bool gact = (int)g < a.Geff;
    const uint32_t gp = g * (uint32_t)a.p;
    const uint32_t swk = g & (uint32_t)(a.B - 1);  // column swizzle of this block
    const uint32_t sbase = gact ? g * (uint32_t)a.Lc + l : 0u;  // idle threads read block 0 (never live)
    uint64_t realm = 0;
#pragma unroll
    for (int kk = 0; kk < C; kk++) {
        const uint32_t pos = l + ((uint32_t)kk << a.logL);
        realm |= (uint64_t)(gact && (int)pos < a.p && (int)(gp + pos) < N) << kk;
    }
    const int nreal = __popcll(realm);  // the real slots are the thread's first nreal
    // slot kk0 + u (kk0 a multiple of 4, u < 4) of this thread: sbase +
    // ((kk0 ^ swk) << logL) + offu[u], the swizzle split over the two parts
    uint32_t offu[4];
#pragma unroll
    for (int u = 0; u < 4; u++) offu[u] = ((uint32_t)u ^ (swk & 3u)) << a.logL;
    const bool scorer = (int)wv < a.tpr;  // wavefront-uniform
    const uint32_t j = lane & 31, c = 32 * wv + j;
    const bool blead = scorer && lane < 32 && (j % a.k) == 0 && (int)c < a.NC;
    const int NW = (N + 31) >> 5;
    const int NZc = (int)((Z + 63) >> 6);  // 64-wide chunks of a block row or column

    const FrameRange fr = xcd_frames(a.F);
    // The next frame's row is loaded into registers while this frame
    // decodes (rows of at most PW * WIDE_T words): with one frame per compute
    // unit nothing else would hide the memory latency.
    constexpr int PW = 16;
    const int nwords = (N * (int)sizeof(Y)) >> 2;
    uint32_t pre[PW];
    bool have = false;  // pre[] holds this frame's row
    for (int64_t f = fr.first; f < fr.end; f += fr.step) {
        const Y *yrow = (const Y *)a.y + f * a.stride;
        if (tid == 0) { ctl[CW_WEIGHT] = 0; ctl[CW_FLAGS] = 0; ctl[CW_NTOG] = 0; ctl[CW_SAT] = 0; }
        {
            // ---- the row into LDS, over the slots (y of bit n at element n)
            uint32_t *stw = slots;
            const Y *sty = (const Y *)slots;
            if (have) {
#pragma unroll
                for (int i = 0; i < PW; i++) {
                    const int w = tid + i * WIDE_T;
                    if (w < nwords) stw[w] = pre[i];
                }
            } else if (a.pref) {
                const uint32_t *src = (const uint32_t *)yrow;
#pragma unroll
                for (int i = 0; i < PW; i++) {
                    const int w = tid + i * WIDE_T;
                    pre[i] = w < nwords ? src[w] : 0u;
                }
#pragma unroll
                for (int i = 0; i < PW; i++) {
                    const int w = tid + i * WIDE_T;
                    if (w < nwords) stw[w] = pre[i];
                }
            } else {
                for (int n0 = tid; n0 < N; n0 += 8 * WIDE_T) {
                    Y v[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) v[u] = n0 + u * WIDE_T < N ? yrow[n0 + u * WIDE_T] : (Y)0;
#pragma unroll
                    for (int u = 0; u < 8; u++)
                        if (n0 + u * WIDE_T < N) ((Y *)slots)[n0 + u * WIDE_T] = v[u];
                }
            }
            // the syndrome is built by OR-ing 64-bit ballots at any bit offset
            for (int w = tid; w < 2 * ((M + 63) >> 6); w += WIDE_T) syn[w] = 0u;
            __syncthreads();
            // ---- z_0 = [y < 0] from the staged row, 64 bits per ballot
            for (int n0 = 64 * (int)wv; n0 < N; n0 += 4 * WIDE_T) {
                int v[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int n = n0 + u * WIDE_T + (int)lane;
                    v[u] = n < N ? (int)sty[n] : 0;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const unsigned long long b = __ballot(v[u] < 0);
                    const int w = (n0 + u * WIDE_T) >> 5;
                    if (lane < 2 && n0 + u * WIDE_T < N) zw[w + (int)lane] = lane ? (uint32_t)(b >> 32) : (uint32_t)b;
                }
            }
            // ---- check minima and syndrome s_0 from the staged row. A
            // wavefront takes 64 consecutive checks of one block row, so the
            // row's shifts are uniform and the members' addresses consecutive
            // (conflict-free) up to one wrap. Lanes past the row's end read
            // in-bounds values that are never stored.
            for (int ch = (int)wv; ch < 3 * NZc; ch += WIDE_T / 64) {
                const int i = ch / NZc;
                const uint32_t r0 = (uint32_t)(ch - i * NZc) << 6, r = r0 + lane;
                const uint32_t rm = r - Z;  // rm + s wraps below Z
                const uint32_t *si = sh + i * dc;
                // the two smallest keys |y| << 5 | q: min1 and min2 (with
                // multiplicity) and the position holding min1 (any one of equal
                // minima: min2 then equals min1)
                uint32_t k1 = 0xFFFFFFFFu, k2 = 0xFFFFFFFFu;
                int sx = 0;
                int q0 = 0;
                for (; q0 + 8 <= dc; q0 += 8) member_keys<8>(sty, si, Z, r, rm, q0, k1, k2, sx);
                if (q0 + 4 <= dc) { member_keys<4>(sty, si, Z, r, rm, q0, k1, k2, sx); q0 += 4; }
                if (q0 + 2 <= dc) { member_keys<2>(sty, si, Z, r, rm, q0, k1, k2, sx); q0 += 2; }
                if (q0 < dc) member_keys<1>(sty, si, Z, r, rm, q0, k1, k2, sx);
                const bool valid = r < Z;
                const uint32_t m = (uint32_t)i * Z + r;
                if (valid) {
                    chk[m] = (k1 >> 5) | ((k2 >> 5) << 16);
                    chkp[m] = (uint8_t)(k1 & 31u);
                }
                const unsigned long long b = __ballot(valid && sx < 0);
                if (b) {
                    or_bits(syn, (uint32_t)i * Z + r0, b, lane);
                    if (lane == 0) atomicAdd(&ctl[CW_WEIGHT], __popcll(b));
                }
            }
            __syncthreads();
            // ---- slot words: 64 consecutive bits of one block column per
            // wavefront, S and u gathered from the bits' three checks with
            // min1 as every weight (the argmin members are corrected below),
            // |y| read again from the row in global memory (the staged copy is
            // dead once the slots take its place)
            {
                int ch = (int)wv;
                int xn = 0;
                uint32_t maxav = 0;  // (lanes past a column's end read a real bit of it)
                if (ch < dc * NZc) {
                    const int jb = ch / NZc;
                    const uint32_t c = ((uint32_t)(ch - jb * NZc) << 6) + lane;
                    xn = yrow[(uint32_t)jb * Z + (c < Z ? c : 0u)];
                }
                for (; ch < dc * NZc; ch += WIDE_T / 64) {
                    const int x = xn;
                    const int jb = ch / NZc;
                    // (the uniform chunk start kept apart from the lane index)
                    const uint32_t c0 = __builtin_amdgcn_readfirstlane((uint32_t)(ch - jb * NZc) << 6);
                    const uint32_t c = c0 + lane, cz = c + Z;
                    {   // the next chunk's y, in flight while this one is built
                        const int chn = ch + WIDE_T / 64;
                        if (chn < dc * NZc) {
                            const int jn = chn / NZc;
                            const uint32_t cn = ((uint32_t)(chn - jn * NZc) << 6) + lane;
                            xn = yrow[(uint32_t)jn * Z + (cn < Z ? cn : 0u)];
                        }
                    }
                    uint32_t s3[3];
#pragma unroll
                    for (int tt = 0; tt < 3; tt++) s3[tt] = sh[tt * dc + jb];  // broadcast reads
                    // S = 2 (sum of w over unsatisfied checks) - (sum of w)
                    uint32_t su = 0, sw = 0, uu = 0;
#pragma unroll
                    for (int tt = 0; tt < 3; tt++) {
                        const uint32_t mm = (uint32_t)tt * Z + min(c - s3[tt], cz - s3[tt]);
                        const uint32_t w = ((const uint16_t *)chk)[2 * mm];  // min1
                        // bit mm of the syndrome (the extract takes the offset mod 32)
                        const uint32_t sb = __builtin_amdgcn_ubfe(syn[__builtin_amdgcn_ubfe(mm, 5, 27)], mm, 1);
                        su += sb * w;
                        sw += w;
                        uu += sb;
                    }
                    const uint32_t av = (uint32_t)(x < 0 ? -x : x);
                    if (c < Z)
                        slots[wide_slot(a, (uint32_t)jb * Z + c)] =
                            ((2u * su - sw) << 14) | (min(av, WSAT) << 2) | uu;
                    maxav = max(maxav, av);
                }
                // some magnitude saturates its field: the scan then reads it from global memory
                if (__ballot(maxav >= WSAT) && lane == 0) ctl[CW_SAT] = 1;
            }
            __syncthreads();
            // ---- the member of each check at min1 takes min2: one correction
            // of +-(min2 - min1) to its S
            for (int ch = (int)wv; ch < 3 * NZc; ch += WIDE_T / 64) {
                const int i = ch / NZc;
                const uint32_t r = ((uint32_t)(ch - i * NZc) << 6) + lane;
                if (r < Z) {
                    const uint32_t m = (uint32_t)i * Z + r, cwd = chk[m];
                    const uint32_t d = (cwd >> 16) - (cwd & 0xFFFFu);
                    if (d) {
                        const uint32_t q = chkp[m], s = sh[i * dc + (int)q];
                        const uint32_t sb = (syn[m >> 5] >> (m & 31)) & 1u;
                        const uint32_t n = mul24(q, Z) + min(r + s, r + s - Z);
                        atomicAdd(&slots[wide_slot(a, n)], (sb ? d : 0u - d) << 14);
                    }
                }
            }
            __syncthreads();
            // ---- the next frame's row, loaded while this one decodes
            have = false;
            if (a.pref && f + fr.step < fr.end) {
                const uint32_t *src = (const uint32_t *)((const Y *)a.y + (f + fr.step) * a.stride);
#pragma unroll
                for (int i = 0; i < PW; i++) {
                    const int w = tid + i * WIDE_T;
                    pre[i] = w < nwords ? src[w] : 0u;
                }
                have = true;
            }
        }

        int t = 0, okf = 0, rec_end = 0;
        uint32_t prv = NONE;
        const uint32_t *cw = a.pool ? a.pool + (size_t)((a.f0 + f) % a.pool_n) * NW : nullptr;
        const bool anysat = DT == FWBF_I16 && ctl[CW_SAT] != 0;  // uniform
        for (;;) {
            // this round's copies of the launch's switches
            const int kr = fresh(a.k), Lr = fresh(a.L), logLr = fresh(a.logL);
            fwbf_record *const rec = fresh(a.rec);
            const bool pool = fresh(a.pool) != nullptr;
            const float invA = fresh(a.invA);
            if (ctl[CW_WEIGHT] == 0) { okf = 1; break; }
            if (t == a.T) break;
            const float al = a.params[O_AL + t], be = a.params[O_AL + a.T + t];
            // ---- the k best live slots of each block by E_t (ties: lower index)
            uint64_t excl = 0;
            for (int rk = 0; rk < kr; rk++) {
                const uint64_t livem = realm & ~excl;
                float bE = -__builtin_huge_valf();
                uint32_t bi = NONE;
                // four slot reads in flight at a time (the loop itself is not
                // unrolled: register pressure at 1024 threads per workgroup);
                // two forms: one proposal per block and no saturated magnitude
                // in the frame (the live slots are the real ones), or any case
                auto scan = [&](auto one) {
                    constexpr bool K1 = decltype(one)::value;
#pragma unroll 1
                    for (int kk = 0; kk < C; kk += 4) {
                        uint32_t v[4];
                        const uint32_t base = sbase + (((uint32_t)kk ^ (swk & ~3u)) << logLr);
#pragma unroll
                        for (int u = 0; u < 4; u++) v[u] = slots[base + offu[u]];
#pragma unroll
                        for (int u = 0; u < 4; u++) {
                            const bool live = K1 ? kk + u < nreal : ((livem >> (kk + u)) & 1) != 0;
                            uint32_t av = (v[u] >> 2) & WSAT;
                            if constexpr (DT == FWBF_I16 && !K1)
                                if (live && av == WSAT) av = wide_mag<DT>(yrow, gp + l + ((uint32_t)(kk + u) << logLr));
                            const float E = __builtin_fmaf(-al, (float)av, be * (float)((int32_t)v[u] >> 14));
                            const bool take = live && E > bE;
                            bE = take ? E : bE;
                            bi = take ? (uint32_t)(kk + u) : bi;
                        }
                    }
                };
                if (kr == 1 && !anysat) scan(std::true_type{});
                else scan(std::false_type{});
                const uint32_t nme = gp + l + (bi << logLr);
                unsigned long long best = bi == NONE ? 0ull : (((unsigned long long)orderable(bE) << 32) | (0xFFFFFFFFu - nme));
                best = group_max64(best, Lr);
                const bool real = (best >> 32) != 0;
                const uint32_t bn = 0xFFFFFFFFu - (uint32_t)best;
                if (real && bi != NONE && bn == nme) excl |= 1ull << bi;
                if (gact && l == 0) cand[g * kr + rk] = real ? bn : NONE;
            }
            if (tid == 0) { ctl[CW_FLAGS] = 0; ctl[CW_NTOG] = 0; }
            __syncthreads();
            // ---- scores of the proposals, the flip decision of every block
            uint32_t nsel = NONE;
            bool flip = false;
            if (scorer) {
                const uint32_t cn = (lane < 32 && (int)c < a.NC) ? cand[c] : NONE;
                const bool realc = cn != NONE;
                uint32_t word = 0, ca = 0;
                if (realc) {
                    word = slots[wide_slot(a, cn)];
                    ca = (word >> 2) & WSAT;
                    if (DT == FWBF_I16 && ca == WSAT) ca = wide_mag<DT>(yrow, cn);
                }
                const int cS = (int32_t)word >> 14;
                const uint32_t cu = word & 3u;
                bf16x4 x = pack4(0.f, 0.f, 0.f, 0.f);
                if (realc) {
                    const float E = __builtin_fmaf(-al, (float)ca, be * (float)cS);
                    float fa, fe;
                    if (invA != 0.0f) { fa = (float)ca * invA; fe = E * invA; }
                    else { fa = (float)ca / a.A; fe = E / a.A; }
                    const float fu = cu == 0 ? 0.0f : cu == 1 ? qu1 : cu == 2 ? qu2 : qu3;
                    x = pack4(fa, fe, fu, nbias[96 + t]);
                }
                const float score = net_score(net, x);
                if (rec && lane < 32) {
                    fwbf_record r;
                    r.S = cS;
                    r.a = (uint16_t)ca;
                    r.u = (uint8_t)cu;
                    r.pad = 0;
                    uint32_t lab = 0;
                    if (realc) {
                        const uint32_t zb = (zw[cn >> 5] >> (cn & 31)) & 1u;
                        const uint32_t cb = pool ? (cw[cn >> 5] >> (cn & 31)) & 1u : 0u;
                        lab = zb ^ cb;
                    }
                    r.label = (uint8_t)lab;
                    r.valid = realc ? 1 : 0;
                    r.n = (uint16_t)(realc ? cn : 0xFFFF);
                    rec[(((size_t)f * a.T + t) * a.tpr + wv) * 32 + j] = r;
                }
                // best score among the k proposals of each block (ties: lower index)
                unsigned long long sk = realc ? (((unsigned long long)orderable(score) << 32) | (0xFFFFFFFFu - cn)) : 0ull;
                if (kr > 1) sk = group_max64(sk, kr);
                nsel = 0xFFFFFFFFu - (uint32_t)sk;
                flip = blead && sk != 0 && (uint32_t)(sk >> 32) > orderable(0.0f);
                const uint32_t cur = flip ? nsel : NONE;
                const unsigned long long fm = __ballot(flip), dm = __ballot(blead && cur != prv);
                prv = blead ? cur : prv;
                if (lane == 0 && (fm | dm)) atomicOr(&ctl[CW_FLAGS], (fm ? 1 : 0) | (dm ? 2 : 0));
            }
            rec_end = t + 1;
            __syncthreads();
            const int flg = ctl[CW_FLAGS];
            if (!(flg & 1) || !(flg & 2)) break;  // no flip, or the previous round's flips: stop
            // ---- flips: z, the three syndrome toggles, the toggle list
            if (scorer) {
                const unsigned long long fm = __ballot(flip);
                if (fm) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(&ctl[CW_NTOG], 3 * __popcll(fm));
                    base = __shfl(base, 0, 64);
                    const int rank = __popcll(fm & ((1ull << lane) - 1));
                    uint32_t ones = 0;
                    if (flip) {
                        const uint32_t n = nsel;
                        atomicXor(&zw[n >> 5], 1u << (n & 31));
                        const uint32_t jb = mul24(n, a.rZ) >> a.sZ, cc = n - mul24(jb, Z);
                        uint32_t mm[3], old[3];
#pragma unroll
                        for (int tt = 0; tt < 3; tt++) mm[tt] = mul24((uint32_t)tt, Z) + submod(cc, sh[tt * dc + jb], Z);
#pragma unroll
                        for (int tt = 0; tt < 3; tt++) old[tt] = atomicXor(&syn[mm[tt] >> 5], 1u << (mm[tt] & 31));
#pragma unroll
                        for (int tt = 0; tt < 3; tt++) {
                            const uint32_t nb1 = ((old[tt] >> (mm[tt] & 31)) & 1u) ^ 1u;
                            ones += nb1;
                            list[base + 3 * rank + tt] = mm[tt] | (nb1 << 31);
                        }
                    }
                    // unsatisfied checks: +1 per toggle to 1, -1 per toggle to 0
                    int dw = flip ? 2 * (int)ones - 3 : 0;
#pragma unroll
                    for (int d = 32; d >= 1; d >>= 1) dw += __shfl_xor(dw, d, 64);
                    if (lane == 0 && dw) atomicAdd(&ctl[CW_WEIGHT], dw);
                }
            }
            t += 1;
            __syncthreads();
            // ---- +-(2w, 1) to S and u of every member of every toggled check
            const int ntask = ctl[CW_NTOG] * dc;
            for (int id = tid; id < ntask; id += WIDE_T) {
                const uint32_t e0 = mul24((uint32_t)id, a.rD) >> a.sD, q = id - mul24(e0, (uint32_t)dc);
                const uint32_t ent = list[e0];
                const uint32_t m = ent & 0x7FFFFFFFu;
                const uint32_t i = mul24(m, a.rZ) >> a.sZ, r = m - mul24(i, Z);
                const uint32_t n = mul24(q, Z) + addmod(r, sh[mul24(i, (uint32_t)dc) + q], Z);
                const uint32_t cwd = chk[m];
                const uint32_t w = chkp[m] == q ? (cwd >> 16) : (cwd & 0xFFFFu);
                const uint32_t d = ((2u * w) << 14) + 1u;
                atomicAdd(&slots[wide_slot(a, n)], (ent >> 31) ? d : 0u - d);
            }
            __syncthreads();
        }
        // records of the rounds not run are marked invalid
        if (a.rec && scorer && lane < 32)
            for (int s = rec_end; s < a.T; s++) a.rec[(((size_t)f * a.T + s) * a.tpr + wv) * 32 + j].valid = 0;
        uint32_t *zo = a.z + f * NW;
        for (int w = tid; w < NW; w += WIDE_T) zo[w] = zw[w];
        if (tid == 0) {
            a.iters[f] = t;
            a.ok[f] = (uint8_t)okf;
            if (a.learned_ok) a.learned_ok[f] = (uint8_t)okf;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// training kernels
// ---------------------------------------------------------------------------
struct GradArgs {
    const fwbf_record *rec;
    int64_t n_tiles;
    const float *params;
    float pos_weight, A, dv;
    int T, P, tpr;   // tpr: tiles of 32 records per round
    float *partial;  // [gridDim][P + 2]
    float *scores;   // optional forward output [n_tiles][32]
    int backward;
};

// features of record j of a tile in lanes 0..31 (bfloat16), zero above
__device__ __forceinline__ bf16x4 record_features(const fwbf_record &r, int t, const GradArgs &g, float al, float be)
{
    const float S = (float)r.S;
    const float E = __builtin_fmaf(-al, (float)r.a, be * S);
    return pack4((float)r.a / g.A, E / g.A, (float)r.u / g.dv, (float)t / (float)g.T);
}

__global__ __launch_bounds__(64) void grad_kernel(GradArgs g)
{
    __shared__ float sp2[32][33];  // dpre2 (rounded) [hidden][cand]
    __shared__ float sp1[32][33];  // dpre1 [hidden][cand]
    __shared__ float sh1[32][33];  // h1 (rounded) [hidden][cand]
    __shared__ float sh2[32][33];  // h2 [hidden][cand]
    __shared__ float sx[4][33];    // features (rounded) [feature][cand]
    __shared__ float sab[2][64];   // alpha / beta gradient accumulators per round
    __shared__ float sds[32];      // d loss / d score of every candidate of the tile
    __shared__ float sw1c[32];     // W1[k][1] (rounded), the E_t column of layer 1
    const int l = threadIdx.x, j = l & 31, hi = l >> 5;
    Net net;
    load_net(net, g.params);
    for (int t = l; t < 128; t += 64) (&sab[0][0])[t] = 0.0f;
    // per-lane accumulators
    float aW1a = 0, aW1b = 0, aB = 0, aW3 = 0, aB3 = 0, aLoss = 0, aCnt = 0;
    f32x16 aW2 = {};
    // W2 transposed as the A operand of dh1 = W2^T dpre2: lane l holds
    // W2[8c + 4(l/32) + 0..3][l % 32]
    bf16x4 w2t[4];
    for (int c = 0; c < 4; c++) {
        const int k0 = 8 * c + 4 * hi;
        w2t[c] = pack4(g.params[O_W2 + (k0 + 0) * H + j], g.params[O_W2 + (k0 + 1) * H + j],
                       g.params[O_W2 + (k0 + 2) * H + j], g.params[O_W2 + (k0 + 3) * H + j]);
    }
    if (l < 32) sw1c[l] = bf16_f(bf16_rne(g.params[O_W1 + l * 4 + 1]));
    __syncthreads();
    for (int64_t tile = blockIdx.x; tile < g.n_tiles; tile += gridDim.x) {
        const int t = (int)((tile / g.tpr) % g.T);
        const fwbf_record r = g.rec[tile * 32 + j];
        const bool valid = r.valid != 0;
        if (!__ballot(valid)) {  // empty tile
            if (g.scores && hi == 0) g.scores[tile * 32 + j] = 0.0f;
            continue;
        }
        const float al = g.params[O_AL + t], be = g.params[O_AL + g.T + t];
        bf16x4 x = pack4(0.f, 0.f, 0.f, 0.f);
        if (hi == 0 && valid) x = record_features(r, t, g, al, be);
        Act act;
        const float s = net_forward(net, x, act);
        if (g.scores && hi == 0) g.scores[tile * 32 + j] = valid ? s : 0.0f;
        if (!g.backward) continue;
        // d loss / d score (weighted binary cross-entropy with logits)
        // sigma(s) - 1 = -sigma(-s): both terms without cancellation
        const float y = (float)r.label;
        const float sig = 1.0f / (1.0f + expf(-s)), sign = 1.0f / (1.0f + expf(s));
        const float ds = valid ? (-g.pos_weight * y * sign + (1.0f - y) * sig) : 0.0f;
        if (hi == 0 && valid) {
            const float l1p = log1pf(expf(-fabsf(s)));
            aLoss += g.pos_weight * y * (l1p + fmaxf(-s, 0.0f)) + (1.0f - y) * (l1p + fmaxf(s, 0.0f));
            aCnt += 1.0f;
            aB3 += ds;
        }
        // layer 3 and the ReLU of layer 2
        bf16x4 d2[4];
        for (int q = 0; q < 16; q++) {
            const int row = row_of(q, l);
            const float h2 = fmaxf(act.pre2[q], 0.0f);
            const float dp2 = act.pre2[q] > 0.0f ? ds * net.w3[q] : 0.0f;
            const uint16_t dp2b = bf16_rne(dp2);
            sp2[row][j] = dp2;
            sh2[row][j] = h2;
            sh1[row][j] = bf16_f((uint16_t)act.h1[q >> 2][q & 3]);
            if ((q & 3) == 0) d2[q >> 2] = bf16x4{0, 0, 0, 0};
            d2[q >> 2][q & 3] = (short)dp2b;
        }
        // dh1 = W2^T dpre2 (MFMA, chained layout)
        f32x16 dh1 = {};
        for (int c = 0; c < 4; c++) dh1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(w2t[c], d2[c], dh1, 0, 0, 0);
        for (int q = 0; q < 16; q++) {
            const int row = row_of(q, l);
            sp1[row][j] = act.pre1[q] > 0.0f ? dh1[q] : 0.0f;
        }
        if (hi == 0) {
            sds[j] = ds;
            sx[0][j] = bf16_f((uint16_t)x[0]);
            sx[1][j] = bf16_f((uint16_t)x[1]);
            sx[2][j] = bf16_f((uint16_t)x[2]);
            sx[3][j] = bf16_f((uint16_t)x[3]);
        }
        __syncthreads();
        // dW2 += dpre2 h1^T: A[i][cand] = dpre2 (rounded), B[cand][k] = h1
        for (int c = 0; c < 4; c++) {
            const int k0 = 8 * c + 4 * hi;
            const bf16x4 A = pack4(sp2[j][k0], sp2[j][k0 + 1], sp2[j][k0 + 2], sp2[j][k0 + 3]);
            const bf16x4 B = pack4(sh1[j][k0], sh1[j][k0 + 1], sh1[j][k0 + 2], sh1[j][k0 + 3]);
            aW2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A, B, aW2, 0, 0, 0);
        }
        // row sums over the 32 candidates (fixed order)
        if (hi == 0) {
            float s1a = 0, s1b = 0, sb1 = 0, sw3 = 0;
            for (int c = 0; c < 32; c++) {
                s1a = __builtin_fmaf(sp1[j][c], sx[0][c], s1a);
                s1b = __builtin_fmaf(sp1[j][c], sx[1][c], s1b);
                sb1 += sp1[j][c];
                sw3 = __builtin_fmaf(sh2[j][c], sds[c], sw3);
            }
            aW1a += s1a; aW1b += s1b; aB += sb1; aW3 += sw3;
        } else {
            float s1c = 0, s1d = 0, sb2 = 0;
            for (int c = 0; c < 32; c++) {
                s1c = __builtin_fmaf(sp1[j][c], sx[2][c], s1c);
                s1d = __builtin_fmaf(sp1[j][c], sx[3][c], s1d);
                sb2 += sp2[j][c];
            }
            aW1a += s1c; aW1b += s1d; aB += sb2;
        }
        // d x1 of candidate j -> alpha_t, beta_t
        float dx1 = 0;
        for (int k = 0; k < 32; k++) dx1 = __builtin_fmaf(sp1[k][j], sw1c[k], dx1);
        float ga = 0, gb = 0;
        if (hi == 0 && valid) {
            ga = dx1 * (-(float)r.a / g.A);
            gb = dx1 * ((float)r.S / g.A);
        }
        for (int d = 16; d >= 1; d >>= 1) {
            ga += __shfl_xor(ga, d, 64);
            gb += __shfl_xor(gb, d, 64);
        }
        if (l == 0) {
            sab[0][t] += ga;
            sab[1][t] += gb;
        }
        __syncthreads();
    }
    if (!g.backward) return;  // forward only: no partials (g.partial may be null)
    // write this workgroup's partial gradient
    float *out = g.partial + (size_t)blockIdx.x * (g.P + 2);
    if (hi == 0) {
        out[O_W1 + j * 4 + 0] = aW1a;
        out[O_W1 + j * 4 + 1] = aW1b;
        out[O_B1 + j] = aB;
        out[O_W3 + j] = aW3;
    } else {
        out[O_W1 + j * 4 + 2] = aW1a;
        out[O_W1 + j * 4 + 3] = aW1b;
        out[O_B2 + j] = aB;
    }
    for (int q = 0; q < 16; q++) out[O_W2 + row_of(q, l) * H + j] = aW2[q];
    float b3 = aB3, ls = aLoss, cn = aCnt;
    for (int d = 32; d >= 1; d >>= 1) {
        b3 += __shfl_xor(b3, d, 64);
        ls += __shfl_xor(ls, d, 64);
        cn += __shfl_xor(cn, d, 64);
    }
    if (l == 0) {
        out[O_B3] = b3;
        out[g.P] = ls;
        out[g.P + 1] = cn;
    }
    for (int t = l; t < g.T; t += 64) {
        out[O_AL + t] = sab[0][t];
        out[O_AL + g.T + t] = sab[1][t];
    }
}

// sums the per-workgroup partials and divides by the number of valid
// records: out[0..P) gradient, out[P] loss, out[P+1] count.  A workgroup
// takes 64 consecutive entries (one per lane); its wavefront w adds the
// partials w, w + RED_W, w + 2 RED_W, ... in that order, and wavefront 0 then
// adds the RED_W sums in wavefront order: a fixed order, so the result does
// not depend on scheduling.  Sums in double precision.
constexpr int RED_W = 16;
__global__ __launch_bounds__(64 * RED_W) void reduce_kernel(const float *partial, int nparts, int P, float *out)
{
    __shared__ double acc_s[RED_W][64];
    __shared__ double cnt_s[RED_W];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const bool live = i < P + 2;
    double acc = 0.0, cnt = 0.0;
#pragma unroll 4
    for (int b = w; b < nparts; b += RED_W) {
        const float *row = partial + (size_t)b * (P + 2);
        if (live) acc += row[i];
        cnt += row[P + 1];
    }
    acc_s[w][lane] = acc;
    if (lane == 0) cnt_s[w] = cnt;
    __syncthreads();
    if (w == 0 && live) {
        double a = 0.0, c = 0.0;
        for (int v = 0; v < RED_W; v++) {
            a += acc_s[v][lane];
            c += cnt_s[v];
        }
        out[i] = (i == P + 1) ? (float)c : (float)(c > 0 ? a / c : 0.0);
    }
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int P, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {
int ilog2l(uint32_t v) { int r = 0; while ((1u << r) < v) r++; return r; }
void magic_l(uint32_t d, uint32_t *mag, uint32_t *mask)
{
    if (d <= 1) { *mag = 0; *mask = 0xFFFFFFFFu; return; }
    *mag = (uint32_t)(((1ULL << 32) + d - 1) / d);
    *mask = 0;
}
// r, s with x / d == (x * r) >> s for every x < limit, the product below 2^32
// and r below 2^24 (a full-rate 24-bit multiply); checked for every x
bool recip24(uint32_t d, uint32_t limit, uint32_t *r, uint32_t *s)
{
    for (int sh = 31; sh >= 0; sh--) {
        const uint64_t rr = ((1ull << sh) + d - 1) / d;
        if (rr >= (1u << 24) || (uint64_t)(limit - 1) * rr >= (1ull << 32)) continue;
        bool ok = true;
        for (uint32_t x = 0; x < limit && ok; x++) ok = (uint32_t)(((uint64_t)x * rr) >> sh) == x / d;
        if (!ok) continue;
        *r = (uint32_t)rr;
        *s = (uint32_t)sh;
        return true;
    }
    return false;
}
int check_lp(const fwbf_learned_params *lp)
{
    if (!lp) return fail(FWBF_E_INVALID, "null learned params");
    if (lp->rounds < 1 || lp->rounds > 64) return fail(FWBF_E_INVALID, "rounds must be in [1, 64]");
    if (lp->topk < 1 || lp->topk > 4 || (lp->topk & (lp->topk - 1)))
        return fail(FWBF_E_INVALID, "topk must be 1, 2 or 4");
    if (lp->groups < 1) return fail(FWBF_E_INVALID, "groups must be >= 1");
    if (lp->groups * lp->topk > 512) return fail(FWBF_E_INVALID, "groups * topk must be <= 512");
    if (!(lp->scale > 0.0f)) return fail(FWBF_E_INVALID, "scale must be > 0");
    return FWBF_OK;
}
}  // namespace

}  // namespace fwbf

using namespace fwbf;

extern "C" int fwbf_scorer_size(int rounds) { return rounds < 1 ? fail(FWBF_E_INVALID, "rounds must be >= 1") : 1249 + 2 * rounds; }

namespace fwbf {
namespace {
// The learned pass with one frame per workgroup, then plain FWBF (general
// kernel) for the frames it leaves with a nonzero syndrome.
int learned_wide(const fwbf_code *code, const fwbf_params *plain, const fwbf_learned_params *lp,
                 const float *scorer_dev, const void *y_dev, int64_t F, int64_t y_stride, uint32_t *z_dev,
                 int32_t *iters_dev, uint8_t *ok_dev, uint8_t *learned_ok_dev, fwbf_record *records_dev,
                 const uint32_t *pool_dev, int64_t pool_n, int64_t f0, hipStream_t st)
{
    WideArgs a;
    memset(&a, 0, sizeof a);
    a.p = (code->N + lp->groups - 1) / lp->groups;
    a.Geff = (code->N + a.p - 1) / a.p;
    a.k = lp->topk;
    a.NC = a.Geff * a.k;
    a.tpr = (lp->groups * lp->topk + 31) / 32;
    if (a.tpr > WIDE_T / 64) return fail(FWBF_E_UNSUPPORTED, "groups * topk must be <= 512");
    // the smallest C with L = 2^ceil(log2(ceil(p / C))) <= 64 lanes per block,
    // L * C >= 64 (the bank swizzle) and a thread for every (block, lane)
    int C = 0, L = 0;
    for (int cc : {8, 16, 32, 64}) {
        const int l = 1 << ilog2l((uint32_t)((a.p + cc - 1) / cc));
        if (l > 64 || cc * l < 64 || (int64_t)a.Geff * l > WIDE_T) continue;
        C = cc;
        L = l;
        break;
    }
    if (!C) return fail(FWBF_E_UNSUPPORTED, "blocks do not fit one workgroup of 1024 threads");
    a.L = L; a.logL = ilog2l(L); a.Lc = L * C; a.B = 64 / L;
    a.N = code->N; a.M = code->M; a.Z = code->Z; a.nb = code->nb;
    // bit and check indices stay below N; task indices below 3 Geff nb
    if (!recip24(a.Z, (uint32_t)code->N, &a.rZ, &a.sZ) || !recip24(a.p, (uint32_t)code->N, &a.rP, &a.sP) ||
        !recip24(a.nb, (uint32_t)(3 * a.Geff * a.nb), &a.rD, &a.sD))
        return fail(FWBF_E_UNSUPPORTED, "no exact 24-bit reciprocal for this code's sizes");
    a.T = lp->rounds;
    a.A = lp->scale;
    {
        int ex = 0;
        const float mant = std::frexp(lp->scale, &ex);
        a.invA = (mant == 0.5f && ex > -120 && ex < 120) ? std::ldexp(1.0f, 1 - ex) : 0.0f;
    }
    a.dv = 3.0f;
    int off = a.Geff * a.Lc * 4;  // slots at offset 0
    auto take = [&](int bytes, int align) { off = (off + align - 1) / align * align; int o = off; off += bytes; return o; };
    a.o_chk = take(4 * code->M, 4);
    a.o_chkp = take(code->M, 1);
    a.o_z = take(((code->N + 63) / 64) * 8, 8);
    a.o_syn = take(((code->M + 63) / 64) * 8, 8);
    a.o_cand = take(4 * 32 * a.tpr, 4);
    a.o_list = take(4 * 3 * a.Geff, 4);
    a.o_ctl = take(16, 4);
    a.o_sh = take(4 * 3 * code->nb, 4);
    a.o_net = take(4 * (96 + 64), 16);
    a.o_netw = take(64 * 5 * 8, 16);
    a.lds_bytes = (off + 15) / 16 * 16;
    if (a.lds_bytes > 160 * 1024) return fail(FWBF_E_UNSUPPORTED, "frame state exceeds 160 KiB of LDS");
    int rc = FWBF_OK;
    a.y = y_dev; a.F = F; a.stride = y_stride;
    a.z = z_dev; a.iters = iters_dev; a.ok = ok_dev; a.learned_ok = learned_ok_dev;
    a.rec = records_dev; a.pool = pool_dev; a.pool_n = pool_n; a.f0 = f0;
    a.params = scorer_dev;
    for (int t = 0; t < 3 * code->nb; t++) a.shv[t] = (uint16_t)code->shift[t];
    {
        const int esz = plain->dtype == FWBF_I8 ? 1 : 2;
        a.pref = ((uintptr_t)y_dev % 4 == 0) && ((y_stride * esz) % 4 == 0) &&
                 ((code->N * esz) % 4 == 0) && (code->N * esz / 4 <= 16 * WIDE_T);
    }
    auto launch = [&](auto kern) -> int {
        int blocks = 0, dev = 0, cus = 0;
        if (a.lds_bytes > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes);
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, WIDE_T, a.lds_bytes);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "learned decode occupancy");
        if (blocks < 1) return fail(FWBF_E_UNSUPPORTED, "learned kernel does not fit");
        const int64_t grid = std::min<int64_t>(F, (int64_t)blocks * cus);
        hipLaunchKernelGGL(kern, dim3((int)grid), dim3(WIDE_T), a.lds_bytes, st, a);
        e = hipGetLastError();
        return e == hipSuccess ? FWBF_OK : hip_fail(e, "learned decode launch");
    };
#define FWBF_WIDE(DT)                                                    \
    switch (C) {                                                         \
    case 8: rc = launch(learned_wide_kernel<DT, 8>); break;              \
    case 16: rc = launch(learned_wide_kernel<DT, 16>); break;            \
    case 32: rc = launch(learned_wide_kernel<DT, 32>); break;            \
    default: rc = launch(learned_wide_kernel<DT, 64>); break;            \
    }
    if (plain->dtype == FWBF_I8) { FWBF_WIDE(FWBF_I8) }
    else { FWBF_WIDE(FWBF_I16) }
#undef FWBF_WIDE
    if (rc) return rc;
    // plain FWBF from the original y for every frame the learned pass left
    // with a nonzero syndrome; its rounds add to the learned ones
    return decode_general(code, plain, y_dev, F, y_stride, z_dev, iters_dev, ok_dev, st, ok_dev);
}
}  // namespace
}  // namespace fwbf

extern "C" int fwbf_decode_learned(const fwbf_code *code, const fwbf_params *plain, const fwbf_learned_params *lp,
                                   const float *scorer_dev, const void *y_dev, int64_t F, int64_t y_stride,
                                   uint32_t *z_dev, int32_t *iters_dev, uint8_t *ok_dev, uint8_t *learned_ok_dev,
                                   fwbf_record *records_dev, const uint32_t *pool_dev, int64_t pool_n, int64_t f0,
                                   void *stream)
{
    int rc = check_lp(lp);
    if (rc) return rc;
    if (!code || !plain) return fail(FWBF_E_INVALID, "null code or params");
    if (plain->dtype != FWBF_I8 && plain->dtype != FWBF_I16)
        return fail(FWBF_E_UNSUPPORTED, "the learned decoder takes int8 or int16 inputs");
    if (code->mb != 3 || code->nb < 2 || code->nb > 32 || code->multi)
        return fail(FWBF_E_UNSUPPORTED, "the learned decoder covers bases of 3 block rows, 2..32 block columns "
                                        "and single shifts");
    for (int v : code->shift)
        if (v < 0) return fail(FWBF_E_UNSUPPORTED, "the learned decoder needs a full base (no zero blocks)");
    if (code->N > 65536) return fail(FWBF_E_UNSUPPORTED, "the learned decoder takes N <= 65536");
    if (plain->select != FWBF_GROUPS || plain->threads_per_frame != 0)
        return fail(FWBF_E_UNSUPPORTED, "the fallback must be plain FWBF (GROUPS)");
    if (F < 0 || y_stride < code->N || f0 < 0 || (pool_dev && pool_n < 1)) return fail(FWBF_E_INVALID, "invalid size");
    if (lp->groups > code->N) return fail(FWBF_E_INVALID, "groups must be <= N");
    if (F == 0) return FWBF_OK;
    if (!scorer_dev || !y_dev || !z_dev || !iters_dev || !ok_dev) return fail(FWBF_E_INVALID, "null buffer");
    const bool wave = plain->dtype == FWBF_I8 && code->nb == 6 && lp->groups * lp->topk <= 32 &&
                      !(plain->flags & FWBF_FLAG_GENERIC_KERNEL);
    if (!wave)
        return learned_wide(code, plain, lp, scorer_dev, y_dev, F, y_stride, z_dev, iters_dev, ok_dev, learned_ok_dev,
                            records_dev, pool_dev, pool_n, f0, (hipStream_t)stream);
    LearnArgs a;
    memset(&a, 0, sizeof a);
    a.p = (code->N + lp->groups - 1) / lp->groups;
    a.Geff = (code->N + a.p - 1) / a.p;
    a.k = lp->topk;
    if (a.Geff * a.k > 32) return fail(FWBF_E_UNSUPPORTED, "groups * topk must be <= 32");
    int C = 0, L = 0;
    for (int cc : {4, 8, 16, 32, 64}) {
        const int need = (a.p + cc - 1) / cc;
        const int l = 1 << ilog2l(need);
        if ((int64_t)a.Geff * l <= 64) { C = cc; L = l; break; }
    }
    if (!C)  // blocks too long for one wavefront: one frame per workgroup
        return learned_wide(code, plain, lp, scorer_dev, y_dev, F, y_stride, z_dev, iters_dev, ok_dev, learned_ok_dev,
                            records_dev, pool_dev, pool_n, f0, (hipStream_t)stream);
    a.L = L; a.logL = ilog2l(L);
    a.N = code->N; a.M = code->M; a.Z = code->Z; a.nb = code->nb;
    // a 24-bit reciprocal of Z that divides every bit index exactly (so for
    // Z <= 835, every code this kernel takes: N = 6Z <= 4096)
    // (exact for every n < N when (N - 1) (rZ24 Z - 2^22) < 2^22)
    a.rZ24 = (uint32_t)(((1u << 22) + code->Z - 1) / code->Z);
    if ((uint64_t)(code->N - 1) * ((uint64_t)a.rZ24 * code->Z - (1u << 22)) >= (1u << 22) ||
        (uint64_t)code->N * a.rZ24 >= (1ull << 32))
        return fail(FWBF_E_UNSUPPORTED, "block size too large for the learned kernel");
    magic_l(a.p, &a.magP, &a.maskP);
    a.T = lp->rounds;
    a.A = lp->scale;
    {
        int ex = 0;
        const float mant = std::frexp(lp->scale, &ex);
        a.invA = (mant == 0.5f && ex > -120 && ex < 120) ? std::ldexp(1.0f, 1 - ex) : 0.0f;
    }
    a.dv = 3.0f;
    int off = 0;
    auto take = [&](int bytes, int align) { off = (off + align - 1) / align * align; int o = off; off += bytes; return o; };
    a.o_net = take(4 * (96 + 64), 16);  // b1, b2, W3, then t / T for t < 64 rounds
    a.o_netw = take(64 * 5 * 8, 16);
    a.o_sh = take(4 * 3 * code->nb, 4);
    a.o_slot = take(2 * 2 * code->N, 4);
    a.o_wave0 = (off + 15) / 16 * 16;
    off = 64 * C * 4;  // slots, then the rest of one wavefront's frame state
    a.o_chk = take(4 * code->M, 4);
    a.o_y = take((code->N + 15) / 16 * 16, 16);
    a.o_z = take(((code->N + 63) / 64) * 8, 8);
    a.o_list = take(4 * 3 * a.Geff, 4);
    a.o_cand = take(16 * 32, 16);
    a.wave_bytes = (off + 15) / 16 * 16;
    a.lds_bytes = a.o_wave0 + LEARN_WAVES * a.wave_bytes;
    if (a.lds_bytes > 160 * 1024) return fail(FWBF_E_UNSUPPORTED, "frame state exceeds 160 KiB of LDS");
    DeviceTables tb;
    rc = device_tables(const_cast<fwbf_code *>(code), &tb);
    if (rc) return rc;
    a.y = (const int8_t *)y_dev; a.F = F; a.stride = y_stride;
    a.vec_ok = (((uintptr_t)y_dev & 15) == 0) && (y_stride % 16 == 0);
    a.z = z_dev; a.iters = iters_dev; a.ok = ok_dev; a.learned_ok = learned_ok_dev;
    a.rec = records_dev; a.pool = pool_dev; a.pool_n = pool_n; a.f0 = f0;
    a.params = scorer_dev; a.shift = tb.shift;
    hipStream_t st = (hipStream_t)stream;
    auto launch = [&](auto kern) -> int {
        int blocks = 0, dev = 0, cus = 0;
        if (a.lds_bytes > 65536)
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_bytes);
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, 64 * LEARN_WAVES, a.lds_bytes);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "learned decode occupancy");
        if (blocks < 1) return fail(FWBF_E_UNSUPPORTED, "learned kernel does not fit");
        const int64_t grid = std::min<int64_t>((F + LEARN_WAVES - 1) / LEARN_WAVES, (int64_t)blocks * cus);
        hipLaunchKernelGGL(kern, dim3((int)grid), dim3(64 * LEARN_WAVES), a.lds_bytes, st, a);
        e = hipGetLastError();
        return e == hipSuccess ? FWBF_OK : hip_fail(e, "learned decode launch");
    };
    switch (C) {
    case 4: rc = launch(learned_kernel<3, 6, 4>); break;
    case 8: rc = launch(learned_kernel<3, 6, 8>); break;
    case 16: rc = launch(learned_kernel<3, 6, 16>); break;
    case 32: rc = launch(learned_kernel<3, 6, 32>); break;
    default: rc = launch(learned_kernel<3, 6, 64>); break;
    }
    if (rc) return rc;
    // plain FWBF from the original y for every frame the learned pass left
    // with a nonzero syndrome; its rounds add to the learned ones
    rc = try_fast_decode(code, plain, y_dev, F, y_stride, z_dev, iters_dev, ok_dev, st, tb.shift, ok_dev, 1);
    if (rc == 0) return fail(FWBF_E_UNSUPPORTED, "no fallback kernel for these parameters");
    return rc < 0 ? rc : FWBF_OK;
}

namespace fwbf {
namespace {
constexpr int GRAD_PARTS = 1024;  // workgroups of grad_kernel = partial gradient rows

// Forward / backward over n_tiles tiles into `partial` (GRAD_PARTS rows of
// P + 2 floats, every entry written by the kernel), then the fixed-order
// reduction into out_dev.
int launch_grad(const fwbf_record *records_dev, int64_t n_tiles, const fwbf_learned_params *lp,
                const float *scorer_dev, float pos_weight, float *out_dev, float *scores_dev, float *partial,
                hipStream_t st)
{
    const int P = 1249 + 2 * lp->rounds;
    GradArgs g;
    g.rec = records_dev; g.n_tiles = n_tiles; g.params = scorer_dev;
    g.pos_weight = pos_weight; g.A = lp->scale; g.dv = 3.0f;
    g.T = lp->rounds; g.P = P;
    g.tpr = (lp->groups * lp->topk + 31) / 32;
    g.partial = partial; g.scores = scores_dev; g.backward = out_dev != nullptr;
    hipLaunchKernelGGL(grad_kernel, dim3(GRAD_PARTS), dim3(64), 0, st, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "scorer gradient launch");
    if (out_dev) {
        hipLaunchKernelGGL(reduce_kernel, dim3((P + 2 + 63) / 64), dim3(64 * RED_W), 0, st, partial, GRAD_PARTS, P,
                           out_dev);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "gradient reduction launch");
    }
    return FWBF_OK;
}

int check_grad_args(const fwbf_record *records_dev, int64_t n_tiles, const fwbf_learned_params *lp,
                    const float *scorer_dev, const float *out_dev, const float *scores_dev)
{
    int rc = check_lp(lp);
    if (rc) return rc;
    if (n_tiles < 0) return fail(FWBF_E_INVALID, "n_tiles must be >= 0");
    if (!scorer_dev || (!out_dev && !scores_dev)) return fail(FWBF_E_INVALID, "null buffer");
    if (n_tiles > 0 && !records_dev) return fail(FWBF_E_INVALID, "null records");
    return FWBF_OK;
}

}  // namespace
}  // namespace fwbf

extern "C" int fwbf_scorer_grad(const fwbf_record *records_dev, int64_t n_tiles, const fwbf_learned_params *lp,
                                const float *scorer_dev, float pos_weight, float *out_dev, float *scores_dev,
                                float *workspace_dev, int64_t workspace_floats, void *stream)
{
    int rc = check_grad_args(records_dev, n_tiles, lp, scorer_dev, out_dev, scores_dev);
    if (rc) return rc;
    const int P = 1249 + 2 * lp->rounds;
    if (out_dev && (!workspace_dev || workspace_floats < (int64_t)GRAD_PARTS * (P + 2)))
        return fail(FWBF_E_INVALID, "workspace too small (need 1024 * (P + 2) floats)");
    return launch_grad(records_dev, n_tiles, lp, scorer_dev, pos_weight, out_dev, scores_dev, workspace_dev,
                       (hipStream_t)stream);
}

extern "C" int fwbf_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, int P, int step,
                         float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!params_dev || !grad_dev || !m_dev || !v_dev || P < 1 || step < 1) return fail(FWBF_E_INVALID, "invalid argument");
    // bias corrections 1 - beta^step of the single-precision betas, formed
    // in double: in float, 1 - powf(0.999f, t) loses ~1e-5 to cancellation
    const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3((P + 255) / 256), dim3(256), 0, (hipStream_t)stream, params_dev, grad_dev,
                       m_dev, v_dev, P, lr, beta1, beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FWBF_OK : hip_fail(e, "adam launch");
}
