/*
 * fwbf.h -- C ABI of libfwbf.so, an MI355X (gfx950) implementation of fast
 * weighted bit-flipping (FWBF) decoding of LDPC codes (Ma, Li, Zhu, Zhang,
 * Qi, "An Improved WBF Algorithm for Higher-Speed Decoding of LDPC Codes").
 *
 * Conventions shared by every entry point:
 *   - Return value: FWBF_OK (0) on success, a negative FWBF_E_* code
 *     otherwise; fwbf_last_error() then returns a message (thread-local,
 *     valid until the next call on the same thread).  Arguments are checked
 *     before anything is enqueued: a call that fails enqueues nothing.
 *   - "_dev" pointers are device memory on the current HIP device, owned by
 *     the caller (e.g. torch tensors); "_host" pointers are host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Device work is enqueued asynchronously on it and ordered with the
 *     caller's other work on that stream; nothing synchronises unless stated.
 *   - Packed hard decisions / codewords: bit n of a frame sits in 32-bit
 *     word n/32 at bit position n%32; padding bits of the last word are 0.
 *   - fwbf_code objects are created and freed by the library, immutable
 *     after creation and shareable across threads and streams.
 */
#ifndef FWBF_H
#define FWBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWBF_OK 0
#define FWBF_E_INVALID (-1)     /* null pointer, out-of-range size or parameter */
#define FWBF_E_PARSE (-2)       /* malformed code description */
#define FWBF_E_GIRTH (-3)       /* no draw met the girth constraint */
#define FWBF_E_UNSUPPORTED (-4) /* parameters outside what the kernels handle */
#define FWBF_E_NOMEM (-5)       /* host or device allocation failed */
#define FWBF_E_HIP (-6)         /* HIP runtime or launch error */

/* received-value type: float, or fixed point (int8 / int16) */
enum { FWBF_F32 = 0, FWBF_I8 = 1, FWBF_I16 = 2 };
/* check reliability: WBF (minimum over N(m), no alpha term), MWBF (same
 * minimum, minus alpha|y_n|), IMWBF (minimum over N(m)\n, eq. (1)) */
enum { FWBF_WBF = 0, FWBF_MWBF = 1, FWBF_IMWBF = 2 };
/* bit choice: GROUPS = FWBF (at most one flip per block, if its metric is
 * > 0; Section III, Step 2; block g = bits [g p, (g+1) p)), SINGLE = largest
 * metric flipped unconditionally (IMWBF rule after eq. (1)), TOPL = the
 * lambda largest positive metrics (the multi-bit choice of MLP-WBF,
 * Section III), STRIDED = GROUPS with block g = {n : n mod G = g} (the
 * blocks that an interleaver of depth G makes contiguous, Section III) */
enum { FWBF_GROUPS = 0, FWBF_SINGLE = 1, FWBF_TOPL = 2, FWBF_STRIDED = 3 };

/* flags */
#define FWBF_FLAG_NO_CYCLE_EXIT 1u /* run every round up to max_iter even after
                                      the state repeats (for verification) */
#define FWBF_FLAG_GENERIC_KERNEL 2u /* use the general kernel even where the
                                       specialised one applies (verification) */
#define FWBF_FLAG_SPECIALISED_ONLY 4u /* fail with FWBF_E_UNSUPPORTED (enqueue
                                         nothing) unless a one-wave specialised
                                         kernel (regular full-base codes with
                                         fixed-point inputs, or single
                                         circulants) takes the call: lets a
                                         test pin the kernel it exercises */
#define FWBF_FLAG_EXECUTED_ROUNDS 8u /* diagnostic: iters_dev receives, for a
                                        frame whose state repeats (a round
                                        with no flip, or with the previous
                                        round's flips), the rounds run before
                                        that round instead of the equivalent
                                        max_iter; z and ok are unchanged */

typedef struct fwbf_code fwbf_code;

/* Decoder parameters (eq. (1) and Section III). */
typedef struct {
    int32_t dtype;     /* FWBF_F32 / FWBF_I8 / FWBF_I16 */
    int32_t weights;   /* FWBF_WBF / FWBF_MWBF / FWBF_IMWBF */
    int32_t select;    /* FWBF_GROUPS / FWBF_SINGLE / FWBF_TOPL / FWBF_STRIDED */
    int32_t groups;    /* G: number of blocks (GROUPS, STRIDED), 1 <= G <= N;
                          block length p = ceil(N/G) */
    int32_t lambda;    /* TOPL: flips per round, >= 1 */
    int32_t max_iter;  /* K_max: maximum number of flip rounds, >= 0 */
    float alpha;       /* F32: alpha of eq. (1) (ignored for WBF) */
    int32_t alpha_num; /* I8/I16: alpha = alpha_num / alpha_den (>= 0, > 0) */
    int32_t alpha_den;
    int32_t threads_per_frame; /* 0 = automatic (by N; doubled when the
                                  whole batch fits on the device at once at
                                  the doubled width); else 64, 128, 256, 512
                                  or 1024 */
    uint32_t flags;            /* FWBF_FLAG_* */
} fwbf_params;

/* ---- codes (Section II: H, M(n), N(m), RC constraint) ------------------- */

/* Parse a QC description:
 *     qc-ldpc v1
 *     Z <circulant size>
 *     base <mb> <nb>
 *     <mb rows of nb shifts>
 * Shift s >= 0 is the Z x Z permutation taking row r to column (r+s) mod Z;
 * -1 is the zero block.  '#' starts a comment.  N = nb Z, M = mb Z.
 * Limits: 1 <= Z <= 65535, N <= 65535, every row and column of the base
 * with at most 64 nonzero blocks.  *out is owned by the caller and released
 * with fwbf_code_free.  FWBF_E_PARSE on malformed text. */
int fwbf_code_from_text(const char *text, fwbf_code **out);

/* Seeded draw of an mb x nb base of circulant permutations: shifts drawn
 * row-major as SplitMix64(seed) mod Z; with min_girth = 6 the whole base is
 * redrawn (continuing the stream) until no 4-cycle exists, i.e. the RC
 * constraint holds.  min_girth must be 4 (no check) or 6.  FWBF_E_GIRTH
 * after 100000 rejected draws. */
int fwbf_code_from_seed(int mb, int nb, int Z, uint64_t seed, int min_girth, fwbf_code **out);

/* Canonical text of a code.  Writes at most `cap` bytes including the NUL;
 * *needed (if not NULL) receives the full length including the NUL.
 * FWBF_E_INVALID if cap is too small (nothing written then). */
int fwbf_code_to_text(const fwbf_code *code, char *buf, size_t cap, size_t *needed);

/* Dimensions; any output pointer may be NULL.  K = N - rank_GF2(H) (the
 * rank is computed on first request and cached). */
int fwbf_code_dims(const fwbf_code *code, int *N, int *M, int *K, int *dv_max, int *dc_max);

/* Base shifts, row-major mb x nb (-1 = zero block); also returns mb, nb, Z. */
int fwbf_code_shifts(const fwbf_code *code, int *mb, int *nb, int *Z, int *shifts_host);

/* 1 if H violates the RC constraint (has a 4-cycle), else 0. */
int fwbf_code_has_4cycle(const fwbf_code *code);

void fwbf_code_free(fwbf_code *code);

/* ---- encoder (Section II: codewords are the null space of H) ----------- */

/* Info positions: the K non-pivot columns of the reduced row-echelon form
 * of H over GF(2), ascending (out_host holds K ints). */
int fwbf_code_info_positions(const fwbf_code *code, int *out_host);

/* Codewords first .. first+count-1 of the seeded pool, packed, into
 * out_host[count][ceil(N/32)].  Info bit k of codeword w is bit k%64 of
 * SplitMix64 output number w*ceil(K/64) + k/64 of the stream seeded with
 * `seed`; parity bits follow from H c = 0.  Host-side, synchronous. */
int fwbf_encode(const fwbf_code *code, uint64_t seed, int64_t first, int64_t count,
                uint32_t *out_host);

/* ---- channel (Section II BPSK, Section V AWGN) ------------------------- */

/* Received frames f0 .. f0+F-1 into y_dev[F][y_stride] (y_stride >= N):
 * y = (1 - 2c) + sigma g, c = pool_dev row (f % pool_n) (pool_dev NULL:
 * all-zero codeword), g standard normal from Philox4x32-10 keyed by `seed`,
 * counter (n/4, f low, f high, stream_id), Box-Muller over pairs of words
 * (u = ((x >> 9) + 1/2) 2^-23, exact in single precision; cosine member for even n, sine for odd).
 * sigma_dev (F floats, may be NULL) overrides `sigma` per frame.
 * dtype F32 stores y; I8 / I16 store clamp(rint(scale y), -127/-32767,
 * 127/32767).  Single-precision arithmetic. */
int fwbf_channel(int N, int64_t F, int64_t f0, const uint32_t *pool_dev, int64_t pool_n,
                 uint64_t seed, uint32_t stream_id, float sigma, const float *sigma_dev,
                 float scale, int dtype, void *y_dev, int64_t y_stride, void *stream);

/* ---- decoding (eq. (1), Section III) ------------------------------------ */

/* Decode F frames y_dev[F][y_stride] (element type per params->dtype).
 * Outputs: z_dev[F][ceil(N/32)] packed hard decisions z_k, iters_dev[F]
 * the number of flip rounds run (0..max_iter), ok_dev[F] = 1 iff the final
 * syndrome is zero.  The result is a deterministic function of (H, y,
 * params): a decoder state that repeats (no flip, or the same flips as the
 * round before) is followed to max_iter analytically, so outputs equal those
 * of running every round.  F = 0 is a no-op. */
int fwbf_decode(const fwbf_code *code, const fwbf_params *params, const void *y_dev, int64_t F,
                int64_t y_stride, uint32_t *z_dev, int32_t *iters_dev, uint8_t *ok_dev,
                void *stream);

/* ---- min-sum belief propagation (the BP reference of Sections I, V) ----- */

/* Flooding min-sum with R_{m,n} = (product of the other members' signs of
 * Q) r(minimum of the other members' |Q|), Q_{n,m} = P_n - R_{m,n},
 * P_n = y_n + sum over M(n) of R_{m,n} in ascending check order, z = [P < 0];
 * r(x) = c x (offset = 0, normalised) or max(x - c, 0) (offset = 1).
 * The paper names BP and its normalised and offset forms without equations;
 * this is the textbook schedule, single precision. */
typedef struct {
    int32_t offset;            /* 0: normalised, 1: offset */
    float c;                   /* normalisation factor or offset, finite, >= 0 */
    int32_t max_iter;          /* iterations, >= 0 */
    int32_t threads_per_frame; /* 0 = automatic; else 64, 128, 256, 512 or 1024 */
} fwbf_minsum_params;

/* Decode F float frames y_dev[F][y_stride]: z_dev[F][ceil(N/32)] packed hard
 * decisions, iters_dev[F] iterations run (0 when [y < 0] satisfies H),
 * ok_dev[F] = 1 iff the final syndrome is zero.  Any code (the kernels keep
 * one frame per workgroup in LDS: FWBF_E_UNSUPPORTED beyond 160 KiB).
 * Stream-ordered; F = 0 is a no-op. */
int fwbf_decode_minsum(const fwbf_code *code, const fwbf_minsum_params *params, const float *y_dev,
                       int64_t F, int64_t y_stride, uint32_t *z_dev, int32_t *iters_dev, uint8_t *ok_dev,
                       void *stream);

/* One decode job of a mixed-code batch (buffers as for fwbf_decode). */
typedef struct {
    const fwbf_code *code;
    const fwbf_params *params; /* all items share params->dtype */
    const void *y_dev;
    int64_t F, y_stride;
    uint32_t *z_dev;
    int32_t *iters_dev;
    uint8_t *ok_dev;
} fwbf_batch_item;

/* Decodes the frames of up to 8 items (each with its own code and
 * parameters) in one persistent launch: workgroups claim frames one at a
 * time from a ticket counter in workspace_dev (>= 256 bytes of device
 * memory, owned by the caller, reset by the call), so frames that finish
 * early free their workgroup for the next unclaimed frame of any item.
 * Results are those of fwbf_decode on each item (the general kernel).
 * threads_per_frame: 0 = automatic (the largest code decides), else 64..1024;
 * blocks_per_cu: 0 = as many as fit, else an upper bound.  Concurrent calls
 * must use distinct workspaces. */
int fwbf_decode_batched(const fwbf_batch_item *items, int n_items, int threads_per_frame, int blocks_per_cu,
                        void *workspace_dev, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Decodes as
 * fwbf_decode_batched does (same kernel, same results, same argument
 * checks), but calls no hipMalloc, hipFree or other allocating routine:
 *  - the ticket counter lives in a library-owned device array of 256 bytes
 *    (one copy per device, held until the process ends); the call needs 8
 *    of them whatever the batch, so no input size can exceed it;
 *  - the first call on a device looks up that device's copy
 *    (hipGetSymbolAddress) with the device current;
 *  - every item's code must already have its tables on the current device,
 *    uploaded by an earlier allocating call with that code there
 *    (fwbf_decode or fwbf_decode_batched); otherwise FWBF_E_INVALID and
 *    nothing is enqueued.
 * The counter is cleared by a kernel at the start of each call (no memset
 * node).  All calls on one device share its array: calls that overlap on
 * one device (other streams or host threads) race on the counter and must
 * be serialised by the caller. */
int fwbf_decode_batched_noalloc(const fwbf_batch_item *items, int n_items, int threads_per_frame,
                                int blocks_per_cu, void *stream);

/* ---- error accounting (Section V) --------------------------------------- */

/* Adds, for frames f0 .. f0+F-1 against pool row (f % pool_n) (pool NULL:
 * all-zero codeword), into counters_dev (int64, max_iter + 7 entries):
 * [0] bit errors, [1] frame errors, [2] undetected frame errors (ok = 1 but
 * z != c), [3] sum of rounds, [4] frames, [5] frames with ok = 1,
 * [6 .. 6+max_iter] histogram of rounds.  Counters are accumulated, not
 * cleared. */
int fwbf_count(int N, int64_t F, int64_t f0, const uint32_t *z_dev, const uint32_t *pool_dev,
               int64_t pool_n, const int32_t *iters_dev, const uint8_t *ok_dev, int max_iter,
               int64_t *counters_dev, void *stream);

/* ---- Eb/N0 sweep in one HIP graph ---------------------------------------- */

typedef struct fwbf_sweep fwbf_sweep;

/* Records, for each of n_points noise levels sigma_host[i], frame generation
 * (fwbf_channel with stream_id i, frames 0 .. frames_per_point-1) ->
 * fwbf_decode -> fwbf_count into one HIP graph, instantiated for the
 * current device.  The sweep owns its frame, output and counter buffers,
 * one set of frames and outputs per point (n_points * frames_per_point
 * frames in all; counters cleared by a kernel at the start of every replay,
 * never by a memset node).  pool_dev must stay valid while the sweep is
 * used. */
int fwbf_sweep_create(const fwbf_code *code, const fwbf_params *params, const float *sigma_host, int n_points,
                      int64_t frames_per_point, const uint32_t *pool_dev, int64_t pool_n, uint64_t seed,
                      float scale, fwbf_sweep **out);
/* Replays the whole sweep on `stream` (one graph launch). */
int fwbf_sweep_launch(fwbf_sweep *sweep, void *stream);
/* Copies the counters (n_points x (max_iter + 7) int64, layout of
 * fwbf_count) to host memory after the work queued on `stream`; waits. */
int fwbf_sweep_counters(fwbf_sweep *sweep, int64_t *counters_host, void *stream);
/* Copies point `point`'s received frames (y_dev: [frames_per_point][N] of
 * the sweep's dtype) and the decoder outputs of the last replay (layouts of
 * fwbf_decode) into caller device buffers, stream-ordered after the work on
 * `stream`; any destination may be NULL. */
int fwbf_sweep_outputs(const fwbf_sweep *sweep, int point, void *y_dev, uint32_t *z_dev, int32_t *iters_dev,
                       uint8_t *ok_dev, void *stream);
void fwbf_sweep_free(fwbf_sweep *sweep);

/* ---- learned flip scorer (extension; keeps the per-block choice) -------- */

/* The learned pass: in round t (t < rounds) the metric
 * E_t = fmaf(-alpha_t, |y_n|, beta_t S_n), with S_n the check sum of eq. (1),
 * proposes the `topk` best bits of each of `groups` blocks (Section III);
 * a ReLU network 4 -> 32 -> 32 -> 1 (bfloat16 weights, MFMA, single-precision
 * sums) scores each proposal from [|y|/scale, E_t/scale, u_n/dv, t/rounds]
 * (u_n: unsatisfied checks of bit n) and, in each block, the best-scoring
 * proposal is flipped if its score is positive.  The pass stops on a zero
 * syndrome, on a round without flips, on a round repeating the previous
 * round's flips, or after `rounds` rounds.  Scorer parameters: float32
 * vector of fwbf_scorer_size(rounds) = 1249 + 2*rounds values:
 * W1[32][4], b1[32], W2[32][32], b2[32], W3[32], b3, alpha[rounds],
 * beta[rounds]. */
typedef struct {
    int32_t rounds; /* 1..64 */
    int32_t groups; /* blocks of the learned pass; groups * topk <= 512 */
    int32_t topk;   /* proposals per block: 1, 2 or 4 */
    float scale;    /* fixed-point scale of y (16 for int8, 256 for int16 inputs) */
} fwbf_learned_params;

/* Proposal slots per round in the record layout: 32 * ceil(groups * topk /
 * 32), i.e. whole tiles of 32 (one tile when groups * topk <= 32). */
#define FWBF_RECORD_SLOTS(groups, topk) (32 * (((groups) * (topk) + 31) / 32))

/* One scored proposal, emitted by fwbf_decode_learned for training:
 * records[frame][round][slot], slot = block * topk + rank, with
 * FWBF_RECORD_SLOTS(groups, topk) slots per round (12 bytes each). */
typedef struct {
    int32_t S;      /* check sum S_n of eq. (1) when scored */
    uint16_t a;     /* |y_n| */
    uint16_t n;     /* bit index (codes with N <= 65536) */
    uint8_t u;      /* unsatisfied checks of bit n */
    uint8_t label;  /* z_n xor c_n when scored: 1 if the bit is wrong */
    uint8_t valid;  /* 0 for empty slots and rounds not run */
    uint8_t pad;
} fwbf_record;

/* Number of scorer parameters for `rounds` rounds (or a negative error). */
int fwbf_scorer_size(int rounds);

/* Learned decoding, then plain FWBF (params `plain`: FWBF_GROUPS, same
 * dtype) from the original y for every frame whose syndrome is still
 * nonzero; such frames report the learned rounds plus the plain rounds.
 * Codes: a full base (no zero blocks) of single circulant shifts with column
 * weight 3 and N <= 65536; inputs int8 or int16 (plain->dtype).  int8 frames
 * of (3,6) codes whose proposals fit one tile (groups * topk <= 32) run one
 * frame per wavefront; every other case (and any call with
 * FWBF_FLAG_GENERIC_KERNEL in plain->flags) runs one frame per workgroup of
 * 1024 threads, with groups * topk <= 512 and the frame state within
 * 160 KiB of LDS (N = 32400 fits).  Outputs as fwbf_decode; learned_ok_dev
 * (optional, F bytes) receives 1 for frames decoded by the learned pass
 * alone.  records_dev (optional, F * rounds * FWBF_RECORD_SLOTS(groups,
 * topk) records) receives the proposals; labels compare with pool_dev row
 * ((f0 + f) % pool_n) (NULL: all-zero codeword).  scorer_dev: device
 * float32 parameters, read only. */
int fwbf_decode_learned(const fwbf_code *code, const fwbf_params *plain, const fwbf_learned_params *lp,
                        const float *scorer_dev, const void *y_dev, int64_t F, int64_t y_stride,
                        uint32_t *z_dev, int32_t *iters_dev, uint8_t *ok_dev, uint8_t *learned_ok_dev,
                        fwbf_record *records_dev, const uint32_t *pool_dev, int64_t pool_n, int64_t f0,
                        void *stream);

/* Scorer forward and backward over n_tiles tiles of 32 records (records laid
 * out as emitted: tile index = (frame * rounds + round) * tiles_per_round +
 * tile of the round, tiles_per_round = ceil(groups * topk / 32)).  scores_dev
 * (optional, n_tiles * 32 floats) receives the scores.  out_dev (optional,
 * P + 2 floats) receives the gradient of the mean weighted binary
 * cross-entropy with logits over the valid records (positives weighted by
 * pos_weight), then the mean loss and the number of valid records; the sum
 * over records runs per workgroup and then over workgroups in a fixed
 * order, so results do not depend on scheduling.  workspace_dev: at least
 * 1024 * (P + 2) floats when out_dev is given. */
int fwbf_scorer_grad(const fwbf_record *records_dev, int64_t n_tiles, const fwbf_learned_params *lp,
                     const float *scorer_dev, float pos_weight, float *out_dev, float *scores_dev,
                     float *workspace_dev, int64_t workspace_floats, void *stream);

/* One Adam step (Kingma & Ba) on P float32 parameters: moments m, v updated
 * in place, bias correction for step number `step` (>= 1). */
int fwbf_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, int P, int step, float lr,
              float beta1, float beta2, float eps, void *stream);

/* ---- misc ---------------------------------------------------------------- */

const char *fwbf_last_error(void);
const char *fwbf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FWBF_H */
