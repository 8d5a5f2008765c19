/*
 * fwbf_oracle.c -- CPU oracle for fast weighted bit-flipping (FWBF) decoding
 * of LDPC codes (Ma, Li, Zhu, Zhang, Qi, "An Improved WBF Algorithm for
 * Higher-Speed Decoding of LDPC Codes").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or constant
 * generator with the HIP library; the two sides only agree on the published
 * definitions they both implement (the QC description text, SplitMix64,
 * Philox4x32-10, reduced row-echelon form over GF(2)).
 *
 * Everything here is written in its most literal form: the parity-check
 * matrix is materialised as adjacency lists, the check reliabilities are
 * computed by an explicit minimum loop over each check's neighbours, the
 * syndrome is recomputed from scratch every round, every metric is
 * recomputed every round, and the group maxima are found by a plain scan.
 * No incremental update, packed key, stall shortcut or other optimisation of
 * the GPU path appears here.
 *
 * Readings adopted where the paper is silent:
 *   - rounds: at most K_max flip rounds; stop as soon as the syndrome is zero
 *     (Section III, Step 1 together with the definition of z_k in Section II);
 *   - z_0,n = 1 iff y_n < 0 (Section III, Initialization; sgn(0) taken as +);
 *   - blocks: p = ceil(N/G), block g covers [g p, min(N,(g+1)p)), the short
 *     last block stands for the paper's "null" metric padding (footnote 1);
 *     the strided variant takes block g = {n : n mod G = g} instead (the
 *     blocks an interleaver of depth G would make contiguous, Section III);
 *   - all blocks choose from the same syndrome (one syndrome per round);
 *   - ties are broken by the lowest bit index;
 *   - GROUPS/TOPL flip only if the metric is > 0 (Section III, Step 2),
 *     SINGLE flips the global maximum unconditionally (Section II, after
 *     eq. (1));
 *   - WBF and MWBF use the check minimum over all of N(m) (Section I names
 *     them; standard published definitions), WBF has no alpha term;
 *   - integer inputs use a rational alpha = a_num / a_den and the scaled
 *     metric a_den*S - a_num*|y| (exact, order-equivalent to eq. (1));
 *   - float inputs: S summed over M(n) in ascending check order starting from
 *     the first term, E = fmaf(-alpha, |y|, S) (single precision: the float
 *     metric decides an argmax, so it is taken in the kernel's precision).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EPARSE (-2)
#define OR_EGIRTH (-3)
#define OR_ENOMEM (-4)

enum { W_WBF = 0, W_MWBF = 1, W_IMWBF = 2 };
enum { S_GROUPS = 0, S_SINGLE = 1, S_TOPL = 2, S_STRIDED = 3 };
enum { D_F32 = 0, D_I8 = 1, D_I16 = 2 };

typedef struct {
    int Z, mb, nb;
    int *shift; /* mb*nb: first shift of each block, -1 = all-zero block */
    int nent;   /* circulant permutations: (block row, block column, shift) */
    int *ent;
    int N, M;
    int *row_ptr, *row_bits; /* N(m), ascending bit index */
    int *col_ptr, *col_chks; /* M(n), ascending check index */
    /* GF(2) reduced row-echelon form of H (computed on demand) */
    int have_rref;
    int rank, K, words;
    uint64_t *rref; /* rank rows of `words` 64-bit words */
    int *piv_col;   /* pivot column of each rref row */
    int *info_pos;  /* K non-pivot columns, ascending */
} ocode;

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014): state advances by the golden-ratio */
/* increment, the output is the variant-13 finaliser of the new state.      */
/* ------------------------------------------------------------------------ */
static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static uint64_t sm64_next(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ULL;
    return sm64_mix(*state);
}
/* the idx-th output (0-based) of a SplitMix64 stream started at `seed` */
static uint64_t sm64_at(uint64_t seed, uint64_t idx)
{
    return sm64_mix(seed + (idx + 1) * 0x9E3779B97F4A7C15ULL);
}

uint64_t or_splitmix64(uint64_t seed, uint64_t idx) { return sm64_at(seed, idx); }

/* ------------------------------------------------------------------------ */
/* Code construction: QC description -> materialised Tanner adjacency.      */
/* Block (i,j) with shift s >= 0 is the Z x Z permutation taking row r to   */
/* column (r + s) mod Z; shift -1 is the zero block; a list of distinct      */
/* shifts is the sum of their permutations (a circulant of that weight).    */
/* Section II defines M(n) and N(m) as the positions of ones in column n    */
/* and row m of H.                                                          */
/* ------------------------------------------------------------------------ */
static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static void code_release(ocode *c)
{
    if (!c) return;
    free(c->shift);
    free(c->ent);
    free(c->row_ptr); free(c->row_bits);
    free(c->col_ptr); free(c->col_chks);
    free(c->rref); free(c->piv_col); free(c->info_pos);
    free(c);
}
void or_code_free(ocode *c) { code_release(c); }

/* ent: nent triples (i, j, s) */
static ocode *code_build(int mb, int nb, int Z, int nent, const int *ent)
{
    ocode *c = (ocode *)calloc(1, sizeof(ocode));
    if (!c) return NULL;
    c->Z = Z; c->mb = mb; c->nb = nb;
    c->N = nb * Z; c->M = mb * Z;
    c->nent = nent;
    c->shift = (int *)malloc(sizeof(int) * mb * nb);
    c->ent = (int *)malloc(sizeof(int) * 3 * (nent ? nent : 1));
    c->row_ptr = (int *)calloc(c->M + 1, sizeof(int));
    c->col_ptr = (int *)calloc(c->N + 1, sizeof(int));
    if (!c->shift || !c->ent || !c->row_ptr || !c->col_ptr) { code_release(c); return NULL; }
    memcpy(c->ent, ent, sizeof(int) * 3 * nent);
    for (int t = 0; t < mb * nb; t++) c->shift[t] = -1;
    for (int e = nent - 1; e >= 0; e--) c->shift[ent[3 * e] * nb + ent[3 * e + 1]] = ent[3 * e + 2];

    /* count the ones of every row and column of H */
    for (int e = 0; e < nent; e++) {
        int i = ent[3 * e], j = ent[3 * e + 1], sh = ent[3 * e + 2];
        for (int r = 0; r < Z; r++) {
            int m = i * Z + r, n = j * Z + (r + sh) % Z;
            c->row_ptr[m + 1]++;
            c->col_ptr[n + 1]++;
        }
    }
    for (int m = 0; m < c->M; m++) c->row_ptr[m + 1] += c->row_ptr[m];
    for (int n = 0; n < c->N; n++) c->col_ptr[n + 1] += c->col_ptr[n];
    int E = c->row_ptr[c->M];
    c->row_bits = (int *)malloc(sizeof(int) * (E ? E : 1));
    c->col_chks = (int *)malloc(sizeof(int) * (E ? E : 1));
    int *rfill = (int *)calloc(c->M, sizeof(int));
    int *cfill = (int *)calloc(c->N, sizeof(int));
    if (!c->row_bits || !c->col_chks || !rfill || !cfill) {
        free(rfill); free(cfill); code_release(c); return NULL;
    }
    for (int e = 0; e < nent; e++) {
        int i = ent[3 * e], j = ent[3 * e + 1], sh = ent[3 * e + 2];
        for (int r = 0; r < Z; r++) {
            int m = i * Z + r, n = j * Z + (r + sh) % Z;
            c->row_bits[c->row_ptr[m] + rfill[m]++] = n;
            c->col_chks[c->col_ptr[n] + cfill[n]++] = m;
        }
    }
    free(rfill); free(cfill);
    for (int m = 0; m < c->M; m++)
        qsort(c->row_bits + c->row_ptr[m], c->row_ptr[m + 1] - c->row_ptr[m], sizeof(int), cmp_int);
    for (int n = 0; n < c->N; n++)
        qsort(c->col_chks + c->col_ptr[n], c->col_ptr[n + 1] - c->col_ptr[n], sizeof(int), cmp_int);
    return c;
}

static ocode *code_build_single(int mb, int nb, int Z, const int *shift)
{
    int *ent = (int *)malloc(sizeof(int) * 3 * mb * nb);
    if (!ent) return NULL;
    int k = 0;
    for (int i = 0; i < mb; i++)
        for (int j = 0; j < nb; j++)
            if (shift[i * nb + j] >= 0) {
                ent[3 * k] = i; ent[3 * k + 1] = j; ent[3 * k + 2] = shift[i * nb + j];
                k++;
            }
    ocode *c = code_build(mb, nb, Z, k, ent);
    free(ent);
    return c;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* RC constraint (Section II): no two columns share ones in more than one
 * row.  Literal form: list, for every column, every pair of rows in which it
 * has ones; the constraint is violated iff some pair occurs twice. */
int or_code_violates_rc(const ocode *c)
{
    int64_t npairs = 0;
    for (int n = 0; n < c->N; n++) {
        int d = c->col_ptr[n + 1] - c->col_ptr[n];
        npairs += (int64_t)d * (d - 1) / 2;
    }
    if (npairs == 0) return 0;
    int64_t *pairs = (int64_t *)malloc(sizeof(int64_t) * npairs);
    if (!pairs) return -1;
    int64_t k = 0;
    for (int n = 0; n < c->N; n++)
        for (int a = c->col_ptr[n]; a < c->col_ptr[n + 1]; a++)
            for (int b = a + 1; b < c->col_ptr[n + 1]; b++)
                pairs[k++] = (int64_t)c->col_chks[a] * c->M + c->col_chks[b];
    qsort(pairs, npairs, sizeof(int64_t), cmp_i64);
    int bad = 0;
    for (int64_t t = 1; t < npairs; t++)
        if (pairs[t] == pairs[t - 1]) { bad = 1; break; }
    free(pairs);
    return bad;
}

/* Text description: "qc-ldpc v1", then "Z <int>", "base <mb> <nb>", then
 * mb rows of nb entries: -1 (zero block), a shift, or a comma-separated list
 * of distinct shifts.  '#' starts a comment. */
static int next_token(const char **p, char *tok, int cap)
{
    const char *s = *p;
    for (;;) {
        while (*s == ' ' || *s == '\t' || *s == '\n' || *s == '\r') s++;
        if (*s == '#') { while (*s && *s != '\n') s++; continue; }
        break;
    }
    if (!*s) { *p = s; return 0; }
    int n = 0;
    while (*s && *s != ' ' && *s != '\t' && *s != '\n' && *s != '\r' && *s != '#') {
        if (n + 1 < cap) tok[n++] = *s;
        s++;
    }
    tok[n] = 0;
    *p = s;
    return 1;
}
static int parse_int(const char *tok, long *out)
{
    char *end;
    long v = strtol(tok, &end, 10);
    if (*tok == 0 || *end != 0) return 0;
    *out = v;
    return 1;
}

int or_code_from_text(const char *text, ocode **out)
{
    if (!text || !out) return OR_EINVAL;
    *out = NULL;
    const char *p = text;
    char tok[64];
    long Z, mb, nb;
    if (!next_token(&p, tok, sizeof tok) || strcmp(tok, "qc-ldpc")) return OR_EPARSE;
    if (!next_token(&p, tok, sizeof tok) || strcmp(tok, "v1")) return OR_EPARSE;
    if (!next_token(&p, tok, sizeof tok) || strcmp(tok, "Z")) return OR_EPARSE;
    if (!next_token(&p, tok, sizeof tok) || !parse_int(tok, &Z)) return OR_EPARSE;
    if (!next_token(&p, tok, sizeof tok) || strcmp(tok, "base")) return OR_EPARSE;
    if (!next_token(&p, tok, sizeof tok) || !parse_int(tok, &mb)) return OR_EPARSE;
    if (!next_token(&p, tok, sizeof tok) || !parse_int(tok, &nb)) return OR_EPARSE;
    if (Z < 1 || mb < 1 || nb < 1 || Z > 65536 || mb > 4096 || nb > 4096 || Z * nb > (1L << 20) ||
        Z * mb > (1L << 20))
        return OR_EPARSE;
    int cap = (int)(mb * nb) + 16, nent = 0;
    int *ent = (int *)malloc(sizeof(int) * 3 * cap);
    if (!ent) return OR_ENOMEM;
    char big[4096];
    for (long t = 0; t < mb * nb; t++) {
        if (!next_token(&p, big, sizeof big)) { free(ent); return OR_EPARSE; }
        if (!strcmp(big, "-1")) continue;
        int first = nent;
        char *q = big;
        for (;;) {
            char *comma = strchr(q, ',');
            if (comma) *comma = 0;
            long v;
            if (!parse_int(q, &v) || v < 0 || v >= Z) { free(ent); return OR_EPARSE; }
            for (int e = first; e < nent; e++)
                if (ent[3 * e + 2] == v) { free(ent); return OR_EPARSE; } /* repeated shift */
            if (nent == cap) {
                cap *= 2;
                int *ne = (int *)realloc(ent, sizeof(int) * 3 * cap);
                if (!ne) { free(ent); return OR_ENOMEM; }
                ent = ne;
            }
            ent[3 * nent] = (int)(t / nb); ent[3 * nent + 1] = (int)(t % nb); ent[3 * nent + 2] = (int)v;
            nent++;
            if (!comma) break;
            q = comma + 1;
        }
    }
    if (next_token(&p, tok, sizeof tok)) { free(ent); return OR_EPARSE; }
    ocode *c = code_build((int)mb, (int)nb, (int)Z, nent, ent);
    free(ent);
    if (!c) return OR_ENOMEM;
    *out = c;
    return OR_OK;
}

/* Seeded draw: shifts drawn row-major as SplitMix64(seed) % Z; the whole base
 * matrix is redrawn (continuing the same stream) until the materialised H
 * satisfies the RC constraint, when min_girth >= 6. */
int or_code_from_seed(int mb, int nb, int Z, uint64_t seed, int min_girth, ocode **out)
{
    if (!out || mb < 1 || nb < 1 || Z < 1 || Z > 65536 || (long)Z * nb > (1L << 20)) return OR_EINVAL;
    if (min_girth != 4 && min_girth != 6) return OR_EINVAL;
    *out = NULL;
    uint64_t st = seed;
    int *sh = (int *)malloc(sizeof(int) * mb * nb);
    if (!sh) return OR_ENOMEM;
    for (int attempt = 0; attempt < 100000; attempt++) {
        for (int t = 0; t < mb * nb; t++) sh[t] = (int)(sm64_next(&st) % (uint64_t)Z);
        ocode *c = code_build_single(mb, nb, Z, sh);
        if (!c) { free(sh); return OR_ENOMEM; }
        if (min_girth < 6 || !or_code_violates_rc(c)) {
            free(sh);
            *out = c;
            return OR_OK;
        }
        code_release(c);
    }
    free(sh);
    return OR_EGIRTH;
}

void or_code_dims(const ocode *c, int *N, int *M, int *Z, int *mb, int *nb)
{
    *N = c->N; *M = c->M; *Z = c->Z; *mb = c->mb; *nb = c->nb;
}
void or_code_shifts(const ocode *c, int *out) { memcpy(out, c->shift, sizeof(int) * c->mb * c->nb); }
int or_code_n_entries(const ocode *c) { return c->nent; }
void or_code_entries(const ocode *c, int *out) { memcpy(out, c->ent, sizeof(int) * 3 * c->nent); }
int or_code_edges(const ocode *c) { return c->row_ptr[c->M]; }
/* row-major materialised adjacency: for every check, its bits */
void or_code_rows(const ocode *c, int *row_ptr, int *row_bits)
{
    memcpy(row_ptr, c->row_ptr, sizeof(int) * (c->M + 1));
    memcpy(row_bits, c->row_bits, sizeof(int) * c->row_ptr[c->M]);
}

/* ------------------------------------------------------------------------ */
/* GF(2) reduced row-echelon form, rank, systematic encoder.                */
/* Section II: the code is the null space of H; R_c = K/N.                   */
/* Columns are scanned left to right; a column is a pivot iff it is not in  */
/* the span of the columns before it, so the pivot set (and hence the info  */
/* set = non-pivot columns) is a property of H, not of the elimination.      */
/* ------------------------------------------------------------------------ */
static int code_rref(ocode *c)
{
    if (c->have_rref) return OR_OK;
    int W = (c->N + 63) / 64;
    uint64_t *A = (uint64_t *)calloc((size_t)c->M * W, sizeof(uint64_t));
    int *piv = (int *)malloc(sizeof(int) * (c->M ? c->M : 1));
    if (!A || !piv) { free(A); free(piv); return OR_ENOMEM; }
    for (int m = 0; m < c->M; m++)
        for (int e = c->row_ptr[m]; e < c->row_ptr[m + 1]; e++) {
            int n = c->row_bits[e];
            A[(size_t)m * W + n / 64] ^= 1ULL << (n % 64);
        }
    int r = 0;
    for (int col = 0; col < c->N && r < c->M; col++) {
        int w = col / 64;
        uint64_t bit = 1ULL << (col % 64);
        int p = -1;
        for (int i = r; i < c->M; i++)
            if (A[(size_t)i * W + w] & bit) { p = i; break; }
        if (p < 0) continue;
        if (p != r)
            for (int t = 0; t < W; t++) {
                uint64_t tmp = A[(size_t)p * W + t];
                A[(size_t)p * W + t] = A[(size_t)r * W + t];
                A[(size_t)r * W + t] = tmp;
            }
        for (int i = 0; i < c->M; i++)
            if (i != r && (A[(size_t)i * W + w] & bit))
                for (int t = 0; t < W; t++) A[(size_t)i * W + t] ^= A[(size_t)r * W + t];
        piv[r++] = col;
    }
    c->rank = r;
    c->K = c->N - r;
    c->words = W;
    c->rref = A; /* first `rank` rows are the RREF, the rest are zero */
    c->piv_col = piv;
    c->info_pos = (int *)malloc(sizeof(int) * (c->K ? c->K : 1));
    if (!c->info_pos) return OR_ENOMEM;
    int k = 0, t = 0;
    for (int col = 0; col < c->N; col++) {
        if (t < r && piv[t] == col) { t++; continue; }
        c->info_pos[k++] = col;
    }
    c->have_rref = 1;
    return OR_OK;
}

int or_code_rank(ocode *c, int *rank, int *K)
{
    int rc = code_rref(c);
    if (rc) return rc;
    *rank = c->rank;
    *K = c->K;
    return OR_OK;
}
int or_code_info_positions(ocode *c, int *out)
{
    int rc = code_rref(c);
    if (rc) return rc;
    memcpy(out, c->info_pos, sizeof(int) * c->K);
    return OR_OK;
}

/* Codewords first..first+count-1 of the seeded pool: info bit k of codeword
 * w is bit k%64 of SplitMix64 output number w*ceil(K/64) + k/64; info bits
 * sit at the non-pivot columns, parity bits follow from the RREF rows.
 * Output: packed 32-bit words, bit n in word n/32 at position n%32. */
int or_encode(ocode *c, uint64_t seed, int64_t first, int64_t count, uint32_t *out)
{
    int rc = code_rref(c);
    if (rc) return rc;
    int W = c->words, NW = (c->N + 31) / 32, chunks = (c->K + 63) / 64;
    uint64_t *cw = (uint64_t *)malloc(sizeof(uint64_t) * W);
    if (!cw) return OR_ENOMEM;
    for (int64_t w = 0; w < count; w++) {
        memset(cw, 0, sizeof(uint64_t) * W);
        int64_t idx = first + w;
        for (int k = 0; k < c->K; k++) {
            uint64_t word = sm64_at(seed, (uint64_t)idx * chunks + k / 64);
            if ((word >> (k % 64)) & 1) {
                int n = c->info_pos[k];
                cw[n / 64] |= 1ULL << (n % 64);
            }
        }
        for (int r = 0; r < c->rank; r++) {
            int par = 0;
            for (int t = 0; t < W; t++) par ^= __builtin_parityll(c->rref[(size_t)r * W + t] & cw[t]);
            if (par) cw[c->piv_col[r] / 64] |= 1ULL << (c->piv_col[r] % 64);
        }
        uint32_t *o = out + (size_t)w * NW;
        for (int t = 0; t < NW; t++) o[t] = (uint32_t)(cw[t / 2] >> (32 * (t % 2)));
    }
    free(cw);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Decoding.                                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int weights, select, G, lambda, max_iter;
    float alpha;
    int alpha_num, alpha_den;
} oparams;

/* per-thread scratch for one frame */
typedef struct {
    int32_t *ai;  /* |y| integer */
    float *af;    /* |y| float */
    int32_t *wi;  /* per-edge weight (edge in row-major order) */
    float *wf;
    uint8_t *z, *s;
    int64_t *Ei;
    float *Ef;
    int *flip;
    int *order; /* TOPL */
} scratch;

static int scratch_alloc(const ocode *c, scratch *w)
{
    int E = c->row_ptr[c->M];
    memset(w, 0, sizeof *w);
    w->ai = (int32_t *)malloc(sizeof(int32_t) * c->N);
    w->af = (float *)malloc(sizeof(float) * c->N);
    w->wi = (int32_t *)malloc(sizeof(int32_t) * (E ? E : 1));
    w->wf = (float *)malloc(sizeof(float) * (E ? E : 1));
    w->z = (uint8_t *)malloc(c->N);
    w->s = (uint8_t *)malloc(c->M ? c->M : 1);
    w->Ei = (int64_t *)malloc(sizeof(int64_t) * c->N);
    w->Ef = (float *)malloc(sizeof(float) * c->N);
    w->flip = (int *)malloc(sizeof(int) * c->N);
    w->order = (int *)malloc(sizeof(int) * c->N);
    return (w->ai && w->af && w->wi && w->wf && w->z && w->s && w->Ei && w->Ef && w->flip && w->order)
               ? OR_OK : OR_ENOMEM;
}
static void scratch_free(scratch *w)
{
    free(w->ai); free(w->af); free(w->wi); free(w->wf); free(w->z); free(w->s);
    free(w->Ei); free(w->Ef); free(w->flip); free(w->order);
}

/* weight of edge (m, n) where n = row_bits[e]: literal minimum over N(m)
 * (excluding n itself for IMWBF, as in the definition below eq. (1)) */
static void compute_weights(const ocode *c, const oparams *P, int isf, scratch *w)
{
    for (int m = 0; m < c->M; m++)
        for (int e = c->row_ptr[m]; e < c->row_ptr[m + 1]; e++) {
            int n = c->row_bits[e];
            int have = 0;
            int32_t mi = 0;
            float mf = 0.0f;
            for (int t = c->row_ptr[m]; t < c->row_ptr[m + 1]; t++) {
                int i = c->row_bits[t];
                if (P->weights == W_IMWBF && i == n) continue;
                if (isf) { if (!have || w->af[i] < mf) mf = w->af[i]; }
                else { if (!have || w->ai[i] < mi) mi = w->ai[i]; }
                have = 1;
            }
            w->wi[e] = mi; /* empty minimum (degree-1 check under IMWBF) is 0 */
            w->wf[e] = mf;
        }
}

/* weight of edge (m, n) looked up by scanning N(m) for n */
static int edge_of(const ocode *c, int m, int n)
{
    for (int t = c->row_ptr[m]; t < c->row_ptr[m + 1]; t++)
        if (c->row_bits[t] == n) return t;
    return -1;
}

/* metric of bit n, eq. (1); returns nothing, fills Ei[n] or Ef[n] */
static void metric(const ocode *c, const oparams *P, int isf, scratch *w, int n)
{
    if (isf) {
        float S = 0.0f;
        int first = 1;
        for (int t = c->col_ptr[n]; t < c->col_ptr[n + 1]; t++) {
            int m = c->col_chks[t];
            float wt = w->wf[edge_of(c, m, n)];
            float term = w->s[m] ? wt : -wt; /* (2 s_m - 1) w_{n,m} */
            if (first) { S = term; first = 0; }
            else S = S + term;
        }
        float alpha = (P->weights == W_WBF) ? 0.0f : P->alpha;
        w->Ef[n] = fmaf(-alpha, w->af[n], S);
    } else {
        int64_t S = 0;
        for (int t = c->col_ptr[n]; t < c->col_ptr[n + 1]; t++) {
            int m = c->col_chks[t];
            int64_t wt = w->wi[edge_of(c, m, n)];
            S += w->s[m] ? wt : -wt;
        }
        int64_t an = (P->weights == W_WBF) ? 0 : P->alpha_num;
        w->Ei[n] = (int64_t)P->alpha_den * S - an * (int64_t)w->ai[n];
    }
}

/* a > b in the metric order: larger metric, ties to the lower bit index */
static int better(const scratch *w, int isf, int a, int b)
{
    if (isf) {
        if (w->Ef[a] != w->Ef[b]) return w->Ef[a] > w->Ef[b];
    } else {
        if (w->Ei[a] != w->Ei[b]) return w->Ei[a] > w->Ei[b];
    }
    return a < b;
}
static int positive(const scratch *w, int isf, int n) { return isf ? (w->Ef[n] > 0.0f) : (w->Ei[n] > 0); }

/* optional trace of one frame: metric values of round 0 and flips per round */
typedef struct {
    double *E0;     /* N values (scaled integer metric or float metric), may be NULL */
    int *nflips;    /* max_iter counts, may be NULL */
    int *flips;     /* max_iter * N indices, may be NULL */
} otrace;

static const scratch *g_sort_w;
static int g_sort_isf;
static int cmp_order(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    if (better(g_sort_w, g_sort_isf, x, y)) return -1;
    if (better(g_sort_w, g_sort_isf, y, x)) return 1;
    return 0;
}
static pthread_mutex_t g_sort_lock = PTHREAD_MUTEX_INITIALIZER;

static void decode_frame(const ocode *c, const oparams *P, int dtype, const void *yrow,
                         scratch *w, uint32_t *zout, int32_t *iters, uint8_t *ok, otrace *tr)
{
    const int N = c->N, M = c->M;
    const int isf = (dtype == D_F32);
    /* Initialization (Section III): |y|, hard decision z_0, check weights */
    for (int n = 0; n < N; n++) {
        if (dtype == D_F32) {
            float v = ((const float *)yrow)[n];
            w->af[n] = fabsf(v);
            w->z[n] = v < 0.0f;
        } else if (dtype == D_I8) {
            int v = ((const int8_t *)yrow)[n];
            w->ai[n] = v < 0 ? -v : v;
            w->z[n] = v < 0;
        } else {
            int v = ((const int16_t *)yrow)[n];
            w->ai[n] = v < 0 ? -v : v;
            w->z[n] = v < 0;
        }
    }
    compute_weights(c, P, isf, w);
    int k = 0, done_ok = 0;
    for (;;) {
        /* Step 1: syndrome s_k = z_k H^T and its weight */
        int weight = 0;
        for (int m = 0; m < M; m++) {
            int x = 0;
            for (int t = c->row_ptr[m]; t < c->row_ptr[m + 1]; t++) x ^= w->z[c->row_bits[t]];
            w->s[m] = (uint8_t)x;
            weight += x;
        }
        if (weight == 0) { done_ok = 1; break; }
        if (k == P->max_iter) break;
        /* Step 2: metrics by eq. (1) */
        for (int n = 0; n < N; n++) metric(c, P, isf, w, n);
        if (tr && tr->E0 && k == 0)
            for (int n = 0; n < N; n++) tr->E0[n] = isf ? (double)w->Ef[n] : (double)w->Ei[n];
        int nf = 0;
        if (P->select == S_GROUPS) {
            int p = (N + P->G - 1) / P->G;
            for (int lo = 0; lo < N; lo += p) {
                int hi = lo + p < N ? lo + p : N;
                int b = lo;
                for (int n = lo + 1; n < hi; n++)
                    if (better(w, isf, n, b)) b = n;
                if (positive(w, isf, b)) w->flip[nf++] = b;
            }
        } else if (P->select == S_STRIDED) {
            for (int g = 0; g < P->G; g++) {
                int b = g;
                for (int n = g + P->G; n < N; n += P->G)
                    if (better(w, isf, n, b)) b = n;
                if (positive(w, isf, b)) w->flip[nf++] = b;
            }
        } else if (P->select == S_SINGLE) {
            int b = 0;
            for (int n = 1; n < N; n++)
                if (better(w, isf, n, b)) b = n;
            w->flip[nf++] = b;
        } else {
            for (int n = 0; n < N; n++) w->order[n] = n;
            pthread_mutex_lock(&g_sort_lock);
            g_sort_w = w;
            g_sort_isf = isf;
            qsort(w->order, N, sizeof(int), cmp_order);
            pthread_mutex_unlock(&g_sort_lock);
            for (int t = 0; t < N && nf < P->lambda; t++) {
                if (!positive(w, isf, w->order[t])) break;
                w->flip[nf++] = w->order[t];
            }
        }
        if (tr && tr->nflips) tr->nflips[k] = nf;
        if (tr && tr->flips)
            for (int t = 0; t < nf; t++) tr->flips[(size_t)k * N + t] = w->flip[t];
        for (int t = 0; t < nf; t++) w->z[w->flip[t]] ^= 1;
        k += 1;
    }
    int NW = (N + 31) / 32;
    for (int t = 0; t < NW; t++) zout[t] = 0;
    for (int n = 0; n < N; n++)
        if (w->z[n]) zout[n / 32] |= 1u << (n % 32);
    *iters = k;
    *ok = (uint8_t)done_ok;
}

static int params_valid(const ocode *c, const oparams *P, int dtype)
{
    if (dtype < D_F32 || dtype > D_I16) return 0;
    if (P->weights < W_WBF || P->weights > W_IMWBF) return 0;
    if (P->select < S_GROUPS || P->select > S_STRIDED) return 0;
    if ((P->select == S_GROUPS || P->select == S_STRIDED) && (P->G < 1 || P->G > c->N)) return 0;
    if (P->select == S_TOPL && P->lambda < 1) return 0;
    if (P->max_iter < 0) return 0;
    if (dtype != D_F32 && P->alpha_den < 1) return 0;
    return 1;
}

typedef struct {
    const ocode *c;
    const oparams *P;
    int dtype;
    const uint8_t *y;
    int64_t f0, f1, stride_bytes;
    uint32_t *z;
    int32_t *iters;
    uint8_t *ok;
    int rc;
} job;

static void *worker(void *arg)
{
    job *j = (job *)arg;
    scratch w;
    j->rc = scratch_alloc(j->c, &w);
    if (j->rc == OR_OK) {
        int NW = (j->c->N + 31) / 32;
        for (int64_t f = j->f0; f < j->f1; f++)
            decode_frame(j->c, j->P, j->dtype, j->y + f * j->stride_bytes, &w, j->z + f * NW,
                         j->iters + f, j->ok + f, NULL);
    }
    scratch_free(&w);
    return NULL;
}

int or_decode(const ocode *c, int weights, int select, int G, int lambda, int max_iter, float alpha,
              int alpha_num, int alpha_den, int dtype, const void *y, int64_t F, int64_t stride,
              uint32_t *z, int32_t *iters, uint8_t *ok, int nthreads)
{
    oparams P = {weights, select, G, lambda, max_iter, alpha, alpha_num, alpha_den};
    if (!c || (!y && F > 0) || F < 0 || stride < c->N || !params_valid(c, &P, dtype)) return OR_EINVAL;
    if (F == 0) return OR_OK;
    int esz = dtype == D_F32 ? 4 : dtype == D_I8 ? 1 : 2;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > F) nthreads = (int)F;
    job *jobs = (job *)calloc(nthreads, sizeof(job));
    pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return OR_ENOMEM; }
    for (int t = 0; t < nthreads; t++) {
        jobs[t] = (job){c, &P, dtype, (const uint8_t *)y, F * t / nthreads, F * (t + 1) / nthreads,
                        stride * esz, z, iters, ok, 0};
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    int rc = OR_OK;
    for (int t = 0; t < nthreads; t++) {
        pthread_join(th[t], NULL);
        if (jobs[t].rc) rc = jobs[t].rc;
    }
    free(jobs); free(th);
    return rc;
}

/* one frame with a trace of the round-0 metrics and the flips of every round */
int or_decode_trace(const ocode *c, int weights, int select, int G, int lambda, int max_iter,
                    float alpha, int alpha_num, int alpha_den, int dtype, const void *y,
                    uint32_t *z, int32_t *iters, uint8_t *ok, double *E0, int *nflips, int *flips)
{
    oparams P = {weights, select, G, lambda, max_iter, alpha, alpha_num, alpha_den};
    if (!c || !y || !params_valid(c, &P, dtype)) return OR_EINVAL;
    scratch w;
    int rc = scratch_alloc(c, &w);
    if (rc == OR_OK) {
        otrace tr = {E0, nflips, flips};
        decode_frame(c, &P, dtype, y, &w, z, iters, ok, &tr);
    }
    scratch_free(&w);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Channel (Section II: BPSK s = 1 - 2c; Section V: AWGN, variance N0/2).   */
/* Noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw 2011) keyed by the seed,*/
/* counter (n/4, frame low, frame high, stream); the four words give two    */
/* Box-Muller pairs (u = (x>>9 + 1/2) 2^-23, r = sqrt(-2 ln u_a),           */
/* angle 2 pi u_b; cosine for the even member, sine for the odd one).       */
/* Computed in double precision.                                            */
/* ------------------------------------------------------------------------ */
static void philox_round(uint32_t x[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * x[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x[1] ^ k[0];
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x[3] ^ k[1];
    uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(x, k);
    }
    memcpy(out, x, sizeof x);
}

static double gauss_of(uint64_t seed, uint32_t stream, int64_t f, int n)
{
    uint32_t ctr[4] = {(uint32_t)(n / 4), (uint32_t)(uint64_t)f, (uint32_t)((uint64_t)f >> 32), stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    or_philox4x32_10(ctr, key, x);
    int pair = (n % 4) / 2, odd = n % 2;
    double ua = ((double)(x[2 * pair] >> 9) + 0.5) / 8388608.0;
    double ub = ((double)(x[2 * pair + 1] >> 9) + 0.5) / 8388608.0;
    double r = sqrt(-2.0 * log(ua));
    double ang = 2.0 * M_PI * ub;
    return odd ? r * sin(ang) : r * cos(ang);
}

/* y[f][n] for frames f0..f0+F-1.  Codeword of frame f: pool row f % pool_n
 * (pool == NULL: all-zero codeword).  dtype F32 writes float y; I8/I16
 * write clamp(rint(scale*y), -qmax, qmax) with qmax 127 / 32767.  The
 * unquantised double values are written to yd when yd != NULL. */
int or_channel(int N, int64_t F, int64_t f0, const uint32_t *pool, int64_t pool_n, uint64_t seed,
               uint32_t stream, double sigma, double scale, int dtype, void *out, double *yd)
{
    if (N < 1 || F < 0 || (pool && pool_n < 1)) return OR_EINVAL;
    int NW = (N + 31) / 32;
    for (int64_t f = 0; f < F; f++) {
        const uint32_t *cw = pool ? pool + (size_t)((f0 + f) % pool_n) * NW : NULL;
        for (int n = 0; n < N; n++) {
            int cbit = cw ? (cw[n / 32] >> (n % 32)) & 1 : 0;
            double yv = (1.0 - 2.0 * cbit) + sigma * gauss_of(seed, stream, f0 + f, n);
            size_t idx = (size_t)f * N + n;
            if (yd) yd[idx] = yv;
            if (dtype == D_F32) ((float *)out)[idx] = (float)yv;
            else {
                double qmax = dtype == D_I8 ? 127.0 : 32767.0;
                double q = rint(scale * yv);
                if (q > qmax) q = qmax;
                if (q < -qmax) q = -qmax;
                if (dtype == D_I8) ((int8_t *)out)[idx] = (int8_t)q;
                else ((int16_t *)out)[idx] = (int16_t)q;
            }
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Error accounting (Section V): bit errors, frame errors, undetected frame */
/* errors (zero syndrome but a wrong codeword), iteration sum, histogram.   */
/* counts[0..4] = bit errors, frame errors, undetected, iteration sum,      */
/* frames; hist has max_iter+1 bins.                                        */
/* ------------------------------------------------------------------------ */
int or_count(int N, int64_t F, int64_t f0, const uint32_t *z, const uint32_t *pool, int64_t pool_n,
             const int32_t *iters, const uint8_t *ok, int max_iter, int64_t *counts, int64_t *hist)
{
    if (N < 1 || F < 0 || max_iter < 0 || (pool && pool_n < 1)) return OR_EINVAL;
    int NW = (N + 31) / 32;
    for (int64_t f = 0; f < F; f++) {
        const uint32_t *cw = pool ? pool + (size_t)((f0 + f) % pool_n) * NW : NULL;
        int64_t be = 0;
        for (int n = 0; n < N; n++) {
            int zb = (z[(size_t)f * NW + n / 32] >> (n % 32)) & 1;
            int cb = cw ? (cw[n / 32] >> (n % 32)) & 1 : 0;
            be += zb != cb;
        }
        counts[0] += be;
        counts[1] += be != 0;
        counts[2] += (be != 0) && ok[f];
        counts[3] += iters[f];
        counts[4] += 1;
        int it = iters[f];
        if (it >= 0 && it <= max_iter) hist[it] += 1;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Min-sum belief propagation: the BP reference decoder the paper compares  */
/* FWBF with (Section I names normalised and offset min-sum; Section V      */
/* reports BP 0.5 dB ahead of FWBF).  The paper gives no equations for it;  */
/* this is the textbook flooding schedule, float32, written out literally:  */
/*   iteration i >= 1, every edge (m, n):                                   */
/*     Q_{n,m} = P_n - R_{m,n}       (P, R of iteration i-1; R = 0, P = L)  */
/*     R_{m,n} = s * c * min |Q_{n',m}|   over n' in N(m)\n, s = product of */
/*               the signs of those Q (sign -1 iff Q < 0)                    */
/*       normalised: c * min (one float product), offset: max(min - c, 0)   */
/*     P_n = L_n + sum_{m in M(n)} R_{m,n}, in ascending m                  */
/*     z_n = [P_n < 0]; stop on a zero syndrome or after K_max iterations.  */
/* L_n = y_n (the channel LLR up to a positive factor, which min-sum does   */
/* not need).  Iterations are counted like the flip rounds of FWBF: 0 when  */
/* z_0 = [y < 0] already satisfies H.                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    const ocode *c;
    int offset, max_iter;
    float cst;
    const float *y;
    int64_t f0, f1, stride;
    uint32_t *z;
    int32_t *iters;
    uint8_t *ok;
    int rc;
} msjob;

static int ms_syndrome_zero(const ocode *c, const uint8_t *z)
{
    for (int m = 0; m < c->M; m++) {
        int x = 0;
        for (int t = c->row_ptr[m]; t < c->row_ptr[m + 1]; t++) x ^= z[c->row_bits[t]];
        if (x) return 0;
    }
    return 1;
}

static void *ms_worker(void *arg)
{
    msjob *j = (msjob *)arg;
    const ocode *c = j->c;
    const int N = c->N, M = c->M, E = c->row_ptr[M];
    float *L = (float *)malloc(sizeof(float) * N), *P = (float *)malloc(sizeof(float) * N);
    float *R = (float *)malloc(sizeof(float) * (E ? E : 1)), *Rn = (float *)malloc(sizeof(float) * (E ? E : 1));
    float *Q = (float *)malloc(sizeof(float) * (E ? E : 1));
    uint8_t *z = (uint8_t *)malloc(N);
    /* edge index of (m, n) seen from the bit side: for bit n, its checks in
       ascending order and the edge of each */
    int *bedge = (int *)malloc(sizeof(int) * (E ? E : 1));
    if (!L || !P || !R || !Rn || !Q || !z || !bedge) { j->rc = OR_ENOMEM; goto out; }
    for (int n = 0; n < N; n++)
        for (int u = c->col_ptr[n]; u < c->col_ptr[n + 1]; u++) {
            int m = c->col_chks[u], e = -1;
            for (int t = c->row_ptr[m]; t < c->row_ptr[m + 1]; t++)
                if (c->row_bits[t] == n) e = t;
            bedge[u] = e;
        }
    for (int64_t f = j->f0; f < j->f1; f++) {
        const float *y = j->y + f * j->stride;
        for (int n = 0; n < N; n++) { L[n] = y[n]; P[n] = y[n]; z[n] = y[n] < 0.0f; }
        for (int e = 0; e < E; e++) R[e] = 0.0f;
        int it = 0, okf = ms_syndrome_zero(c, z);
        while (!okf && it < j->max_iter) {
            for (int m = 0; m < M; m++) {
                for (int t = c->row_ptr[m]; t < c->row_ptr[m + 1]; t++) Q[t] = P[c->row_bits[t]] - R[t];
                for (int t = c->row_ptr[m]; t < c->row_ptr[m + 1]; t++) {
                    float mn = INFINITY;
                    int neg = 0;
                    for (int u = c->row_ptr[m]; u < c->row_ptr[m + 1]; u++) {
                        if (u == t) continue;
                        float a = fabsf(Q[u]);
                        if (a < mn) mn = a;
                        neg ^= Q[u] < 0.0f;
                    }
                    if (c->row_ptr[m + 1] - c->row_ptr[m] < 2) mn = 0.0f;
                    float mag;
                    if (j->offset) { mag = mn - j->cst; if (!(mag > 0.0f)) mag = 0.0f; }
                    else mag = j->cst * mn;
                    Rn[t] = neg ? -mag : mag;
                }
            }
            for (int e = 0; e < E; e++) R[e] = Rn[e];
            for (int n = 0; n < N; n++) {
                float s = L[n];
                for (int u = c->col_ptr[n]; u < c->col_ptr[n + 1]; u++) s = s + R[bedge[u]];
                P[n] = s;
                z[n] = s < 0.0f;
            }
            it++;
            okf = ms_syndrome_zero(c, z);
        }
        int NW = (N + 31) / 32;
        uint32_t *zo = j->z + f * NW;
        for (int t = 0; t < NW; t++) zo[t] = 0;
        for (int n = 0; n < N; n++)
            if (z[n]) zo[n / 32] |= 1u << (n % 32);
        j->iters[f] = it;
        j->ok[f] = (uint8_t)okf;
    }
out:
    free(L); free(P); free(R); free(Rn); free(Q); free(z); free(bedge);
    return NULL;
}

/* offset = 0: normalised min-sum with factor cst; 1: offset min-sum */
int or_decode_minsum(const ocode *c, int offset, float cst, int max_iter, const float *y, int64_t F,
                     int64_t stride, uint32_t *z, int32_t *iters, uint8_t *ok, int nthreads)
{
    if (!c || (!y && F > 0) || F < 0 || stride < c->N || max_iter < 0 || (offset != 0 && offset != 1) ||
        !(cst >= 0.0f))
        return OR_EINVAL;
    if (F == 0) return OR_OK;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > F) nthreads = (int)F;
    msjob *jobs = (msjob *)calloc(nthreads, sizeof(msjob));
    pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return OR_ENOMEM; }
    for (int t = 0; t < nthreads; t++) {
        jobs[t] = (msjob){c, offset, max_iter, cst, y, F * t / nthreads, F * (t + 1) / nthreads, stride, z,
                          iters, ok, 0};
        pthread_create(&th[t], NULL, ms_worker, &jobs[t]);
    }
    int rc = OR_OK;
    for (int t = 0; t < nthreads; t++) {
        pthread_join(th[t], NULL);
        if (jobs[t].rc) rc = jobs[t].rc;
    }
    free(jobs); free(th);
    return rc;
}
