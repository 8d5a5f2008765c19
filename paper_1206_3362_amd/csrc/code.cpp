// Host side of libfwbf.so: QC-LDPC code objects (Section II of the paper:
// H, M(n), N(m), the RC constraint), the seeded base draw, GF(2) rank and the
// systematic encoder, error reporting.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <sstream>

#include "internal.h"

namespace fwbf {

static thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(FWBF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", 2014): Weyl increment then the variant-13 output mix.
struct SplitMix64 {
    uint64_t x;
    static uint64_t mix(uint64_t v)
    {
        v = (v ^ (v >> 30)) * 0xBF58476D1CE4E5B9ULL;
        v = (v ^ (v >> 27)) * 0x94D049BB133111EBULL;
        return v ^ (v >> 31);
    }
    uint64_t next() { return mix(x += 0x9E3779B97F4A7C15ULL); }
    // output number idx (0-based) of the stream seeded with s
    static uint64_t at(uint64_t s, uint64_t idx) { return mix(s + (idx + 1) * 0x9E3779B97F4A7C15ULL); }
};

// Circulant-permutation lifting has a 4-cycle iff some base rectangle
// (i1,j1),(i1,j2),(i2,j2),(i2,j1) of nonzero blocks has shift sum
// s11 - s12 + s22 - s21 = 0 mod Z (two rows of one block row never share a
// column, so every 4-cycle spans two block rows and two block columns).
bool base_has_4cycle(int mb, int nb, int Z, const int *s)
{
    for (int i1 = 0; i1 < mb; i1++)
        for (int i2 = i1 + 1; i2 < mb; i2++)
            for (int j1 = 0; j1 < nb; j1++) {
                int a = s[i1 * nb + j1], d = s[i2 * nb + j1];
                if (a < 0 || d < 0) continue;
                for (int j2 = j1 + 1; j2 < nb; j2++) {
                    int b = s[i1 * nb + j2], c = s[i2 * nb + j2];
                    if (b < 0 || c < 0) continue;
                    long v = ((long)a - b + c - d) % Z;
                    if (v == 0) return true;
                }
            }
    return false;
}

// A block may hold several distinct shifts (a circulant of that weight).
// cells[i * nb + j] lists the shifts of block (i, j); an empty list is the
// zero block.  Within a block the kernels' tables list the shifts in
// descending order, so that for bit c of a block column the checks of one
// block row come in ascending order after a rotation: those with shift <= c
// first, then the wrapped ones (row (c - s) mod Z).
int make_code(int mb, int nb, int Z, std::vector<std::vector<int>> cells, fwbf_code **out)
{
    if (Z < 1 || Z > 65535 || mb < 1 || nb < 1 || (long)nb * Z > 65535 || (long)mb * Z > 65535)
        return fail(FWBF_E_INVALID, "code dimensions out of range (Z <= 65535, N, M <= 65535)");
    fwbf_code *c = new (std::nothrow) fwbf_code;
    if (!c) return fail(FWBF_E_NOMEM, "out of host memory");
    c->Z = Z; c->mb = mb; c->nb = nb;
    c->N = nb * Z; c->M = mb * Z;
    c->shift.assign((size_t)mb * nb, -1);
    c->coldeg.assign(nb, 0);
    c->rowdeg.assign(mb, 0);
    std::vector<int> cdeg(nb, 0), rdeg(mb, 0);
    for (int i = 0; i < mb; i++)
        for (int j = 0; j < nb; j++) {
            auto &v = cells[(size_t)i * nb + j];
            std::sort(v.begin(), v.end(), [](int x, int y) { return x > y; });
            if (v.size() > 1) c->multi = true;
            if (!v.empty()) c->shift[(size_t)i * nb + j] = v[0];
            cdeg[j] += (int)v.size();
            rdeg[i] += (int)v.size();
        }
    for (int j = 0; j < nb; j++) c->dv_max = std::max(c->dv_max, cdeg[j]);
    for (int i = 0; i < mb; i++) c->dc_max = std::max(c->dc_max, rdeg[i]);
    if (c->dv_max > 64 || c->dc_max > 64 || c->dv_max == 0) {
        delete c;
        return fail(FWBF_E_UNSUPPORTED, "column and row weights must be at most 64 (and some column nonzero)");
    }
    for (int j = 0; j < nb; j++) c->coldeg[j] = (uint8_t)cdeg[j];
    for (int i = 0; i < mb; i++) c->rowdeg[i] = (uint8_t)rdeg[i];
    c->cells = cells;
    c->row.assign((size_t)mb * c->dc_max, 0);
    c->col.assign((size_t)nb * c->dv_max, 0);
    std::vector<int> qpos((size_t)mb * nb, -1);  // row-list position of a block's first shift
    for (int i = 0; i < mb; i++) {
        int q = 0;
        for (int j = 0; j < nb; j++) {
            const auto &v = cells[(size_t)i * nb + j];
            if (!v.empty()) qpos[(size_t)i * nb + j] = q;
            for (int s : v) c->row[(size_t)i * c->dc_max + q++] = ((uint32_t)j << 16) | (uint32_t)s;
        }
    }
    for (int j = 0; j < nb; j++) {
        int t = 0;
        for (int i = 0; i < mb; i++) {
            const auto &v = cells[(size_t)i * nb + j];
            for (size_t u = 0; u < v.size(); u++)
                c->col[(size_t)j * c->dv_max + t++] =
                    ((uint32_t)i << 24) | ((uint32_t)(qpos[(size_t)i * nb + j] + u) << 16) | (uint32_t)v[u];
        }
    }
    *out = c;
    return FWBF_OK;
}

int make_code(int mb, int nb, int Z, const std::vector<int> &shift, fwbf_code **out)
{
    std::vector<std::vector<int>> cells((size_t)mb * nb);
    for (size_t t = 0; t < cells.size(); t++)
        if (shift[t] >= 0) cells[t].push_back(shift[t]);
    return make_code(mb, nb, Z, std::move(cells), out);
}

// 4-cycle test on the expanded graph: two checks sharing two bits.  Every
// pair of bits of every check is listed once and the list is searched for a
// repeat (used for bases with multi-shift blocks, where cycles can also lie
// inside one block row).
bool expanded_has_4cycle(const fwbf_code *c)
{
    std::vector<uint64_t> pairs;
    std::vector<int> bits;
    for (int i = 0; i < c->mb; i++)
        for (int r = 0; r < c->Z; r++) {
            bits.clear();
            for (int q = 0; q < c->rowdeg[i]; q++) {
                const uint32_t e = c->row[(size_t)i * c->dc_max + q];
                bits.push_back((int)(e >> 16) * c->Z + (r + (int)(e & 0xFFFF)) % c->Z);
            }
            for (size_t a = 0; a < bits.size(); a++)
                for (size_t b = a + 1; b < bits.size(); b++) {
                    const uint64_t lo = std::min(bits[a], bits[b]), hi = std::max(bits[a], bits[b]);
                    pairs.push_back(lo << 32 | hi);
                }
        }
    std::sort(pairs.begin(), pairs.end());
    return std::adjacent_find(pairs.begin(), pairs.end()) != pairs.end();
}

// tokenizer for the description text
struct Lexer {
    const char *p;
    bool next(std::string &tok)
    {
        for (;;) {
            while (*p == ' ' || *p == '\t' || *p == '\r' || *p == '\n') p++;
            if (*p == '#') {
                while (*p && *p != '\n') p++;
                continue;
            }
            break;
        }
        if (!*p) return false;
        tok.clear();
        while (*p && *p != ' ' && *p != '\t' && *p != '\r' && *p != '\n' && *p != '#') tok += *p++;
        return true;
    }
    bool integer(long &v)
    {
        std::string t;
        if (!next(t)) return false;
        char *end = nullptr;
        v = strtol(t.c_str(), &end, 10);
        return !t.empty() && *end == 0;
    }
    bool word(const char *w)
    {
        std::string t;
        return next(t) && t == w;
    }
};

}  // namespace

// Reduced row-echelon form over GF(2): forward elimination (pivot = first
// remaining row with a one in the current column, scanning columns left to
// right), then back-substitution clearing the pivot columns above each pivot.
// The pivot columns are those not in the span of the columns to their left,
// so the info set does not depend on the elimination order.
int ensure_rref(fwbf_code *c)
{
    std::call_once(c->rref_once, [c]() {
        const int W = (c->N + 63) / 64;
        std::vector<uint64_t> A;
        try {
            A.assign((size_t)c->M * W, 0);
        } catch (...) {
            c->rref_rc = FWBF_E_NOMEM;
            return;
        }
        for (int i = 0; i < c->mb; i++)
            for (int q = 0; q < c->rowdeg[i]; q++) {
                uint32_t e = c->row[(size_t)i * c->dc_max + q];
                int j = e >> 16, s = e & 0xFFFF;
                for (int r = 0; r < c->Z; r++) {
                    int m = i * c->Z + r, n = j * c->Z + (r + s) % c->Z;
                    A[(size_t)m * W + n / 64] |= 1ULL << (n % 64);
                }
            }
        std::vector<int> piv;
        int rank = 0;
        for (int col = 0; col < c->N && rank < c->M; col++) {
            const int w = col / 64;
            const uint64_t b = 1ULL << (col % 64);
            int p = rank;
            while (p < c->M && !(A[(size_t)p * W + w] & b)) p++;
            if (p == c->M) continue;
            if (p != rank)
                for (int t = 0; t < W; t++) std::swap(A[(size_t)p * W + t], A[(size_t)rank * W + t]);
            const uint64_t *pr = &A[(size_t)rank * W];
            for (int r = rank + 1; r < c->M; r++) {
                uint64_t *rr = &A[(size_t)r * W];
                if (rr[w] & b)
                    for (int t = w; t < W; t++) rr[t] ^= pr[t];
            }
            piv.push_back(col);
            rank++;
        }
        for (int r = rank - 1; r >= 0; r--) {
            const int col = piv[r], w = col / 64;
            const uint64_t b = 1ULL << (col % 64);
            const uint64_t *pr = &A[(size_t)r * W];
            for (int u = 0; u < r; u++) {
                uint64_t *ur = &A[(size_t)u * W];
                if (ur[w] & b)
                    for (int t = w; t < W; t++) ur[t] ^= pr[t];
            }
        }
        A.resize((size_t)rank * W);
        c->rref.swap(A);
        c->piv = piv;
        c->rank = rank;
        c->K = c->N - rank;
        c->words = W;
        c->info.clear();
        size_t t = 0;
        for (int col = 0; col < c->N; col++) {
            if (t < piv.size() && piv[t] == col) { t++; continue; }
            c->info.push_back(col);
        }
        c->rref_rc = FWBF_OK;
    });
    if (c->rref_rc) return fail(c->rref_rc, "GF(2) elimination failed (out of memory)");
    return FWBF_OK;
}

int device_tables_resident(const fwbf_code *c, DeviceTables *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    fwbf_code *m = const_cast<fwbf_code *>(c);
    std::lock_guard<std::mutex> lk(m->mu);
    auto it = m->dev.find(dev);
    if (it == m->dev.end())
        return fail(FWBF_E_INVALID, "code tables are not on this device yet: decode with this code once "
                                    "(fwbf_decode or fwbf_decode_batched) before a no-allocation call");
    *out = it->second;
    return FWBF_OK;
}

int device_tables(fwbf_code *c, DeviceTables *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->dev.find(dev);
    if (it != c->dev.end()) {
        *out = it->second;
        return FWBF_OK;
    }
    size_t ncol = c->col.size() * 4, nrow = c->row.size() * 4, nsh = c->shift.size() * 4;
    size_t total = nsh + ncol + nrow + c->coldeg.size() + c->rowdeg.size();
    char *base = nullptr;
    e = hipMalloc((void **)&base, total);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(code tables)");
    std::vector<char> host(total);
    memcpy(host.data(), c->shift.data(), nsh);
    memcpy(host.data() + nsh, c->col.data(), ncol);
    memcpy(host.data() + nsh + ncol, c->row.data(), nrow);
    memcpy(host.data() + nsh + ncol + nrow, c->coldeg.data(), c->coldeg.size());
    memcpy(host.data() + nsh + ncol + nrow + c->coldeg.size(), c->rowdeg.data(), c->rowdeg.size());
    e = hipMemcpy(base, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(base);
        return hip_fail(e, "hipMemcpy(code tables)");
    }
    DeviceTables t;
    t.shift = (uint32_t *)base;
    t.col = (uint32_t *)(base + nsh);
    t.row = (uint32_t *)(base + nsh + ncol);
    t.coldeg = (uint8_t *)(base + nsh + ncol + nrow);
    t.rowdeg = (uint8_t *)(base + nsh + ncol + nrow + c->coldeg.size());
    c->dev[dev] = t;
    *out = t;
    return FWBF_OK;
}

}  // namespace fwbf

using namespace fwbf;

extern "C" {

const char *fwbf_last_error(void) { return g_err.c_str(); }

const char *fwbf_version(void) { return "fwbf 0.1 (gfx950)"; }

int fwbf_code_from_text(const char *text, fwbf_code **out)
{
    if (!text || !out) return fail(FWBF_E_INVALID, "null argument");
    *out = nullptr;
    Lexer lx{text};
    long Z, mb, nb;
    if (!lx.word("qc-ldpc") || !lx.word("v1")) return fail(FWBF_E_PARSE, "expected 'qc-ldpc v1'");
    if (!lx.word("Z") || !lx.integer(Z)) return fail(FWBF_E_PARSE, "expected 'Z <int>'");
    if (!lx.word("base") || !lx.integer(mb) || !lx.integer(nb))
        return fail(FWBF_E_PARSE, "expected 'base <mb> <nb>'");
    if (Z < 1 || Z > 65535 || mb < 1 || nb < 1 || mb > 4096 || nb > 4096 || nb * Z > 65535 ||
        mb * Z > 65535)
        return fail(FWBF_E_PARSE, "dimensions out of range");
    std::vector<std::vector<int>> cells((size_t)mb * nb);
    for (long t = 0; t < mb * nb; t++) {
        std::string tok;
        if (!lx.next(tok)) return fail(FWBF_E_PARSE, "expected " + std::to_string(mb * nb) + " blocks");
        if (tok == "-1") continue;
        size_t at = 0;
        for (;;) {
            const size_t comma = tok.find(',', at);
            const std::string part = tok.substr(at, comma == std::string::npos ? std::string::npos : comma - at);
            char *end = nullptr;
            const long v = strtol(part.c_str(), &end, 10);
            if (part.empty() || *end != 0) return fail(FWBF_E_PARSE, "bad block '" + tok + "'");
            if (v < 0 || v >= Z) return fail(FWBF_E_PARSE, "shift out of range [0, Z) in '" + tok + "'");
            auto &cell = cells[(size_t)t];
            if (std::find(cell.begin(), cell.end(), (int)v) != cell.end())
                return fail(FWBF_E_PARSE, "repeated shift in '" + tok + "'");
            cell.push_back((int)v);
            if (comma == std::string::npos) break;
            at = comma + 1;
        }
    }
    std::string extra;
    if (lx.next(extra)) return fail(FWBF_E_PARSE, "trailing text '" + extra + "'");
    return make_code((int)mb, (int)nb, (int)Z, std::move(cells), out);
}

int fwbf_code_from_seed(int mb, int nb, int Z, uint64_t seed, int min_girth, fwbf_code **out)
{
    if (!out) return fail(FWBF_E_INVALID, "null argument");
    *out = nullptr;
    if (mb < 1 || nb < 1 || Z < 1 || Z > 65535 || (long)nb * Z > 65535 || (long)mb * Z > 65535)
        return fail(FWBF_E_INVALID, "dimensions out of range");
    if (min_girth != 4 && min_girth != 6) return fail(FWBF_E_INVALID, "min_girth must be 4 or 6");
    SplitMix64 g{seed};
    std::vector<int> sh((size_t)mb * nb);
    for (int attempt = 0; attempt < 100000; attempt++) {
        for (auto &v : sh) v = (int)(g.next() % (uint64_t)Z);
        if (min_girth == 6 && base_has_4cycle(mb, nb, Z, sh.data())) continue;
        return make_code(mb, nb, Z, sh, out);
    }
    return fail(FWBF_E_GIRTH, "no base without 4-cycles in 100000 draws");
}

int fwbf_code_to_text(const fwbf_code *c, char *buf, size_t cap, size_t *needed)
{
    if (!c) return fail(FWBF_E_INVALID, "null code");
    std::ostringstream os;
    os << "qc-ldpc v1\nZ " << c->Z << "\nbase " << c->mb << " " << c->nb << "\n";
    for (int i = 0; i < c->mb; i++) {
        for (int j = 0; j < c->nb; j++) {
            const auto &v = c->cells[(size_t)i * c->nb + j];
            os << (j ? " " : "");
            if (v.empty()) os << -1;
            for (size_t u = 0; u < v.size(); u++) os << (u ? "," : "") << v[u];
        }
        os << "\n";
    }
    std::string s = os.str();
    if (needed) *needed = s.size() + 1;
    if (!buf || cap < s.size() + 1) return fail(FWBF_E_INVALID, "buffer too small");
    memcpy(buf, s.c_str(), s.size() + 1);
    return FWBF_OK;
}

int fwbf_code_dims(const fwbf_code *cc, int *N, int *M, int *K, int *dv_max, int *dc_max)
{
    if (!cc) return fail(FWBF_E_INVALID, "null code");
    fwbf_code *c = const_cast<fwbf_code *>(cc);  // lazy rank cache only
    if (N) *N = c->N;
    if (M) *M = c->M;
    if (dv_max) *dv_max = c->dv_max;
    if (dc_max) *dc_max = c->dc_max;
    if (K) {
        int rc = ensure_rref(c);
        if (rc) return rc;
        *K = c->K;
    }
    return FWBF_OK;
}

int fwbf_code_shifts(const fwbf_code *c, int *mb, int *nb, int *Z, int *shifts)
{
    if (!c) return fail(FWBF_E_INVALID, "null code");
    if (mb) *mb = c->mb;
    if (nb) *nb = c->nb;
    if (Z) *Z = c->Z;
    if (shifts && c->multi)
        return fail(FWBF_E_UNSUPPORTED, "the base has blocks with several shifts (use fwbf_code_to_text)");
    if (shifts) memcpy(shifts, c->shift.data(), sizeof(int) * c->shift.size());
    return FWBF_OK;
}

int fwbf_code_has_4cycle(const fwbf_code *c)
{
    if (!c) return fail(FWBF_E_INVALID, "null code");
    if (c->multi) return expanded_has_4cycle(c) ? 1 : 0;
    return base_has_4cycle(c->mb, c->nb, c->Z, c->shift.data()) ? 1 : 0;
}

void fwbf_code_free(fwbf_code *c)
{
    if (!c) return;
    for (auto &kv : c->dev) {
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && hipSetDevice(kv.first) == hipSuccess) {
            (void)hipFree(kv.second.shift);
            (void)hipSetDevice(cur);
        }
    }
    delete c;
}

int fwbf_code_info_positions(const fwbf_code *cc, int *out)
{
    if (!cc || !out) return fail(FWBF_E_INVALID, "null argument");
    fwbf_code *c = const_cast<fwbf_code *>(cc);
    int rc = ensure_rref(c);
    if (rc) return rc;
    memcpy(out, c->info.data(), sizeof(int) * c->info.size());
    return FWBF_OK;
}

int fwbf_encode(const fwbf_code *cc, uint64_t seed, int64_t first, int64_t count, uint32_t *out)
{
    if (!cc || (!out && count > 0) || first < 0 || count < 0)
        return fail(FWBF_E_INVALID, "invalid argument");
    fwbf_code *c = const_cast<fwbf_code *>(cc);
    int rc = ensure_rref(c);
    if (rc) return rc;
    const int W = c->words, NW = (c->N + 31) / 32;
    const uint64_t chunks = (uint64_t)(c->K + 63) / 64;
    std::vector<uint64_t> cw(W);
    for (int64_t w = 0; w < count; w++) {
        std::fill(cw.begin(), cw.end(), 0);
        const uint64_t base = (uint64_t)(first + w) * chunks;
        uint64_t word = 0;
        for (int k = 0; k < c->K; k++) {
            if (k % 64 == 0) word = SplitMix64::at(seed, base + k / 64);
            if ((word >> (k % 64)) & 1) cw[c->info[k] / 64] |= 1ULL << (c->info[k] % 64);
        }
        for (int r = 0; r < c->rank; r++) {
            const uint64_t *row = &c->rref[(size_t)r * W];
            uint64_t acc = 0;
            for (int t = 0; t < W; t++) acc ^= row[t] & cw[t];
            if (__builtin_popcountll(acc) & 1) cw[c->piv[r] / 64] |= 1ULL << (c->piv[r] % 64);
        }
        uint32_t *o = out + (size_t)w * NW;
        for (int t = 0; t < NW; t++) o[t] = (uint32_t)(cw[t >> 1] >> ((t & 1) * 32));
    }
    return FWBF_OK;
}

}  // extern "C"
