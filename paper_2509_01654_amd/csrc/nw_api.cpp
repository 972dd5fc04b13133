// nw_api.cpp -- host runtime behind include/nw.h: argument validation, the
// device layout of a dictionary (length-sorted blocks, row pairs, similarity
// table), range proofs for the 16-bit DP, and the kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nw.h"
#include "nw_internal.h"

using namespace nw;

struct nw_vocab {
    DevVocab dev;
    uint64_t n = 0;
    uint32_t max_len = 0;
    uint64_t num_pairs = 0;
    uint64_t num_cells = 0;
    int32_t lo = 0, hi = 0;      // score bounds
    bool symmetric = true;
    void *d_mem = nullptr;
    uint64_t d_bytes = 0;
};

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    return NW_OK;
}

int dev_fail(hipError_t e, const char *what)
{
    return fail(NW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

int choose_block(uint64_t n) { return n <= 16384 ? 256 : 1024; }


// Byte offsets of every region inside d_mem.
struct Layout {
    uint64_t csym, clen, bsym, blen, bcol, rpairs, rp_off, wtab, submat, total;
    int CB, WB, nb;
};

Layout make_layout(uint64_t n, uint32_t max_len)
{
    Layout L{};
    L.CB = choose_block(n);
    (void)max_len;
    L.WB = kWordBytes;
    L.nb = (int)((n + L.CB - 1) / L.CB);
    const uint64_t slots = (uint64_t)L.nb * L.CB;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align_up(o + (bytes ? bytes : 1), 256);
        return at;
    };
    L.csym = take(n * L.WB);
    L.clen = take(n);
    L.bsym = take(slots * L.WB);
    L.blen = take(slots);
    L.bcol = take(slots * 2);
    L.rpairs = take(slots * 2 * 4);
    L.rp_off = take(((uint64_t)L.nb * (kMaxLen + 1) + 1) * 4);
    L.wtab = take(256 * 256 * 2);
    L.submat = take(256 * 256);
    L.total = o;
    return L;
}

uint16_t f16_bits_of_int(int v)
{
    // exact for |v| <= 2048 (checked by the caller)
    _Float16 h = (_Float16)v;
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}

}  // namespace

extern "C" {

const char *nw_last_error(void) { return g_err.c_str(); }

int nw_max_word_length(void) { return kMaxLen; }

int nw_vocab_bytes(uint64_t n, uint64_t total_symbols, uint32_t max_len, uint64_t *dev_bytes)
{
    (void)total_symbols;
    if (!dev_bytes) return fail(NW_EINVAL, "dev_bytes is NULL");
    if (max_len > (uint32_t)kMaxLen) return fail(NW_EINVAL, "max_len %u exceeds the maximum word length %d", max_len, kMaxLen);
    if (n >= (1ull << 31)) return fail(NW_EINVAL, "n must be < 2^31");
    *dev_bytes = make_layout(n, max_len).total;
    return ok();
}

int nw_load_vocab(const uint8_t *h_symbols, const uint64_t *h_offsets, uint64_t n, const nw_scoring *sc, void *d_mem,
                  uint64_t d_bytes, void *hip_stream, nw_vocab **out)
{
    if (!out) return fail(NW_EINVAL, "out is NULL");
    *out = nullptr;
    if (!sc) return fail(NW_EINVAL, "scoring is NULL");
    if (!h_offsets) return fail(NW_EINVAL, "offsets is NULL");
    if (n >= (1ull << 31)) return fail(NW_EINVAL, "n must be < 2^31");
    const int A = sc->alphabet;
    if (A < 1 || A > 255) return fail(NW_EINVAL, "alphabet %d outside 1..255", A);
    if (sc->gap > 0) return fail(NW_EINVAL, "gap penalty %d must be <= 0", sc->gap);
    if (sc->gap < -1024) return fail(NW_ERANGE, "gap penalty %d below -1024", sc->gap);

    // words
    uint32_t max_len = 0;
    uint64_t sum_l = 0, sum_l2 = 0;
    if (h_offsets[0] != 0) return fail(NW_EINVAL, "offsets[0] must be 0");
    for (uint64_t i = 0; i < n; ++i) {
        if (h_offsets[i + 1] < h_offsets[i]) return fail(NW_EINVAL, "offsets decrease at word %llu", (unsigned long long)i);
        const uint64_t l = h_offsets[i + 1] - h_offsets[i];
        if (l > (uint64_t)kMaxLen)
            return fail(NW_EINVAL, "word %llu has %llu symbols; the maximum is %d", (unsigned long long)i,
                        (unsigned long long)l, kMaxLen);
        max_len = std::max<uint32_t>(max_len, (uint32_t)l);
        sum_l += l;
        sum_l2 += l * l;
    }
    if (sum_l > 0 && !h_symbols) return fail(NW_EINVAL, "symbols is NULL");
    for (uint64_t t = 0; t < sum_l; ++t)
        if (h_symbols[t] >= A) return fail(NW_EINVAL, "symbol %u at position %llu is >= alphabet %d", h_symbols[t], (unsigned long long)t, A);

    // similarity, shifted weights w = sim - 2p, and the range proofs
    std::vector<int> sim((size_t)A * A);
    bool symmetric = true;
    for (int x = 0; x < A; ++x)
        for (int y = 0; y < A; ++y)
            sim[(size_t)x * A + y] = sc->submat ? (int)sc->submat[(size_t)x * A + y] : (x == y ? sc->match : sc->mismatch);
    for (int x = 0; x < A; ++x)
        for (int y = 0; y < x; ++y)
            if (sim[(size_t)x * A + y] != sim[(size_t)y * A + x]) symmetric = false;
    int smin = sim[0], smax = sim[0];
    for (int s : sim) { smin = std::min(smin, s); smax = std::max(smax, s); }
    if (!sc->submat && (std::abs((long)sc->match) > 1024 || std::abs((long)sc->mismatch) > 1024))
        return fail(NW_ERANGE, "match/mismatch must lie in [-1024, 1024]");
    const long wmax = (long)smax - 2L * sc->gap, wmin = (long)smin - 2L * sc->gap;
    // every DP value G lies in [0, L*max(wmax,0)] and every candidate in
    // [wmin, L*max(wmax,0)]; binary16 holds them exactly up to 2048
    if ((long)max_len * std::max(wmax, 0L) > 2048 || wmin < -2048)
        return fail(NW_ERANGE, "DP values (%ld .. %ld) leave the exact 16-bit range [-2048, 2048]",
                    std::min(wmin, 0L), (long)max_len * std::max(wmax, 0L));
    const long lo = (long)max_len * std::min({(long)smin, (long)sc->gap, 0L});
    const long hi = (long)max_len * std::max((long)smax, 0L);
    if (lo < -32768 || hi > 32767) return fail(NW_ERANGE, "score bounds [%ld, %ld] leave int16", lo, hi);

    const Layout L = make_layout(n, max_len);
    if (!d_mem) return fail(NW_EINVAL, "d_mem is NULL");
    if ((uintptr_t)d_mem % 256) return fail(NW_EINVAL, "d_mem must be 256-byte aligned");
    if (d_bytes < L.total)
        return fail(NW_ENOMEM, "d_mem holds %llu bytes; the dictionary needs %llu", (unsigned long long)d_bytes,
                    (unsigned long long)L.total);

    // host image of the device layout
    std::vector<uint8_t> img(L.total, 0);
    // lane words are padded with the sentinel symbol (= alphabet)
    std::memset(img.data() + L.bsym, A, (size_t)L.nb * L.CB * L.WB);
    uint8_t *csym = img.data() + L.csym;
    uint8_t *clen = img.data() + L.clen;
    uint8_t *bsym = img.data() + L.bsym;
    uint8_t *blen = img.data() + L.blen;
    uint16_t *bcol = reinterpret_cast<uint16_t *>(img.data() + L.bcol);
    int32_t *rpairs = reinterpret_cast<int32_t *>(img.data() + L.rpairs);
    uint32_t *rp_off = reinterpret_cast<uint32_t *>(img.data() + L.rp_off);
    uint16_t *wtab = reinterpret_cast<uint16_t *>(img.data() + L.wtab);
    int8_t *submat = reinterpret_cast<int8_t *>(img.data() + L.submat);

    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t l = h_offsets[i + 1] - h_offsets[i];
        clen[i] = (uint8_t)l;
        if (l) std::memcpy(csym + i * L.WB, h_symbols + h_offsets[i], l);
    }
    const int LM = (int)max_len;
    uint32_t npairs = 0;
    std::vector<std::vector<int>> by_len(LM + 1);
    for (int blk = 0; blk < L.nb; ++blk) {
        const uint64_t u0 = (uint64_t)blk * L.CB;
        const uint64_t u1 = std::min<uint64_t>(u0 + L.CB, n);
        for (auto &v : by_len) v.clear();
        for (uint64_t u = u0; u < u1; ++u) by_len[clen[u]].push_back((int)(u - u0));
        // padding slots first (length 0, marked by column 0xFFFF), then real words by length
        uint64_t s = u0;
        for (uint64_t p = u1; p < u0 + L.CB; ++p, ++s) { blen[s] = 0; bcol[s] = 0xFFFF; }
        std::vector<uint64_t> slot_of(L.CB);
        for (int l = 0; l <= LM; ++l)
            for (int c : by_len[l]) {
                blen[s] = (uint8_t)l;
                bcol[s] = (uint16_t)c;
                if (l) std::memcpy(bsym + s * L.WB, csym + (u0 + c) * L.WB, l);
                slot_of[c] = s;
                ++s;
            }
        for (int l = 0; l <= LM; ++l) {
            rp_off[(size_t)blk * (LM + 1) + l] = npairs;
            const auto &v = by_len[l];
            for (size_t t = 0; t < v.size(); t += 2) {
                rpairs[2 * npairs] = (int32_t)slot_of[v[t]];
                rpairs[2 * npairs + 1] = t + 1 < v.size() ? (int32_t)slot_of[v[t + 1]] : -1;
                ++npairs;
            }
        }
    }
    rp_off[(size_t)L.nb * (LM + 1)] = npairs;
    for (int x = 0; x < A; ++x)
        for (int y = 0; y < A; ++y) {
            wtab[(size_t)x * A + y] = f16_bits_of_int(sim[(size_t)x * A + y] - 2 * sc->gap);
            submat[(size_t)x * A + y] = (int8_t)sim[(size_t)x * A + y];
        }

    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(d_mem, img.data(), L.total, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return dev_fail(e, "copying the dictionary");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_fail(e, "copying the dictionary");

    nw_vocab *v = new nw_vocab();
    uint8_t *base = static_cast<uint8_t *>(d_mem);
    DevVocab &D = v->dev;
    D.csym = base + L.csym;
    D.clen = base + L.clen;
    D.bsym = base + L.bsym;
    D.blen = base + L.blen;
    D.bcol = reinterpret_cast<const uint16_t *>(base + L.bcol);
    D.rpairs = reinterpret_cast<const int32_t *>(base + L.rpairs);
    D.rp_off = reinterpret_cast<const uint32_t *>(base + L.rp_off);
    D.wtab = reinterpret_cast<const uint16_t *>(base + L.wtab);
    D.submat = reinterpret_cast<const int8_t *>(base + L.submat);
    D.n = (int64_t)n;
    D.nb = L.nb;
    D.CB = L.CB;
    D.WB = L.WB;
    D.lmax = LM;
    D.alphabet = A;
    D.gap = sc->gap;
    D.match = sc->match;
    D.mismatch = sc->mismatch;
    D.has_submat = sc->submat ? 1 : 0;
    v->n = n;
    v->max_len = max_len;
    v->num_pairs = n * (n ? n - 1 : 0) / 2;
    v->num_cells = (sum_l * sum_l - sum_l2) / 2;
    v->lo = (int32_t)lo;
    v->hi = (int32_t)hi;
    v->symmetric = symmetric;
    v->d_mem = d_mem;
    v->d_bytes = d_bytes;
    *out = v;
    return ok();
}

void nw_free_vocab(nw_vocab *v) { delete v; }

int nw_vocab_info(const nw_vocab *v, uint64_t *n, uint32_t *max_len, uint64_t *num_pairs, uint64_t *num_cells)
{
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    if (n) *n = v->n;
    if (max_len) *max_len = v->max_len;
    if (num_pairs) *num_pairs = v->num_pairs;
    if (num_cells) *num_cells = v->num_cells;
    return ok();
}

int nw_score_bounds(const nw_vocab *v, int32_t *lo, int32_t *hi)
{
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    if (lo) *lo = v->lo;
    if (hi) *hi = v->hi;
    return ok();
}

static int check_triangle_args(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, void *d_out)
{
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    if (dt != NW_I8 && dt != NW_I16) return fail(NW_EINVAL, "dtype must be NW_I8 or NW_I16");
    if (idx_begin > idx_end || idx_end > v->num_pairs)
        return fail(NW_EINVAL, "pair range [%llu, %llu) outside [0, %llu]", (unsigned long long)idx_begin,
                    (unsigned long long)idx_end, (unsigned long long)v->num_pairs);
    if (!v->symmetric) return fail(NW_EINVAL, "all-pairs scoring needs a symmetric similarity matrix");
    if (dt == NW_I8 && (v->lo < -128 || v->hi > 127))
        return fail(NW_ERANGE, "score bounds [%d, %d] do not fit int8", v->lo, v->hi);
    if (idx_end > idx_begin && !d_out) return fail(NW_EINVAL, "d_out is NULL");
    return NW_OK;
}

int nw_all_pairs_scores(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, void *d_out,
                        void *hip_stream)
{
    int rc = check_triangle_args(v, idx_begin, idx_end, dt, d_out);
    if (rc) return rc;
    hipError_t e = launch_triangle_tiled(v->dev, idx_begin, idx_end, dt == NW_I8 ? OUT_I8 : OUT_I16, d_out,
                                         (hipStream_t)hip_stream);
    if (e != hipSuccess) return dev_fail(e, "launching the tiled triangle kernel");
    return ok();
}

int nw_all_pairs_scores_naive(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, void *d_out,
                              void *hip_stream)
{
    int rc = check_triangle_args(v, idx_begin, idx_end, dt, d_out);
    if (rc) return rc;
    hipError_t e = launch_triangle_naive(v->dev, idx_begin, idx_end, dt == NW_I8 ? OUT_I8 : OUT_I16, d_out,
                                         (hipStream_t)hip_stream);
    if (e != hipSuccess) return dev_fail(e, "launching the naive triangle kernel");
    return ok();
}

}  // extern "C"
