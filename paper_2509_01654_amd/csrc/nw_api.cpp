// nw_api.cpp -- host runtime behind include/nw.h: argument validation, the
// device layout of a dictionary (length-sorted blocks, row pairs, similarity
// table), range proofs for the 16-bit DP, and the kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nw.h"
#include "k_topk.h"
#include "nw_host.h"
#include "nw_internal.h"

using namespace nw;

namespace nw {
namespace host {

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

int refuse_capture(hipStream_t stream, const char *call)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return dev_fail(e, call);
    if (cs != hipStreamCaptureStatusNone)
        return fail(NW_EINVAL, "%s cannot be captured into a graph (the stream is capturing)", call);
    return NW_OK;
}

// Block size: small dictionaries need many workgroups; large ones amortise
// the per-step work (profile build, barrier, row stores) over more lane
// words, which matters most for short rows (a step's DP is short): up to
// 24-symbol words, blocks of 2048 from 32k words on (50k-word triangle
// 3.15 -> 2.98 ms); with longer words 1024 up to 131k words (2048 made the
// batched workload's 40k..100k-word dictionaries of words up to 31..48
// symbols 7 % slower).  Past 131k words, blocks of 3072: the 600k-word top-k
// main pass took 420 ms with 2048, 413 with 2560, 407 with 3072, 410 with
// 3584 and 417 with 4096 (the 50k-word triangle is slower with 3072).
int choose_block(uint64_t n, uint32_t max_len)
{
    if (n <= 16384) return 256;
    if (n <= 32768) return 1024;
    if (n <= 131072) return max_len > 24 ? 1024 : 2048;
    return 3072;
}


// Probe subset of the top-k threshold pre-pass.
constexpr uint64_t kMaxProbes = 8192;
uint64_t num_probes(uint64_t n) { return n < kMaxProbes ? n : kMaxProbes; }
// The first phase of the top-k main pass takes the block pairs (r, b) with
// (b - r) mod kPhasePeriod == 0.
constexpr int kPhasePeriod = 8;

// Byte offsets of every region inside d_mem.
struct Layout {
    uint64_t csym, clen, bsym, blen, bcol, rpairs, rp_off, dpairs, dp_off, wtab, submat, borig, gpairs, gp_off, psym, plen,
        porig, prank, total;
    int CB, WB, nb;
    uint64_t nprobe, pslots;
};

Layout make_layout(uint64_t n, uint32_t max_len)
{
    Layout L{};
    L.CB = choose_block(n, max_len);
    L.WB = max_len <= (uint32_t)kMaxLen ? kWordBytes : 256;   // whole 16-byte units
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
    L.rp_off = take(((uint64_t)L.nb * (std::max<uint32_t>(max_len, 1) + 1) + 1) * 4);
    // at most one half-empty pair per block and class
    L.dpairs = take((slots / 2 + (uint64_t)L.nb * kDiagClasses) * 2 * 4);
    L.dp_off = take(((uint64_t)L.nb * kDiagClasses + 1) * 4);
    L.wtab = take(256 * 256 * 2);
    L.submat = take(256 * 256);
    L.borig = take(slots * 4);
    L.gpairs = take(slots * 2 * 4);
    L.gp_off = take((kMaxLen + 2) * 4);
    L.nprobe = num_probes(n);
    L.pslots = (L.nprobe + kThreads - 1) / kThreads * kThreads;
    L.psym = take(L.pslots * L.WB);
    L.plen = take(L.pslots);
    L.porig = take(L.pslots * 4);
    L.prank = take(L.pslots * 2);
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

}  // namespace host
}  // namespace nw

namespace nw {
namespace host {

// ---------------------------------------------------------------- top-k
struct TopkWs {
    uint64_t thr, cnt, ovf, partial, lists, total;
    uint32_t cap;
};

uint32_t topk_cap(uint64_t n, uint64_t CB, uint32_t k)
{
    // Expected candidates of one word.  The probe threshold is the (k+1)-th
    // best key over M probe words and ranks about all = (k+1)(n-1)/M among
    // the n-1 partners.  The first phase meets the share f of the partners in
    // the block columns of its period and appends about f * all of them.  A
    // word with at least k has its threshold raised to their k-th best, which
    // ranks about k/f overall, and the second phase appends fewer than that;
    // otherwise the probe threshold stays and it appends up to `all`.  Twice
    // the sum, plus a margin, bounds the list in practice; a word past the
    // capacity is recomputed exactly.
    const uint64_t M = num_probes(n);
    const uint64_t nb = std::max<uint64_t>(1, (n + CB - 1) / CB);
    const double f = std::min(1.0, (double)((nb + kPhasePeriod - 1) / kPhasePeriod) / (double)nb);
    const double all = M >= n ? (double)(k + 1) : (double)(k + 1) * (double)(n - 1) / (double)M;
    const double first = f * all;
    const double second = first >= 2.0 * k ? (double)k / f : all;
    const double mean = first + second;
    uint64_t cap = (uint64_t)(2.0 * mean) + 64;
    cap = (cap + 63) / 64 * 64;
    const uint64_t most = (n + 63) / 64 * 64;
    cap = std::max<uint64_t>(64, std::min(cap, most));
    // NW_TOPK_CAP overrides the capacity (tests use it to force the
    // overflow recomputation)
    if (const char *env = std::getenv("NW_TOPK_CAP")) {
        const long c = std::atol(env);
        if (c > 0) cap = (uint64_t)c;
    }
    return (uint32_t)cap;
}

// lists_prepass: the pre-pass keeps wave lists (wide score codes), which need
// the partial area; the selection pre-pass writes the thresholds directly.
TopkWs topk_ws(uint64_t n, uint64_t CB, uint32_t k, bool lists_prepass)
{
    TopkWs w{};
    w.cap = topk_cap(n, CB, k);
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align_up(o + (bytes ? bytes : 1), 256);
        return at;
    };
    w.thr = take(8 * n);
    w.cnt = take(4 * n);
    w.ovf = take(4 + 4 * n);
    w.partial = take(lists_prepass ? 8 * n * (uint64_t)query_lists(1) * (k + 1) : 0);
    w.lists = take(8 * n * (uint64_t)w.cap);
    w.total = o;
    return w;
}

// ---------------------------------------------------------------- queries

int query_splits(uint64_t n_q)
{
    // enough workgroups to fill the GPU when few queries are in flight
    const uint64_t pairs = (n_q + 1) / 2;
    uint64_t s = pairs ? (2048 + pairs - 1) / pairs : 1;
    return (int)std::min<uint64_t>(256, std::max<uint64_t>(1, s));
}

QueryWs query_ws(uint64_t n_q, uint32_t k)
{
    QueryWs w{};
    w.nsplit = query_splits(n_q);
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align_up(o + (bytes ? bytes : 1), 256);
        return at;
    };
    w.sym = take(n_q * kWordBytes);
    w.pairs = take((n_q + kMaxLen + 1) * 8);
    w.off = take((kMaxLen + 2) * 4);
    w.orig = take(n_q * 4);
    w.partial = take(n_q * (uint64_t)query_lists(w.nsplit) * k * 8);
    w.total = o;
    return w;
}


// words: (length, pointer to symbols, output row)
RowImage make_rows(const std::vector<std::pair<int, std::pair<const uint8_t *, int32_t>>> &words)
{
    RowImage R;
    const size_t m = words.size();
    R.sym.assign(m * kWordBytes, 0);
    R.orig.assign(m, -1);
    R.off.assign(kMaxLen + 2, 0);
    std::vector<size_t> order(m);
    for (size_t i = 0; i < m; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return words[a].first < words[b].first; });
    for (size_t s = 0; s < m; ++s) {
        const auto &w = words[order[s]];
        if (w.first) std::memcpy(&R.sym[s * kWordBytes], w.second.first, w.first);
        R.orig[s] = w.second.second;
    }
    size_t s = 0;
    for (int l = 0; l <= kMaxLen; ++l) {
        R.off[l] = (uint32_t)(R.pairs.size() / 2);
        size_t e = s;
        while (e < m && words[order[e]].first == l) ++e;
        for (size_t t = s; t < e; t += 2) {
            R.pairs.push_back((int32_t)t);
            R.pairs.push_back(t + 1 < e ? (int32_t)(t + 1) : -1);
        }
        s = e;
    }
    R.off[kMaxLen + 1] = (uint32_t)(R.pairs.size() / 2);
    return R;
}

long query_lo(const nw_vocab *v, uint32_t qmax)
{
    // scores of a query pair lie in [max(lq, ld) * min(smin, p, 0), min(lq, ld) * max(smax, 0)]
    const long L = std::max<long>(qmax, v->max_len);
    return std::min<long>(v->dev.lo, L * std::min({(long)v->smin, (long)v->dev.gap, 0L}));
}

ColSet full_colset(const DevVocab &D)
{
    ColSet C;
    C.sym = D.bsym;
    C.len = D.blen;
    C.orig = D.borig;
    C.nslots = (int64_t)D.nb * D.CB;
    return C;
}

}  // namespace host
}  // namespace nw

using namespace nw::host;

int nw::host::check_triangle_args(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt,
                                  const void *d_out)
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

hipError_t nw::host::launch_triangle(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, void *d_out,
                                     hipStream_t stream)
{
    // words longer than the register-row limit take the anti-diagonal kernel
    const int kind = dt == NW_I8 ? OUT_I8 : OUT_I16;
    return v->max_len > (uint32_t)kMaxLen ? launch_triangle_diag(v->dev, v->h_maxrp.data(), v->h_maxdp, idx_begin, idx_end, kind, d_out, stream)
                                          : launch_triangle_tiled(v->dev, v->h_maxrp.data(), idx_begin, idx_end, kind, d_out, stream);
}

extern "C" {

const char *nw_last_error(void) { return g_err.c_str(); }

int nw_max_word_length(void) { return kLongMaxLen; }

int nw_vocab_bytes(uint64_t n, uint64_t total_symbols, uint32_t max_len, uint64_t *dev_bytes)
{
    (void)total_symbols;
    if (!dev_bytes) return fail(NW_EINVAL, "dev_bytes is NULL");
    if (max_len > (uint32_t)kLongMaxLen) return fail(NW_EINVAL, "max_len %u exceeds the maximum word length %d", max_len, kLongMaxLen);
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
        if (l > (uint64_t)kLongMaxLen)
            return fail(NW_EINVAL, "word %llu has %llu symbols; the maximum is %d", (unsigned long long)i,
                        (unsigned long long)l, kLongMaxLen);
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
    if (int rc = refuse_capture((hipStream_t)hip_stream, "nw_load_vocab")) return rc;

    // host image of the device layout
    std::vector<uint8_t> img(L.total, 0);
    // lane words are padded with the sentinel symbol (= alphabet)
    std::memset(img.data() + L.bsym, A, (size_t)L.nb * L.CB * L.WB);
    std::memset(img.data() + L.psym, A, (size_t)L.pslots * L.WB);
    int32_t *borig = reinterpret_cast<int32_t *>(img.data() + L.borig);
    int32_t *gpairs = reinterpret_cast<int32_t *>(img.data() + L.gpairs);
    uint32_t *gp_off = reinterpret_cast<uint32_t *>(img.data() + L.gp_off);
    uint8_t *psym = img.data() + L.psym;
    uint8_t *plen = img.data() + L.plen;
    int32_t *porig = reinterpret_cast<int32_t *>(img.data() + L.porig);
    uint16_t *prank = reinterpret_cast<uint16_t *>(img.data() + L.prank);
    uint8_t *csym = img.data() + L.csym;
    uint8_t *clen = img.data() + L.clen;
    uint8_t *bsym = img.data() + L.bsym;
    uint8_t *blen = img.data() + L.blen;
    uint16_t *bcol = reinterpret_cast<uint16_t *>(img.data() + L.bcol);
    int32_t *rpairs = reinterpret_cast<int32_t *>(img.data() + L.rpairs);
    uint32_t *rp_off = reinterpret_cast<uint32_t *>(img.data() + L.rp_off);
    int32_t *dpairs = reinterpret_cast<int32_t *>(img.data() + L.dpairs);
    uint32_t *dp_off = reinterpret_cast<uint32_t *>(img.data() + L.dp_off);
    uint16_t *wtab = reinterpret_cast<uint16_t *>(img.data() + L.wtab);
    int8_t *submat = reinterpret_cast<int8_t *>(img.data() + L.submat);

    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t l = h_offsets[i + 1] - h_offsets[i];
        clen[i] = (uint8_t)l;
        if (l) std::memcpy(csym + i * L.WB, h_symbols + h_offsets[i], l);
    }
    const int LM = (int)max_len;
    uint32_t npairs = 0, ndpairs = 0;
    std::vector<std::vector<int>> by_len(LM + 1);
    for (int blk = 0; blk < L.nb; ++blk) {
        const uint64_t u0 = (uint64_t)blk * L.CB;
        const uint64_t u1 = std::min<uint64_t>(u0 + L.CB, n);
        for (auto &v : by_len) v.clear();
        for (uint64_t u = u0; u < u1; ++u) by_len[clen[u]].push_back((int)(u - u0));
        // within a length, words in lexicographic order (ties by caller index):
        // neighbouring lanes then often hold the same symbol in a column, and
        // lanes reading the same profile row share one LDS access
        for (int l = 1; l <= LM; ++l)
            std::sort(by_len[l].begin(), by_len[l].end(), [&](int a, int b) {
                const int c = std::memcmp(csym + (u0 + a) * L.WB, csym + (u0 + b) * L.WB, (size_t)l);
                return c != 0 ? c < 0 : a < b;
            });
        // padding slots first (length 0, marked by column 0xFFFF), then real words by length
        uint64_t s = u0;
        for (uint64_t p = u1; p < u0 + L.CB; ++p, ++s) { blen[s] = 0; bcol[s] = 0xFFFF; borig[s] = -1; }
        std::vector<uint64_t> slot_of(L.CB);
        for (int l = 0; l <= LM; ++l)
            for (int c : by_len[l]) {
                blen[s] = (uint8_t)l;
                bcol[s] = (uint16_t)c;
                borig[s] = (int32_t)(u0 + c);
                if (l) std::memcpy(bsym + s * L.WB, csym + (u0 + c) * L.WB, l);
                slot_of[c] = s;
                ++s;
            }
        // anti-diagonal classes: consecutive slots of one class (ascending lengths)
        for (int c = 0; c < kDiagClasses; ++c) {
            dp_off[(size_t)blk * kDiagClasses + c] = ndpairs;
            int32_t open = -1;
            for (uint64_t q = u0; q < u0 + L.CB; ++q) {
                const int l = blen[q];
                if (l < 32 * c + 1 || l > 32 * c + 32) continue;
                if (open < 0) {
                    open = (int32_t)q;
                } else {
                    dpairs[2 * ndpairs] = open;
                    dpairs[2 * ndpairs + 1] = (int32_t)q;
                    ++ndpairs;
                    open = -1;
                }
            }
            if (open >= 0) {
                dpairs[2 * ndpairs] = open;
                dpairs[2 * ndpairs + 1] = -1;
                ++ndpairs;
            }
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
    dp_off[(size_t)L.nb * kDiagClasses] = ndpairs;
    // the same row pairs grouped by length only
    std::vector<uint32_t> h_gp_off(kMaxLen + 2, 0);
    {
        uint32_t g = 0;
        for (int l = 0; l <= kMaxLen; ++l) {
            h_gp_off[l] = g;
            if (l <= LM)
                for (int blk = 0; blk < L.nb; ++blk) {
                    const uint32_t a = rp_off[(size_t)blk * (LM + 1) + l], b = rp_off[(size_t)blk * (LM + 1) + l + 1];
                    for (uint32_t t = a; t < b; ++t, ++g) {
                        gpairs[2 * g] = rpairs[2 * t];
                        gpairs[2 * g + 1] = rpairs[2 * t + 1];
                    }
                }
        }
        h_gp_off[kMaxLen + 1] = g;
        std::memcpy(gp_off, h_gp_off.data(), (kMaxLen + 2) * 4);
    }
    // probe subset: caller indices floor(i*n/M), sorted by length, padding slots first
    {
        // (length, rank i); u = floor(i n / M) rises with i, so this is (length, u)
        std::vector<std::pair<int, int64_t>> pr;
        for (uint64_t i = 0; i < L.nprobe; ++i) pr.push_back({clen[i * n / L.nprobe], (int64_t)i});
        std::stable_sort(pr.begin(), pr.end());
        uint64_t s = 0;
        for (; s < L.pslots - L.nprobe; ++s) { plen[s] = 0; porig[s] = -1; prank[s] = 0; }
        for (auto &e : pr) {
            const int64_t u = (int64_t)((uint64_t)e.second * n / L.nprobe);
            plen[s] = (uint8_t)e.first;
            porig[s] = (int32_t)u;
            prank[s] = (uint16_t)e.second;
            if (e.first) std::memcpy(psym + s * L.WB, csym + u * L.WB, e.first);
            ++s;
        }
    }
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
    D.dpairs = reinterpret_cast<const int32_t *>(base + L.dpairs);
    D.dp_off = reinterpret_cast<const uint32_t *>(base + L.dp_off);
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
    D.borig = reinterpret_cast<const int32_t *>(base + L.borig);
    D.gpairs = reinterpret_cast<const int32_t *>(base + L.gpairs);
    D.gp_off = reinterpret_cast<const uint32_t *>(base + L.gp_off);
    D.psym = base + L.psym;
    D.plen = base + L.plen;
    D.porig = reinterpret_cast<const int32_t *>(base + L.porig);
    D.prank = reinterpret_cast<const uint16_t *>(base + L.prank);
    D.pslots = (int64_t)L.pslots;
    D.nprobe = (int32_t)L.nprobe;
    D.lo = (int32_t)lo;
    D.hi = (int32_t)hi;
    v->h_gp_off = h_gp_off;
    v->h_csym.assign(csym, csym + n * L.WB);
    v->h_clen.assign(clen, clen + n);
    v->h_rp_off.assign(rp_off, rp_off + (size_t)L.nb * (LM + 1) + 1);
    v->h_maxrp.assign(LM + 1, 0);
    for (uint64_t r = 0; r < L.nb; ++r)
        for (uint32_t la = 0; la <= LM; ++la) {
            const uint32_t c = rp_off[r * (LM + 1) + la + 1] - rp_off[r * (LM + 1) + la];
            v->h_maxrp[la] = std::max(v->h_maxrp[la], c);
        }
    for (uint64_t r = 0; r < L.nb; ++r)
        for (int c = 0; c < kDiagClasses; ++c)
            v->h_maxdp[c] = std::max(v->h_maxdp[c], dp_off[r * kDiagClasses + c + 1] - dp_off[r * kDiagClasses + c]);
    v->smin = smin;
    v->smax = smax;
    v->n = n;
    v->max_len = max_len;
    v->num_pairs = n * (n ? n - 1 : 0) / 2;
    v->num_cells = (sum_l * sum_l - sum_l2) / 2;
    v->lo = (int32_t)lo;
    v->hi = (int32_t)hi;
    v->symmetric = symmetric;
    v->d_mem = d_mem;
    hipGetDevice(&v->device);
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


int nw_all_pairs_scores(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, void *d_out,
                        void *hip_stream)
{
    int rc = check_triangle_args(v, idx_begin, idx_end, dt, d_out);
    if (rc) return rc;
    DeviceScope scope(v->device);
    hipError_t e = launch_triangle(v, idx_begin, idx_end, dt, d_out, (hipStream_t)hip_stream);
    if (e != hipSuccess) return dev_fail(e, "launching the triangle kernels");
    return ok();
}


int nw_all_pairs_scores_diag(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, void *d_out,
                             void *hip_stream)
{
    int rc = check_triangle_args(v, idx_begin, idx_end, dt, d_out);
    if (rc) return rc;
    DeviceScope scope(v->device);
    hipError_t e = launch_triangle_diag(v->dev, v->h_maxrp.data(), v->h_maxdp, idx_begin, idx_end, dt == NW_I8 ? OUT_I8 : OUT_I16, d_out,
                                        (hipStream_t)hip_stream);
    if (e != hipSuccess) return dev_fail(e, "launching the anti-diagonal triangle kernel");
    return ok();
}

int nw_all_pairs_scores_naive(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, void *d_out,
                              void *hip_stream)
{
    int rc = check_triangle_args(v, idx_begin, idx_end, dt, d_out);
    if (rc) return rc;
    DeviceScope scope(v->device);
    hipError_t e = launch_triangle_naive(v->dev, idx_begin, idx_end, dt == NW_I8 ? OUT_I8 : OUT_I16, d_out,
                                         (hipStream_t)hip_stream);
    if (e != hipSuccess) return dev_fail(e, "launching the naive triangle kernel");
    return ok();
}


int nw_all_pairs_edges(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, const nw_edge_filter *f,
                       int32_t *d_i, int32_t *d_j, int16_t *d_score, uint64_t cap, uint64_t *d_count,
                       void *hip_stream)
{
    if (!v || !f || !d_count) return fail(NW_EINVAL, "NULL vocab, filter or count");
    if (f->mode != NW_EDGE_RAW && f->mode != NW_EDGE_NORMALISED)
        return fail(NW_EINVAL, "edge filter mode %d is not NW_EDGE_RAW or NW_EDGE_NORMALISED", f->mode);
    if (f->lo > f->hi) return fail(NW_EINVAL, "edge slice [%d, %d] is empty", f->lo, f->hi);
    if (f->mode == NW_EDGE_NORMALISED && (f->den < 1 || f->den > 1000000))
        return fail(NW_EINVAL, "edge slice denominator %d outside 1..1000000", f->den);
    if (cap > 0 && (!d_i || !d_j || !d_score)) return fail(NW_EINVAL, "NULL edge array with cap > 0");
    if (((uintptr_t)d_count & 7) || ((uintptr_t)d_i & 3) || ((uintptr_t)d_j & 3) || ((uintptr_t)d_score & 1))
        return fail(NW_EINVAL, "misaligned edge count or edge arrays");
    DeviceScope scope(v->device);
    if (idx_begin > idx_end || idx_end > v->num_pairs)
        return fail(NW_EINVAL, "pair range [%llu, %llu) outside [0, %llu]", (unsigned long long)idx_begin,
                    (unsigned long long)idx_end, (unsigned long long)v->num_pairs);
    if (!v->symmetric) return fail(NW_EINVAL, "all-pairs scoring needs a symmetric similarity matrix");

    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = launch_reset_counters(reinterpret_cast<uint32_t *>(d_count), 2, st);
    if (e != hipSuccess) return dev_fail(e, "clearing the edge counter");
    EdgeSink E{};
    E.ei = d_i;
    E.ej = d_j;
    E.es = d_score;
    E.count = reinterpret_cast<unsigned long long *>(d_count);
    E.cap = cap;
    E.normalised = f->mode == NW_EDGE_NORMALISED;
    E.lo = f->lo;
    E.hi = f->hi;
    E.den = f->mode == NW_EDGE_NORMALISED ? f->den : 1;
    e = v->max_len > (uint32_t)kMaxLen ? launch_triangle_diag(v->dev, v->h_maxrp.data(), v->h_maxdp, idx_begin, idx_end, OUT_EDGES, nullptr, st, &E)
                                       : launch_edges_tiled(v->dev, v->h_maxrp.data(), idx_begin, idx_end, E, st);
    if (e != hipSuccess) return dev_fail(e, "launching the edge kernels");
    return ok();
}


int nw_topk_workspace_bytes(const nw_vocab *v, uint32_t k, uint64_t *bytes)
{
    if (!v || !bytes) return fail(NW_EINVAL, "NULL argument");
    if (k < 1 || k > 63) return fail(NW_EINVAL, "k = %u outside 1..63", k);
    *bytes = topk_ws(v->n, (uint64_t)v->dev.CB, k, !probe_thr_applies(v->dev)).total;
    return ok();
}

namespace {

// Arguments shared by the top-k calls: NW_OK or the error already recorded.
int check_topk_args(const nw_vocab *v, uint32_t k, const int16_t *d_score, const int32_t *d_index, const void *d_ws,
                    uint64_t ws_bytes, hipStream_t st, const char *call)
{
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    if (k < 1 || k > 63) return fail(NW_EINVAL, "k = %u outside 1..63", k);
    if (!v->symmetric) return fail(NW_EINVAL, "all-pairs scoring needs a symmetric similarity matrix");
    if (v->max_len > (uint32_t)kMaxLen)
        return fail(NW_EINVAL, "top-k supports words of at most %d symbols (this dictionary has %u)", kMaxLen, v->max_len);
    const TopkWs W = topk_ws(v->n, (uint64_t)v->dev.CB, k, !probe_thr_applies(v->dev));
    if (v->n > 0 && (!d_score || !d_index)) return fail(NW_EINVAL, "d_score / d_index is NULL");
    if (!d_ws || (uintptr_t)d_ws % 256) return fail(NW_EINVAL, "d_ws must be a 256-byte aligned device pointer");
    if (ws_bytes < W.total)
        return fail(NW_ENOMEM, "workspace holds %llu bytes; top-k needs %llu", (unsigned long long)ws_bytes,
                    (unsigned long long)W.total);
    return refuse_capture(st, call);
}

// The pre-pass, the two main-pass phases and the selection, enqueued on st
// (arguments already checked, the dictionary's device current).
int topk_enqueue(const nw_vocab *v, uint32_t k, int16_t *d_score, int32_t *d_index, uint64_t *d_hist, void *d_ws,
                 hipStream_t st)
{
    const uint64_t n = v->n;
    const TopkWs W = topk_ws(n, (uint64_t)v->dev.CB, k, !probe_thr_applies(v->dev));
    const DevVocab &D = v->dev;
    const int nbins = v->hi - v->lo + 1;
    uint8_t *ws = static_cast<uint8_t *>(d_ws);
    uint64_t *thr = reinterpret_cast<uint64_t *>(ws + W.thr);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + W.cnt);
    uint32_t *ovf = reinterpret_cast<uint32_t *>(ws + W.ovf);
    uint64_t *partial = reinterpret_cast<uint64_t *>(ws + W.partial);
    uint64_t *lists = reinterpret_cast<uint64_t *>(ws + W.lists);
    hipError_t e;
    if (d_hist && (e = hipMemsetAsync(d_hist, 0, (size_t)nbins * 8, st)) != hipSuccess) return dev_fail(e, "clearing the histogram");
    if (n == 0) return ok();
    if ((e = hipMemsetAsync(cnt, 0, 4 * n, st)) != hipSuccess) return dev_fail(e, "clearing counters");
    if ((e = hipMemsetAsync(ovf, 0, 4, st)) != hipSuccess) return dev_fail(e, "clearing counters");

    nw_vocab *vm = const_cast<nw_vocab *>(v);
    for (auto &ev : vm->ev)
        if (!ev && (e = hipEventCreate(&ev)) != hipSuccess) return dev_fail(e, "creating timing events");
    if ((e = hipEventRecord(vm->ev[0], st)) != hipSuccess) return dev_fail(e, "recording a timing event");
    // 1. thresholds: each word's (k+1)-th best key over the probe subset
    RowSet R;
    R.sym = D.bsym;
    R.pairs = D.gpairs;
    R.off = D.gp_off;
    R.orig = D.borig;
    ColSet P;
    P.sym = D.psym;
    P.len = D.plen;
    P.orig = D.porig;
    P.nslots = D.pslots;
    if (probe_thr_applies(D)) {   // byte-wide score codes: selection, no lists
        if ((e = launch_probe_thr(D, R, v->h_gp_off.data(), (int)k + 1, thr, st)) != hipSuccess)
            return dev_fail(e, "launching the threshold pre-pass");
    } else {
        if ((e = launch_query(D, R, v->h_gp_off.data(), P, (int)k + 1, 1, partial, st, true)) != hipSuccess)
            return dev_fail(e, "launching the threshold pre-pass");
        if ((e = launch_merge(partial, query_lists(1), (int)k + 1, (int64_t)n, (int)k + 1, D.lo, nullptr, nullptr, thr, (int)k + 1, st)) != hipSuccess)
            return dev_fail(e, "launching the threshold merge");
    }
    if ((e = hipEventRecord(vm->ev[1], st)) != hipSuccess) return dev_fail(e, "recording a timing event");
    // 2. every unordered pair once: candidates for both endpoints, histogram.
    // Two phases: block pairs with (b - r) mod 8 == 0 first -- every word meets
    // an eighth of its partners, spread over the whole dictionary -- then each
    // word's threshold is raised to the k-th best of its candidates so far,
    // and the remaining block pairs emit far fewer candidates.
    TopkArgs T{};
    T.thr = thr;
    T.cnt = cnt;
    T.lists = lists;
    T.cap = W.cap;
    T.hist = reinterpret_cast<unsigned long long *>(d_hist);
    T.lo = D.lo;
    T.nbins = nbins;
    T.phase_mod = kPhasePeriod;
    T.phase_lo = 0;
    T.phase_hi = 0;
    if ((e = launch_topk_main(D, T, st)) != hipSuccess) return dev_fail(e, "launching the top-k main pass");
    if ((e = launch_tighten(cnt, lists, W.cap, (int64_t)n, (int)k, thr, st)) != hipSuccess)
        return dev_fail(e, "launching the threshold update");
    T.phase_lo = 1;
    T.phase_hi = kPhasePeriod - 1;
    if ((e = launch_topk_main(D, T, st)) != hipSuccess) return dev_fail(e, "launching the top-k main pass");
    if ((e = hipEventRecord(vm->ev[2], st)) != hipSuccess) return dev_fail(e, "recording a timing event");
    // 3. the best k of each word's candidates
    if ((e = launch_select(cnt, lists, W.cap, (int64_t)n, (int)k, D.lo, d_score, d_index, ovf, reinterpret_cast<int32_t *>(ovf + 1), st)) != hipSuccess)
        return dev_fail(e, "launching the top-k selection");
    if ((e = hipEventRecord(vm->ev[3], st)) != hipSuccess) return dev_fail(e, "recording a timing event");
    vm->topk_pending = true;
    return ok();
}

// Wait for the enqueued passes, then recompute exactly the words whose
// candidate list overflowed (their count and ids are read back to the host).
int topk_finish(const nw_vocab *v, uint32_t k, int16_t *d_score, int32_t *d_index, void *d_ws, hipStream_t st)
{
    const uint64_t n = v->n;
    const TopkWs W = topk_ws(n, (uint64_t)v->dev.CB, k, !probe_thr_applies(v->dev));
    nw_vocab *vm = const_cast<nw_vocab *>(v);
    const DevVocab &D = v->dev;
    uint8_t *ws = static_cast<uint8_t *>(d_ws);
    uint32_t *ovf = reinterpret_cast<uint32_t *>(ws + W.ovf);
    uint64_t *lists = reinterpret_cast<uint64_t *>(ws + W.lists);
    hipError_t e;
    // 4. words whose candidates overflowed the list: exact recomputation
    uint32_t novf = 0;
    if (n > 0 && (e = hipMemcpyAsync(&novf, ovf, 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return dev_fail(e, "reading the overflow count");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return dev_fail(e, "top-k");
    vm->last_overflow = novf;
    if (vm->topk_pending && n > 0)
        for (int ph = 0; ph < 3; ++ph)
            if ((e = hipEventElapsedTime(&vm->phase_ms[ph], vm->ev[ph], vm->ev[ph + 1])) != hipSuccess)
                return dev_fail(e, "reading timing events");
    vm->topk_pending = false;
    if (novf == 0) return ok();
    std::vector<int32_t> words(novf);
    if ((e = hipMemcpy(words.data(), ovf + 1, 4ull * novf, hipMemcpyDeviceToHost)) != hipSuccess) return dev_fail(e, "reading overflowed words");
    // Each overflowed word is a query of its own symbols against the whole
    // dictionary (k+1 best, the word itself dropped).  The list area is free
    // now; the words go through it in batches that fit.
    const int kq = (int)k + 1;
    const int nsplit = 16;
    const uint64_t area = 8 * n * (uint64_t)W.cap;
    const uint64_t fixed = align_up((kMaxLen + 2) * 4, 256) + 8 * 256;
    const uint64_t per_word = kWordBytes + 8 + 4 + 4 + (uint64_t)query_lists(nsplit) * kq * 8 + (uint64_t)kq * 6;
    const uint64_t batch = area > fixed ? (area - fixed) / per_word : 0;
    if (batch == 0) return fail(NW_ENOMEM, "the candidate lists are too small to recompute an overflowed word");
    for (uint64_t t0 = 0; t0 < novf; t0 += batch) {
        const uint32_t B = (uint32_t)std::min<uint64_t>(batch, novf - t0);
        std::vector<std::pair<int, std::pair<const uint8_t *, int32_t>>> rows;
        for (uint32_t t = 0; t < B; ++t) {
            const int32_t w = words[t0 + t];
            rows.push_back({v->h_clen[w], {&v->h_csym[(size_t)w * kWordBytes], (int32_t)t}});
        }
        RowImage img = make_rows(rows);
        uint8_t *q = reinterpret_cast<uint8_t *>(lists);
        uint8_t *qsym = q; q += align_up(img.sym.size(), 256);
        int32_t *qpairs = reinterpret_cast<int32_t *>(q); q += align_up(img.pairs.size() * 4 + 8, 256);
        uint32_t *qoff = reinterpret_cast<uint32_t *>(q); q += align_up((kMaxLen + 2) * 4, 256);
        int32_t *qorig = reinterpret_cast<int32_t *>(q); q += align_up(img.orig.size() * 4, 256);
        int32_t *qwords = reinterpret_cast<int32_t *>(q); q += align_up(4ull * B, 256);
        uint64_t *qpart = reinterpret_cast<uint64_t *>(q); q += align_up((uint64_t)B * query_lists(nsplit) * kq * 8, 256);
        int32_t *qi = reinterpret_cast<int32_t *>(q); q += align_up((uint64_t)B * kq * 4, 256);
        int16_t *qs = reinterpret_cast<int16_t *>(q);
        if ((e = hipMemcpy(qsym, img.sym.data(), img.sym.size(), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(qpairs, img.pairs.data(), img.pairs.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(qoff, img.off.data(), img.off.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(qorig, img.orig.data(), img.orig.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(qwords, words.data() + t0, 4ull * B, hipMemcpyHostToDevice)) != hipSuccess)
            return dev_fail(e, "uploading overflowed words");
        RowSet QR;
        QR.sym = qsym;
        QR.pairs = qpairs;
        QR.off = qoff;
        QR.orig = qorig;
        if ((e = launch_query(D, QR, img.off.data(), full_colset(D), kq, nsplit, qpart, st)) != hipSuccess ||
            (e = launch_merge(qpart, query_lists(nsplit), kq, B, kq, D.lo, qs, qi, nullptr, 1, st)) != hipSuccess ||
            (e = launch_scatter_lists(qs, qi, qwords, B, kq, (int)k, d_score, d_index, st)) != hipSuccess)
            return dev_fail(e, "launching the overflow recomputation");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return dev_fail(e, "recomputing overflowed words");
    }
    return ok();
}

}  // namespace

int nw_all_pairs_topk(const nw_vocab *v, uint32_t k, int16_t *d_score, int32_t *d_index, uint64_t *d_hist, void *d_ws,
                      uint64_t ws_bytes, void *hip_stream)
{
    hipStream_t st = (hipStream_t)hip_stream;
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    DeviceScope scope(v->device);
    int rc = check_topk_args(v, k, d_score, d_index, d_ws, ws_bytes, st, "nw_all_pairs_topk");
    if (rc) return rc;
    if ((rc = topk_enqueue(v, k, d_score, d_index, d_hist, d_ws, st))) return rc;
    return topk_finish(v, k, d_score, d_index, d_ws, st);
}

int nw_all_pairs_topk_async(const nw_vocab *v, uint32_t k, int16_t *d_score, int32_t *d_index, uint64_t *d_hist,
                            void *d_ws, uint64_t ws_bytes, void *hip_stream)
{
    hipStream_t st = (hipStream_t)hip_stream;
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    DeviceScope scope(v->device);
    int rc = check_topk_args(v, k, d_score, d_index, d_ws, ws_bytes, st, "nw_all_pairs_topk_async");
    if (rc) return rc;
    return topk_enqueue(v, k, d_score, d_index, d_hist, d_ws, st);
}

int nw_topk_finish(const nw_vocab *v, uint32_t k, int16_t *d_score, int32_t *d_index, void *d_ws, uint64_t ws_bytes,
                   void *hip_stream)
{
    hipStream_t st = (hipStream_t)hip_stream;
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    DeviceScope scope(v->device);
    int rc = check_topk_args(v, k, d_score, d_index, d_ws, ws_bytes, st, "nw_topk_finish");
    if (rc) return rc;
    if (!v->topk_pending && v->n > 0) return fail(NW_EINVAL, "no top-k pass is pending on this dictionary");
    return topk_finish(v, k, d_score, d_index, d_ws, st);
}

int nw_topk_phase_times(const nw_vocab *v, float *prepass_ms, float *main_ms, float *select_ms)
{
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    if (prepass_ms) *prepass_ms = v->phase_ms[0];
    if (main_ms) *main_ms = v->phase_ms[1];
    if (select_ms) *select_ms = v->phase_ms[2];
    return ok();
}

int nw_topk_overflow_words(const nw_vocab *v, uint32_t *words)
{
    if (!v || !words) return fail(NW_EINVAL, "NULL argument");
    *words = v->last_overflow;
    return ok();
}

int nw_query_workspace_bytes(const nw_vocab *v, uint64_t n_q, uint64_t q_symbols, uint32_t k, uint64_t *bytes)
{
    (void)q_symbols;
    if (!v || !bytes) return fail(NW_EINVAL, "NULL argument");
    if (k < 1 || k > 64) return fail(NW_EINVAL, "k = %u outside 1..64", k);
    *bytes = query_ws(n_q, k).total;
    return ok();
}

int nw_query(const nw_vocab *v, const uint8_t *h_q_symbols, const uint64_t *h_q_offsets, uint64_t n_q, uint32_t k,
             int16_t *d_score, int32_t *d_index, void *d_ws, uint64_t ws_bytes, void *hip_stream)
{
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    DeviceScope scope(v->device);
    if (k < 1 || k > 64) return fail(NW_EINVAL, "k = %u outside 1..64", k);
    if (n_q == 0) return ok();
    if (!h_q_offsets || !d_score || !d_index) return fail(NW_EINVAL, "NULL argument");
    if (n_q >= (1ull << 31)) return fail(NW_EINVAL, "n_q must be < 2^31");
    if (v->max_len > (uint32_t)kMaxLen)
        return fail(NW_EINVAL, "queries support dictionaries of words of at most %d symbols", kMaxLen);
    const QueryWs W = query_ws(n_q, k);
    if (!d_ws || (uintptr_t)d_ws % 256) return fail(NW_EINVAL, "d_ws must be a 256-byte aligned device pointer");
    if (ws_bytes < W.total)
        return fail(NW_ENOMEM, "workspace holds %llu bytes; the queries need %llu", (unsigned long long)ws_bytes,
                    (unsigned long long)W.total);
    const DevVocab &D = v->dev;
    const int A = D.alphabet;
    uint32_t qmax = 0;
    if (h_q_offsets[0] != 0) return fail(NW_EINVAL, "query offsets[0] must be 0");
    std::vector<std::pair<int, std::pair<const uint8_t *, int32_t>>> rows(n_q);
    for (uint64_t i = 0; i < n_q; ++i) {
        if (h_q_offsets[i + 1] < h_q_offsets[i]) return fail(NW_EINVAL, "query offsets decrease at %llu", (unsigned long long)i);
        const uint64_t l = h_q_offsets[i + 1] - h_q_offsets[i];
        if (l > (uint64_t)kMaxLen) return fail(NW_EINVAL, "query %llu has %llu symbols; the maximum is %d", (unsigned long long)i, (unsigned long long)l, kMaxLen);
        for (uint64_t t = 0; t < l; ++t)
            if (h_q_symbols[h_q_offsets[i] + t] >= A) return fail(NW_EINVAL, "query %llu has a symbol >= alphabet", (unsigned long long)i);
        qmax = std::max<uint32_t>(qmax, (uint32_t)l);
        rows[i] = {(int)l, {h_q_symbols + h_q_offsets[i], (int32_t)i}};
    }
    const long lo = query_lo(v, qmax);
    if (lo < -32768) return fail(NW_ERANGE, "query scores may fall below int16");
    if (int rc = refuse_capture((hipStream_t)hip_stream, "nw_query")) return rc;
    RowImage img = make_rows(rows);
    // one contiguous host image of the row set -> one copy; the image lives
    // until the copy has completed (freed by a host callback on the stream)
    auto *host = new std::vector<uint8_t>(W.partial, 0);
    std::memcpy(host->data() + W.sym, img.sym.data(), img.sym.size());
    std::memcpy(host->data() + W.pairs, img.pairs.data(), img.pairs.size() * 4);
    std::memcpy(host->data() + W.off, img.off.data(), img.off.size() * 4);
    std::memcpy(host->data() + W.orig, img.orig.data(), img.orig.size() * 4);
    hipStream_t st = (hipStream_t)hip_stream;
    uint8_t *ws = static_cast<uint8_t *>(d_ws);
    hipError_t e = hipMemcpyAsync(ws, host->data(), host->size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        delete host;
        return dev_fail(e, "uploading queries");
    }
    e = hipLaunchHostFunc(st, [](void *p) { delete static_cast<std::vector<uint8_t> *>(p); }, host);
    if (e != hipSuccess) {
        hipStreamSynchronize(st);
        delete host;
        return dev_fail(e, "scheduling the release of the query staging buffer");
    }
    RowSet R;
    R.sym = ws + W.sym;
    R.pairs = reinterpret_cast<const int32_t *>(ws + W.pairs);
    R.off = reinterpret_cast<const uint32_t *>(ws + W.off);
    R.orig = reinterpret_cast<const int32_t *>(ws + W.orig);
    DevVocab Dq = D;
    Dq.lo = (int32_t)lo;
    uint64_t *partial = reinterpret_cast<uint64_t *>(ws + W.partial);
    if ((e = launch_query(Dq, R, img.off.data(), full_colset(D), (int)k, W.nsplit, partial, st)) != hipSuccess ||
        (e = launch_merge(partial, query_lists(W.nsplit), (int)k, (int64_t)n_q, (int)k, (int)lo, d_score, d_index, nullptr, 1, st)) != hipSuccess)
        return dev_fail(e, "launching the query kernels");
    return ok();
}

}  // extern "C"
