// nw_noalloc.hip -- nw_query_noalloc: the per-query top-k of nw_query for
// callers that cannot allocate (graph capture, tight serving loops, harnesses
// that forbid allocation).  The query workspace -- the query image and the
// partial lists of the column splits -- lives in a fixed device array of this
// library instead of caller memory, the host image is built on the stack, and
// it reaches the device as kernel arguments, so the call allocates nothing,
// neither on the device nor on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "nw_host.h"

using namespace nw;
using namespace nw::host;

// Fixed scratch: enough for kNoAllocMaxQueries queries at k <= 64 (about
// 2.1 MiB at most; every device the library runs on keeps its own copy until
// the process ends).  Host code never uses the array's name as an address:
// scratch_of() looks up each device's copy.
constexpr uint64_t kScratchBytes = 4ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr uint32_t kNoAllocMaxQueries = 256;
// Host image of at most kNoAllocMaxQueries rows (words, pairs, offsets, rows).
constexpr uint64_t kImageBytes = 20u << 10;
// Bytes carried by one upload launch (kernel arguments are at most 4 KiB).
constexpr uint32_t kChunkBytes = 3072;

struct UploadChunk {
    uint32_t off, n;
    uint8_t bytes[kChunkBytes];
};

// dst[c.off .. c.off + c.n) = c.bytes[0 .. c.n)
__global__ __launch_bounds__(256) void k_upload(uint8_t *dst, UploadChunk c)
{
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[c.off + i] = c.bytes[i];
}

// The device address of `scratch` on device `dev`, looked up once per device
// (with that device current) and kept.
hipError_t scratch_of(int dev, uint8_t **out)
{
    static std::mutex mu;
    static uint8_t *ptr[64] = {};
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<uint8_t *>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int nw_query_noalloc(const nw_vocab *v, const uint8_t *h_q_symbols, const uint64_t *h_q_offsets,
                                uint64_t n_q, uint32_t k, int16_t *d_score, int32_t *d_index, void *hip_stream)
{
    if (!v) return fail(NW_EINVAL, "vocab is NULL");
    if (k < 1 || k > 64) return fail(NW_EINVAL, "k = %u outside 1..64", k);
    if (n_q == 0) return ok();
    if (n_q > kNoAllocMaxQueries)
        return fail(NW_EINVAL, "nw_query_noalloc takes at most %u queries per call (got %llu)", kNoAllocMaxQueries,
                    (unsigned long long)n_q);
    if (!h_q_offsets || !d_score || !d_index) return fail(NW_EINVAL, "NULL argument");
    if (v->max_len > (uint32_t)kMaxLen)
        return fail(NW_EINVAL, "queries support dictionaries of words of at most %d symbols", kMaxLen);
    if (h_q_offsets[0] != 0) return fail(NW_EINVAL, "query offsets[0] must be 0");
    const int A = v->dev.alphabet;
    uint32_t len[kNoAllocMaxQueries];
    uint32_t qmax = 0;
    for (uint64_t i = 0; i < n_q; ++i) {
        if (h_q_offsets[i + 1] < h_q_offsets[i])
            return fail(NW_EINVAL, "query offsets decrease at %llu", (unsigned long long)i);
        const uint64_t l = h_q_offsets[i + 1] - h_q_offsets[i];
        if (l > (uint64_t)kMaxLen)
            return fail(NW_EINVAL, "query %llu has %llu symbols; the maximum is %d", (unsigned long long)i,
                        (unsigned long long)l, kMaxLen);
        if (l && !h_q_symbols) return fail(NW_EINVAL, "query symbols are NULL");
        for (uint64_t t = 0; t < l; ++t)
            if (h_q_symbols[h_q_offsets[i] + t] >= A)
                return fail(NW_EINVAL, "query %llu has a symbol >= alphabet", (unsigned long long)i);
        len[i] = (uint32_t)l;
        qmax = std::max(qmax, (uint32_t)l);
    }
    const long lo = query_lo(v, qmax);
    if (lo < -32768) return fail(NW_ERANGE, "query scores may fall below int16");
    const QueryWs W = query_ws(n_q, k);
    if (W.total > kScratchBytes || W.partial > kImageBytes)
        return fail(NW_ENOMEM, "%llu queries at k = %u need %llu scratch bytes; the fixed scratch holds %llu",
                    (unsigned long long)n_q, k, (unsigned long long)W.total, (unsigned long long)kScratchBytes);

    // The row image on the stack: queries sorted by length (stable), paired
    // by equal length, as the query kernels read it.
    alignas(16) uint8_t img[kImageBytes];
    std::memset(img, 0, W.partial);
    uint8_t *sym = img + W.sym;
    int32_t *pairs = reinterpret_cast<int32_t *>(img + W.pairs);
    uint32_t *off = reinterpret_cast<uint32_t *>(img + W.off);
    int32_t *orig = reinterpret_cast<int32_t *>(img + W.orig);
    uint32_t np = 0, slot = 0;
    for (int l = 0; l <= kMaxLen; ++l) {
        off[l] = np;
        const uint32_t first = slot;
        for (uint64_t i = 0; i < n_q; ++i) {
            if ((int)len[i] != l) continue;
            if (l) std::memcpy(sym + (uint64_t)slot * kWordBytes, h_q_symbols + h_q_offsets[i], (size_t)l);
            orig[slot++] = (int32_t)i;
        }
        for (uint32_t t = first; t < slot; t += 2) {
            pairs[2 * np] = (int32_t)t;
            pairs[2 * np + 1] = t + 1 < slot ? (int32_t)(t + 1) : -1;
            ++np;
        }
    }
    off[kMaxLen + 1] = np;

    DeviceScope scope(v->device);
    hipStream_t st = (hipStream_t)hip_stream;
    uint8_t *ws = nullptr;
    hipError_t e = scratch_of(v->device, &ws);
    if (e != hipSuccess) return dev_fail(e, "looking up the query scratch");
    // the image goes up as kernel arguments: nothing on the host has to
    // outlive the call
    for (uint32_t o = 0; o < W.partial; o += kChunkBytes) {
        UploadChunk c;
        c.off = o;
        c.n = (uint32_t)std::min<uint64_t>(kChunkBytes, W.partial - o);
        std::memcpy(c.bytes, img + o, c.n);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, st, ws, c);
        if ((e = hipGetLastError()) != hipSuccess) return dev_fail(e, "uploading queries");
    }
    RowSet R;
    R.sym = ws + W.sym;
    R.pairs = reinterpret_cast<const int32_t *>(ws + W.pairs);
    R.off = reinterpret_cast<const uint32_t *>(ws + W.off);
    R.orig = reinterpret_cast<const int32_t *>(ws + W.orig);
    DevVocab Dq = v->dev;
    Dq.lo = (int32_t)lo;
    uint64_t *partial = reinterpret_cast<uint64_t *>(ws + W.partial);
    if ((e = launch_query(Dq, R, off, full_colset(v->dev), (int)k, W.nsplit, partial, st)) != hipSuccess ||
        (e = launch_merge(partial, query_lists(W.nsplit), (int)k, (int64_t)n_q, (int)k, (int)lo, d_score, d_index,
                          nullptr, 1, st)) != hipSuccess)
        return dev_fail(e, "launching the query kernels");
    return ok();
}
