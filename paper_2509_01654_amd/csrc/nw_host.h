// nw_host.h -- host-side pieces shared by the C ABI (nw_api.cpp) and the
// query server (nw_server.cpp): the dictionary descriptor, error reporting,
// query workspace layout and the query row images.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/nw.h"
#include "nw_internal.h"

// Makes `dev` current for the scope and restores the caller's device after.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != dev && hipSetDevice(dev) == hipSuccess) prev = cur;
    }
    ~DeviceScope()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceScope(const DeviceScope &) = delete;
    DeviceScope &operator=(const DeviceScope &) = delete;
};

// Host descriptor of a loaded dictionary (the opaque nw_vocab of nw.h).
struct nw_vocab {
    nw::DevVocab dev;
    std::vector<uint32_t> h_gp_off;   // host copy of dev.gp_off
    std::vector<uint8_t> h_csym;      // host copy of the caller-order padded words
    std::vector<uint8_t> h_clen;
    std::vector<uint32_t> h_rp_off;   // host copy of dev.rp_off
    std::vector<uint32_t> h_maxrp;    // per row length: most row pairs of that length in one block
    uint32_t h_maxdp[nw::kDiagClasses] = {};   // per anti-diagonal class: most row pairs in one block
    int32_t smin = 0, smax = 0;       // similarity extremes
    // phase timing of the last top-k call (HIP events on the caller's stream)
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    float phase_ms[3] = {0, 0, 0};
    uint32_t last_overflow = 0;       // words recomputed exactly by the last top-k call
    bool topk_pending = false;        // a top-k pass was enqueued and not yet finished
    ~nw_vocab()
    {
        for (auto &e : ev)
            if (e) hipEventDestroy(e);
    }
    uint64_t n = 0;
    uint32_t max_len = 0;
    uint64_t num_pairs = 0;
    uint64_t num_cells = 0;
    int32_t lo = 0, hi = 0;      // score bounds
    bool symmetric = true;
    int device = 0;                   // HIP device holding d_mem
    void *d_mem = nullptr;
    uint64_t d_bytes = 0;
};

namespace nw {
namespace host {

// Record a thread-local error message and return `code`.
int fail(int code, const char *fmt, ...);
int ok();
int dev_fail(hipError_t e, const char *what);
uint64_t align_up(uint64_t x, uint64_t a);
// NW_EINVAL (recorded) when `stream` is being captured into a graph: for the
// calls that wait for the device, read results back to the host, copy from
// pageable host memory or run host callbacks, none of which a captured graph
// can replay.  NW_OK otherwise.
int refuse_capture(hipStream_t stream, const char *call);

// Workspace layout of one nw_query call of n_q queries (byte offsets).
struct QueryWs {
    uint64_t sym, pairs, off, orig, partial, total;
    int nsplit;
};
int query_splits(uint64_t n_q);
QueryWs query_ws(uint64_t n_q, uint32_t k);

// Host image of a row set: words sorted by length, paired by equal length.
struct RowImage {
    std::vector<uint8_t> sym;      // [m * kWordBytes]
    std::vector<int32_t> pairs;    // [np * 2]
    std::vector<uint32_t> off;     // [kMaxLen + 2]
    std::vector<int32_t> orig;     // [m]
};
// words: (length, (pointer to symbols, output row))
RowImage make_rows(const std::vector<std::pair<int, std::pair<const uint8_t *, int32_t>>> &words);

// The whole dictionary as a column set.
ColSet full_colset(const DevVocab &D);

// Arguments of the triangle calls (nw_all_pairs_scores and its forms): NW_OK
// or the error already recorded.
int check_triangle_args(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, const void *d_out);
// Enqueue the triangle of pair indices [idx_begin, idx_end) on the kernel the
// dictionary needs (register-row, or anti-diagonal for words past kMaxLen).
hipError_t launch_triangle(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, void *d_out,
                           hipStream_t stream);

// Key origin of a query batch whose longest query has qmax symbols; -1 when
// its scores could leave int16.
long query_lo(const nw_vocab *v, uint32_t qmax);

}  // namespace host
}  // namespace nw
