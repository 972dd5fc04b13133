// nw_export.cpp -- streamed triangle export (nw_export_triangle).
//
// The triangle of a range of pair indices is produced in chunks.  Chunk c is
// computed into device buffer c mod 2 on the caller's stream, then copied to
// host buffer c mod 2 on a copy stream; while chunk c computes and copies,
// the host hands chunk c-1 to the caller.  The two buffers are the only
// storage, so any triangle fits, whatever the device memory (the paper's
// 600,000-word i8 triangle is 1.8e11 bytes; Section 5 names copying parts to
// the host and restarting the index at 0 as the way past its 107,000-word
// limit).
//
// Reuse rules: the kernel for chunk c waits for the copy of chunk c-2 (same
// device buffer); the copy of chunk c is enqueued only after the callback of
// chunk c-2 (same host buffer) has returned, which the host loop orders.
#include <algorithm>

#include "nw_host.h"

using namespace nw;
using namespace nw::host;

namespace {

// Stream and events owned by one export; drained and released on every exit.
struct ExportRes {
    hipStream_t copy = nullptr;
    hipStream_t compute = nullptr;
    hipEvent_t computed[2] = {nullptr, nullptr};
    hipEvent_t copied[2] = {nullptr, nullptr};
    ~ExportRes()
    {
        if (compute) hipStreamSynchronize(compute);
        if (copy) {
            hipStreamSynchronize(copy);
            hipStreamDestroy(copy);
        }
        for (int i = 0; i < 2; ++i) {
            if (computed[i]) hipEventDestroy(computed[i]);
            if (copied[i]) hipEventDestroy(copied[i]);
        }
    }
};

}  // namespace

int nw_export_triangle(const nw_vocab *v, uint64_t idx_begin, uint64_t idx_end, nw_dtype dt, uint64_t chunk_pairs,
                       void *d_ws, void *h_buf, nw_chunk_fn fn, void *user, void *hip_stream)
{
    int rc = check_triangle_args(v, idx_begin, idx_end, dt, d_ws);
    if (rc) return rc;
    if (idx_end == idx_begin) return ok();
    DeviceScope scope(v->device);
    if (!fn || !h_buf) return fail(NW_EINVAL, "NULL callback or host buffer");
    if (chunk_pairs == 0) return fail(NW_EINVAL, "chunk_pairs must be at least 1");
    if ((uintptr_t)d_ws % 256) return fail(NW_EINVAL, "d_ws must be 256-byte aligned");
    if ((rc = refuse_capture((hipStream_t)hip_stream, "nw_export_triangle"))) return rc;
    const uint64_t es = dt == NW_I8 ? 1 : 2;
    const uint64_t total = idx_end - idx_begin;
    const uint64_t nchunks = (total + chunk_pairs - 1) / chunk_pairs;
    uint8_t *dbuf[2] = {static_cast<uint8_t *>(d_ws), static_cast<uint8_t *>(d_ws) + chunk_pairs * es};
    uint8_t *hbuf[2] = {static_cast<uint8_t *>(h_buf), static_cast<uint8_t *>(h_buf) + chunk_pairs * es};

    ExportRes R;
    R.compute = (hipStream_t)hip_stream;
    hipError_t e = hipStreamCreateWithFlags(&R.copy, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&R.computed[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&R.copied[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) return dev_fail(e, "creating the export stream and events");

    auto chunk_begin = [&](uint64_t c) { return idx_begin + c * chunk_pairs; };
    auto chunk_count = [&](uint64_t c) { return std::min(chunk_pairs, idx_end - chunk_begin(c)); };
    for (uint64_t c = 0; c <= nchunks; ++c) {
        if (c < nchunks) {
            const int s = (int)(c & 1);
            if (c >= 2 && (e = hipStreamWaitEvent(R.compute, R.copied[s], 0)) != hipSuccess)
                return dev_fail(e, "ordering the export");
            if ((e = launch_triangle(v, chunk_begin(c), chunk_begin(c) + chunk_count(c), dt, dbuf[s], R.compute)) !=
                    hipSuccess ||
                (e = hipEventRecord(R.computed[s], R.compute)) != hipSuccess ||
                (e = hipStreamWaitEvent(R.copy, R.computed[s], 0)) != hipSuccess ||
                (e = hipMemcpyAsync(hbuf[s], dbuf[s], chunk_count(c) * es, hipMemcpyDeviceToHost, R.copy)) !=
                    hipSuccess ||
                (e = hipEventRecord(R.copied[s], R.copy)) != hipSuccess)
                return dev_fail(e, "enqueuing an export chunk");
        }
        if (c >= 1) {
            const uint64_t p = c - 1;
            if ((e = hipEventSynchronize(R.copied[p & 1])) != hipSuccess) return dev_fail(e, "copying an export chunk");
            if (fn(user, chunk_begin(p), chunk_count(p), hbuf[p & 1]) != 0)
                return fail(NW_ESTOPPED, "export stopped by the callback after pair index %llu",
                            (unsigned long long)(chunk_begin(p) + chunk_count(p)));
        }
    }
    return ok();
}
