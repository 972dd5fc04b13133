// nw_server.cpp -- continuous-batching query server over a device-resident
// dictionary (the online similar-word lookup the paper envisions, Section 6).
//
// A scheduler thread owns `num_slots` slots.  Each slot has its own HIP stream
// (default priority), an event and pinned host buffers for the query image and
// the results.  The caller's device workspace is a pool: every batch reserves
// the bytes its own queries need (the query workspace of q queries plus their
// q*k results) and returns them when it completes.  Requests wait in a FIFO
// queue; whenever a slot is free the oldest requests (up to max_batch) are
// admitted as one batch -- as many of them as the largest free range of the
// pool holds; when not even one fits, admission waits for a running batch to
// return its memory (back-pressure).  A batch runs image -> H2D copy -> query
// kernels (one launch per query length present) -> merge -> D2H copy -> event.
// Batches on different slots overlap on the device, and requests that arrive
// while others run are admitted as soon as a slot and memory free up
// (continuous batching).  Each query's result depends only on the query and
// the dictionary, never on the batch it ran in or the memory it was given.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include "nw_host.h"

using namespace nw;
using namespace nw::host;

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t tag;
    int64_t t_arrival;
    std::vector<uint8_t> sym;
};

struct Completed {
    uint64_t tag;
    int64_t t_arrival, t_done;
    std::vector<int16_t> s;
    std::vector<int32_t> i;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    uint64_t mem_off = 0, mem_bytes = 0;   // the batch's range of the workspace pool
    uint8_t *h_in = nullptr;     // pinned query image
    int16_t *h_s = nullptr;      // pinned results
    int32_t *h_i = nullptr;
    std::vector<Request> batch;
    bool busy = false;
};

// Device bytes one batch of q queries reserves from the pool: its query
// workspace, then its int16 scores and int32 indices.
uint64_t batch_bytes(uint32_t q, uint32_t k)
{
    return align_up(query_ws(q, k).total, 256) + align_up((uint64_t)q * k * 2, 256) + align_up((uint64_t)q * k * 4, 256);
}

// Largest batch_bytes and host image over batches of 1..max_batch queries
// (small batches use many column splits, so the maximum is not always at
// max_batch).
struct SlotSizes {
    uint64_t dev_batch, host_image;
};

SlotSizes slot_sizes(uint32_t k, uint32_t max_batch)
{
    SlotSizes z{0, 0};
    for (uint32_t q = 1; q <= max_batch; ++q) {
        z.dev_batch = std::max(z.dev_batch, batch_bytes(q, k));
        z.host_image = std::max(z.host_image, query_ws(q, k).partial);
    }
    return z;
}

// First-fit ranges of the workspace pool (scheduler thread only).  Ranges are
// multiples of 256 bytes; a released range merges with its free neighbours.
class Pool {
  public:
    void reset(uint64_t bytes)
    {
        size_ = bytes / 256 * 256;
        free_.assign(1, {0, size_});
        used_ = peak_ = 0;
    }
    uint64_t largest() const
    {
        uint64_t m = 0;
        for (const auto &r : free_) m = std::max(m, r.second);
        return m;
    }
    bool take(uint64_t bytes, uint64_t &off)
    {
        for (size_t i = 0; i < free_.size(); ++i) {
            if (free_[i].second < bytes) continue;
            off = free_[i].first;
            free_[i].first += bytes;
            free_[i].second -= bytes;
            if (free_[i].second == 0) free_.erase(free_.begin() + (long)i);
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void give(uint64_t off, uint64_t bytes)
    {
        if (!bytes) return;
        used_ -= bytes;
        size_t i = 0;
        while (i < free_.size() && free_[i].first < off) ++i;
        free_.insert(free_.begin() + (long)i, {off, bytes});
        if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
            free_[i].second += free_[i + 1].second;
            free_.erase(free_.begin() + (long)i + 1);
        }
        if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
            free_[i - 1].second += free_[i].second;
            free_.erase(free_.begin() + (long)i);
        }
    }
    uint64_t size() const { return size_; }
    uint64_t peak() const { return peak_; }

  private:
    std::vector<std::pair<uint64_t, uint64_t>> free_;   // (offset, bytes), sorted by offset
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
};

}  // namespace

struct nw_server {
    const nw_vocab *v = nullptr;
    uint32_t k = 0, max_batch = 0;
    int device = 0;
    SlotSizes sz{};
    std::vector<Slot> slots;
    uint8_t *d_pool = nullptr;
    Pool pool;                          // scheduler thread only
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::deque<Completed> done;
    std::thread th;
    std::atomic<bool> stop{false};
    std::atomic<int> err{0};
    std::atomic<bool> inject{false};    // host-side failure of the next admitted batch (tests)
    std::string err_msg;                // written once, under mu, before err is set
    uint64_t batches = 0, queries = 0;
    uint64_t mem_waits = 0;             // admitted batches that waited or shrank for memory
    bool mem_short = false;             // the next admission has found the pool short
    uint64_t peak_bytes = 0;

    void set_error(const std::string &msg)
    {
        std::lock_guard<std::mutex> g(mu);
        if (!err) {
            err_msg = msg;
            err = NW_EDEVICE;
        }
        cv_done.notify_all();
    }
    void set_error(hipError_t e, const char *what) { set_error(std::string(what) + ": " + hipGetErrorString(e)); }

    // Enqueue one batch on slot s (scheduler thread); its memory is reserved.
    bool launch(Slot &s)
    {
        if (inject.exchange(false)) return set_error("server launch: injected host-side failure"), false;
        const uint32_t q = (uint32_t)s.batch.size();
        std::vector<std::pair<int, std::pair<const uint8_t *, int32_t>>> rows(q);
        uint32_t qmax = 0;
        for (uint32_t t = 0; t < q; ++t) {
            rows[t] = {(int)s.batch[t].sym.size(), {s.batch[t].sym.data(), (int32_t)t}};
            qmax = std::max<uint32_t>(qmax, (uint32_t)s.batch[t].sym.size());
        }
        const RowImage img = make_rows(rows);
        const QueryWs W = query_ws(q, k);
        std::memset(s.h_in, 0, W.partial);
        std::memcpy(s.h_in + W.sym, img.sym.data(), img.sym.size());
        std::memcpy(s.h_in + W.pairs, img.pairs.data(), img.pairs.size() * 4);
        std::memcpy(s.h_in + W.off, img.off.data(), img.off.size() * 4);
        std::memcpy(s.h_in + W.orig, img.orig.data(), img.orig.size() * 4);
        uint8_t *d_ws = d_pool + s.mem_off;
        int16_t *d_s = reinterpret_cast<int16_t *>(d_ws + align_up(W.total, 256));
        int32_t *d_i = reinterpret_cast<int32_t *>(d_ws + align_up(W.total, 256) + align_up((uint64_t)q * k * 2, 256));
        hipError_t e = hipMemcpyAsync(d_ws, s.h_in, W.partial, hipMemcpyHostToDevice, s.st);
        if (e != hipSuccess) return set_error(e, "server upload"), false;
        RowSet R;
        R.sym = d_ws + W.sym;
        R.pairs = reinterpret_cast<const int32_t *>(d_ws + W.pairs);
        R.off = reinterpret_cast<const uint32_t *>(d_ws + W.off);
        R.orig = reinterpret_cast<const int32_t *>(d_ws + W.orig);
        DevVocab Dq = v->dev;
        const long lo = query_lo(v, qmax);
        Dq.lo = (int32_t)lo;
        uint64_t *partial = reinterpret_cast<uint64_t *>(d_ws + W.partial);
        if ((e = launch_query(Dq, R, img.off.data(), full_colset(v->dev), (int)k, W.nsplit, partial, s.st)) != hipSuccess ||
            (e = launch_merge(partial, query_lists(W.nsplit), (int)k, q, (int)k, (int)lo, d_s, d_i, nullptr, 1, s.st)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(s.h_s, d_s, (size_t)q * k * 2, hipMemcpyDeviceToHost, s.st)) != hipSuccess ||
            (e = hipMemcpyAsync(s.h_i, d_i, (size_t)q * k * 4, hipMemcpyDeviceToHost, s.st)) != hipSuccess ||
            (e = hipEventRecord(s.ev, s.st)) != hipSuccess)
            return set_error(e, "server launch"), false;
        s.busy = true;
        return true;
    }

    // Return slot s's memory to the pool (scheduler thread).  A slot whose
    // launch failed part-way may still have work in flight on its stream, so
    // its memory is only returned once the stream is idle.
    void release(Slot &s)
    {
        pool.give(s.mem_off, s.mem_bytes);
        s.mem_off = s.mem_bytes = 0;
    }

    // Admit the oldest requests into free slot s: as many (up to max_batch)
    // as the largest free range of the pool holds.  False when none is
    // waiting or not even one query fits (it then waits for memory).
    bool admit(Slot &s)
    {
        std::lock_guard<std::mutex> g(mu);
        if (pending.empty()) return false;
        uint32_t q = (uint32_t)std::min<size_t>(pending.size(), max_batch);
        const uint64_t room = pool.largest();
        const uint32_t want = q;
        while (q > 0 && batch_bytes(q, k) > room) --q;
        if (q < want) mem_short = true;
        if (q == 0) return false;
        const uint64_t bytes = batch_bytes(q, k);
        if (!pool.take(bytes, s.mem_off)) return false;
        s.mem_bytes = bytes;
        peak_bytes = pool.peak();
        if (mem_short) ++mem_waits;   // this batch waited or shrank for memory
        mem_short = false;
        for (uint32_t t = 0; t < q; ++t) {
            s.batch.push_back(std::move(pending.front()));
            pending.pop_front();
        }
        return true;
    }

    void deliver(Slot &s)
    {
        const int64_t t = now_ns();
        std::lock_guard<std::mutex> g(mu);
        for (size_t b = 0; b < s.batch.size(); ++b) {
            Completed c;
            c.tag = s.batch[b].tag;
            c.t_arrival = s.batch[b].t_arrival;
            c.t_done = t;
            c.s.assign(s.h_s + b * k, s.h_s + (b + 1) * k);
            c.i.assign(s.h_i + b * k, s.h_i + (b + 1) * k);
            done.push_back(std::move(c));
        }
        queries += s.batch.size();
        batches += 1;
        s.batch.clear();
        s.busy = false;
        cv_done.notify_all();
    }

    // After an error nothing more is admitted: the waiting requests are
    // dropped (poll and submit report the error), the batches in flight
    // drain, and the loop ends once stop is set -- whatever was queued.
    void run()
    {
        hipSetDevice(device);
        for (;;) {
            bool progress = false, any_busy = false;
            for (auto &s : slots) {
                if (!s.busy) continue;
                const hipError_t e = hipEventQuery(s.ev);
                if (e == hipSuccess) {
                    deliver(s);
                    release(s);
                    progress = true;
                } else if (e != hipErrorNotReady) {
                    set_error(e, "server completion");
                    hipStreamSynchronize(s.st);
                    s.batch.clear();
                    s.busy = false;
                    release(s);
                } else {
                    any_busy = true;
                }
            }
            for (auto &s : slots) {
                if (s.busy || err) continue;
                if (!admit(s)) break;
                if (launch(s)) {
                    progress = true;
                    any_busy = true;
                } else {
                    // nothing of a failed launch is left waiting: drain its stream first
                    hipStreamSynchronize(s.st);
                    s.batch.clear();
                    release(s);
                }
            }
            if (progress) continue;
            std::unique_lock<std::mutex> g(mu);
            if (err) pending.clear();
            if (stop && pending.empty() && !any_busy) break;
            if (any_busy) {
                g.unlock();
                std::this_thread::yield();   // completion polling while batches run
            } else {
                cv_work.wait_for(g, std::chrono::milliseconds(5),
                                 [&] { return stop.load() || (!pending.empty() && !err); });
            }
        }
    }
};

extern "C" {

int nw_server_workspace_bytes(const nw_vocab *v, uint32_t k, uint32_t max_batch, uint32_t num_slots, uint64_t *bytes)
{
    if (!v || !bytes) return fail(NW_EINVAL, "NULL argument");
    if (k < 1 || k > 64 || max_batch < 1 || max_batch > 4096 || num_slots < 1 || num_slots > 16)
        return fail(NW_EINVAL, "k in 1..64, max_batch in 1..4096, num_slots in 1..16");
    *bytes = (uint64_t)num_slots * slot_sizes(k, max_batch).dev_batch;
    return ok();
}

int nw_server_min_workspace_bytes(const nw_vocab *v, uint32_t k, uint64_t *bytes)
{
    if (!v || !bytes) return fail(NW_EINVAL, "NULL argument");
    if (k < 1 || k > 64) return fail(NW_EINVAL, "k in 1..64");
    *bytes = batch_bytes(1, k);
    return ok();
}

int nw_server_create(const nw_vocab *v, uint32_t k, uint32_t max_batch, uint32_t num_slots, void *d_ws,
                     uint64_t ws_bytes, nw_server **out)
{
    if (!out) return fail(NW_EINVAL, "out is NULL");
    *out = nullptr;
    uint64_t need = 0, least = 0;
    int rc = nw_server_workspace_bytes(v, k, max_batch, num_slots, &need);
    if (rc) return rc;
    if ((rc = nw_server_min_workspace_bytes(v, k, &least))) return rc;
    if (v->max_len > (uint32_t)kMaxLen) return fail(NW_EINVAL, "the server supports words of at most %d symbols", kMaxLen);
    if (!d_ws || (uintptr_t)d_ws % 256) return fail(NW_EINVAL, "d_ws must be a 256-byte aligned device pointer");
    if (ws_bytes < least)
        return fail(NW_ENOMEM, "workspace holds %llu bytes; the server needs at least %llu (one query)",
                    (unsigned long long)ws_bytes, (unsigned long long)least);
    nw_server *S = new nw_server();
    S->v = v;
    S->k = k;
    S->max_batch = max_batch;
    S->device = v->device;
    S->sz = slot_sizes(k, max_batch);
    S->slots.resize(num_slots);
    S->d_pool = static_cast<uint8_t *>(d_ws);
    S->pool.reset(std::min(ws_bytes, need));
    hipError_t e = hipSetDevice(S->device);
    for (uint32_t t = 0; t < num_slots && e == hipSuccess; ++t) {
        Slot &s = S->slots[t];
        if ((e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming)) != hipSuccess) break;
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&s.h_in), std::max<uint64_t>(S->sz.host_image, 256), 0)) != hipSuccess) break;
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&s.h_s), (size_t)max_batch * k * 2, 0)) != hipSuccess) break;
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&s.h_i), (size_t)max_batch * k * 4, 0)) != hipSuccess) break;
    }
    if (e != hipSuccess) {
        nw_server_destroy(S);
        return dev_fail(e, "creating the server");
    }
    S->th = std::thread([S] { S->run(); });
    *out = S;
    return ok();
}

int64_t nw_clock_ns(void) { return now_ns(); }

// The server's error (NW_OK if none), recorded as the thread's last error.
static int server_error(nw_server *S)
{
    if (!S->err) return NW_OK;
    std::lock_guard<std::mutex> g(S->mu);
    return fail(S->err, "%s", S->err_msg.c_str());
}

int nw_server_submit(nw_server *S, const uint8_t *h_symbols, uint32_t len, uint64_t tag, int64_t t_arrival_ns)
{
    if (!S) return fail(NW_EINVAL, "server is NULL");
    if (int rc = server_error(S)) return rc;
    if (len > (uint32_t)kMaxLen) return fail(NW_EINVAL, "query of %u symbols; the maximum is %d", len, kMaxLen);
    if (len && !h_symbols) return fail(NW_EINVAL, "symbols is NULL");
    for (uint32_t t = 0; t < len; ++t)
        if (h_symbols[t] >= S->v->dev.alphabet) return fail(NW_EINVAL, "query symbol >= alphabet");
    if (query_lo(S->v, len) < -32768) return fail(NW_ERANGE, "query scores may fall below int16");
    Request r;
    r.tag = tag;
    r.t_arrival = t_arrival_ns ? t_arrival_ns : now_ns();
    r.sym.assign(h_symbols, h_symbols + len);
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->pending.push_back(std::move(r));
    }
    S->cv_work.notify_one();
    return ok();
}

int nw_server_poll(nw_server *S, uint32_t max_results, int32_t timeout_us, uint64_t *tags, int16_t *scores,
                   int32_t *indices, int64_t *latency_ns, uint32_t *n_out)
{
    if (!S || !n_out) return fail(NW_EINVAL, "NULL argument");
    *n_out = 0;
    std::unique_lock<std::mutex> g(S->mu);
    if (S->done.empty() && timeout_us > 0)
        S->cv_done.wait_for(g, std::chrono::microseconds(timeout_us), [&] { return !S->done.empty() || S->err; });
    if (S->err) return fail(S->err, "%s", S->err_msg.c_str());   // mu is held here
    uint32_t n = 0;
    while (n < max_results && !S->done.empty()) {
        Completed &c = S->done.front();
        if (tags) tags[n] = c.tag;
        if (scores) std::memcpy(scores + (size_t)n * S->k, c.s.data(), S->k * 2);
        if (indices) std::memcpy(indices + (size_t)n * S->k, c.i.data(), S->k * 4);
        if (latency_ns) latency_ns[n] = c.t_done - c.t_arrival;
        S->done.pop_front();
        ++n;
    }
    *n_out = n;
    return ok();
}

int nw_server_replay(nw_server *S, const uint8_t *h_symbols, const uint64_t *h_offsets, uint64_t n_q,
                     const double *arrival_s, int16_t *scores, int32_t *indices, double *latency_s)
{
    if (!S || !h_offsets || !arrival_s || !scores || !indices) return fail(NW_EINVAL, "NULL argument");
    for (uint64_t i = 0; i < n_q; ++i) {
        const uint64_t l = h_offsets[i + 1] - h_offsets[i];
        if (h_offsets[i + 1] < h_offsets[i] || l > (uint64_t)kMaxLen) return fail(NW_EINVAL, "bad query %llu", (unsigned long long)i);
        for (uint64_t t = 0; t < l; ++t)
            if (h_symbols[h_offsets[i] + t] >= S->v->dev.alphabet) return fail(NW_EINVAL, "query symbol >= alphabet");
    }
    const int64_t t0 = now_ns() + 2000000;   // start 2 ms from now
    std::atomic<int> sub_rc{NW_OK};
    std::thread submitter([&] {
        for (uint64_t i = 0; i < n_q; ++i) {
            const int64_t due = t0 + (int64_t)(arrival_s[i] * 1e9);
            int64_t now = now_ns();
            if (due - now > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(due - now - 150000));
            while (now_ns() < due) {
            }
            const int rc = nw_server_submit(S, h_symbols + h_offsets[i], (uint32_t)(h_offsets[i + 1] - h_offsets[i]), i, due);
            if (rc) {
                sub_rc = rc;
                return;
            }
        }
    });
    uint64_t got = 0;
    const uint32_t chunk = 256;
    std::vector<uint64_t> tags(chunk);
    std::vector<int16_t> s(chunk * S->k);
    std::vector<int32_t> ix(chunk * S->k);
    std::vector<int64_t> lat(chunk);
    int rc = NW_OK;
    while (got < n_q) {
        uint32_t n = 0;
        rc = nw_server_poll(S, chunk, 1000, tags.data(), s.data(), ix.data(), lat.data(), &n);
        if (rc) break;
        if (sub_rc != NW_OK) {
            rc = sub_rc;
            break;
        }
        for (uint32_t t = 0; t < n; ++t) {
            const uint64_t q = tags[t];
            std::memcpy(scores + q * S->k, &s[(size_t)t * S->k], S->k * 2);
            std::memcpy(indices + q * S->k, &ix[(size_t)t * S->k], S->k * 4);
            if (latency_s) latency_s[q] = lat[t] * 1e-9;
        }
        got += n;
    }
    submitter.join();
    return rc;
}

int nw_server_stats(nw_server *S, uint64_t *batches, uint64_t *queries)
{
    if (!S) return fail(NW_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    if (batches) *batches = S->batches;
    if (queries) *queries = S->queries;
    return ok();
}

int nw_server_memory_stats(nw_server *S, uint64_t *pool_bytes, uint64_t *peak_bytes, uint64_t *waits)
{
    if (!S) return fail(NW_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    if (pool_bytes) *pool_bytes = S->pool.size();
    if (peak_bytes) *peak_bytes = S->peak_bytes;
    if (waits) *waits = S->mem_waits;
    return ok();
}

int nw_server_inject_failure(nw_server *S)
{
    if (!S) return fail(NW_EINVAL, "server is NULL");
    S->inject = true;
    return ok();
}

void nw_server_destroy(nw_server *S)
{
    if (!S) return;
    if (S->th.joinable()) {
        S->stop = true;
        S->cv_work.notify_all();
        S->th.join();
    }
    for (auto &s : S->slots) {
        if (s.st) hipStreamSynchronize(s.st);
        if (s.ev) hipEventDestroy(s.ev);
        if (s.st) hipStreamDestroy(s.st);
        if (s.h_in) hipHostFree(s.h_in);
        if (s.h_s) hipHostFree(s.h_s);
        if (s.h_i) hipHostFree(s.h_i);
    }
    delete S;
}

}  // extern "C"
