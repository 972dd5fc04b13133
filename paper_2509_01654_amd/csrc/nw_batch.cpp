// nw_batch.cpp -- many dictionaries' triangles in one graph-captured sequence
// of persistent launches, and the autotuner that picks its parameters.
//
// Plan: every dictionary's triangle is cut into work items (block pair, row
// length LA, a chunk of at most `pairs_per_item` row pairs).  Each item's cost
// is estimated as (row pairs) * 2 * LA * (symbols of the column block); items
// are grouped into row-length classes (one per length, or classes of 8
// lengths) and ordered heaviest first, so the persistent workgroups finish
// together.  The batch object captures [counter reset, one persistent kernel
// per non-empty class] into a hipGraph once; each run replays it.
//
// Class width 0 is the other form: every dictionary's launches (as
// nw_all_pairs_scores issues them), spread over one fork of concurrent chains
// (library streams when eager, chains of kernel nodes inside the capture).
//
// Autotuner: times candidate (class width, workgroups per CU, pairs per item)
// settings on the batch itself and caches the best per device and workload
// signature in a JSON-lines file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "k_batch.h"
#include "nw_fork.h"
#include "nw_host.h"
#include "nw_kernels.h"

using namespace nw;
using namespace nw::host;

namespace {

struct Plan {
    std::vector<BatchItem> items;               // grouped by class, heaviest first
    std::vector<uint32_t> class_off;            // [nclass + 1]
    std::vector<uint32_t> class_lds;            // dynamic LDS per class
    int code_es = 0;                            // score-code tiles storing es bytes, or 0: plain tiles
    int width = 8;
    uint64_t ws_bytes = 0;
    uint64_t off_vocabs = 0, off_outs = 0, off_counters = 0, off_items = 0;
};

int num_classes(int width) { return width == 0 ? 0 : width == 1 ? kMaxLen + 1 : kNumClass8; }
int class_of(int la, int width) { return width == 1 ? la : la / 8; }

Plan make_plan(const nw_vocab *const *v, uint32_t nv, const nw_batch_options &o, int es)
{
    Plan P;
    P.width = o.class_width == 0 ? 0 : o.class_width == 1 ? 1 : 8;
    const int nc = num_classes(P.width);
    if (P.width == 0) {   // tiled launches: no items, no counters
        P.class_off.assign(1, 0);
        P.ws_bytes = 256;
        return P;
    }
    std::vector<std::vector<std::pair<double, BatchItem>>> cls(nc);
    P.class_lds.assign(nc, 0);
    // the score-code tiles when every dictionary's scores fit their window
    // and every class's buffers fit
    P.code_es = es;
    for (uint32_t vi = 0; vi < nv; ++vi)
        for (int la = 0; la <= v[vi]->dev.lmax; ++la)
            if (!tri_code_applies(v[vi]->dev, la, es, 1)) P.code_es = 0;
    for (uint32_t vi = 0; vi < nv; ++vi) {
        const nw_vocab &V = *v[vi];
        const DevVocab &D = V.dev;
        const int LM = D.lmax;
        // symbols per column block
        std::vector<double> bcells(D.nb, 0.0);
        for (uint64_t u = 0; u < V.n; ++u) bcells[u / D.CB] += V.h_clen[u];
        for (int la = 0; la <= LM; ++la) {
            const int c = class_of(la, P.width);
            P.class_lds[c] = std::max<uint32_t>(P.class_lds[c], P.code_es ? tri_code_lds_bytes(la, D.alphabet, D.CB, es, 1)
                                                                            : tri_lds_bytes(la, D.alphabet, D.CB));
        }
        for (uint32_t b = 0; b < (uint32_t)D.nb; ++b)
            for (uint32_t r = 0; r <= b; ++r)
                for (int la = 0; la <= LM; ++la) {
                    const uint32_t a0 = V.h_rp_off[(size_t)r * (LM + 1) + la];
                    const uint32_t a1 = V.h_rp_off[(size_t)r * (LM + 1) + la + 1];
                    const uint32_t step = o.pairs_per_item ? o.pairs_per_item : (a1 - a0);
                    for (uint32_t p = a0; p < a1; p += step) {
                        BatchItem I;
                        I.vocab = (uint16_t)vi;
                        I.la = (uint16_t)la;
                        I.r = r;
                        I.b = b;
                        I.pbeg = p;
                        I.pend = std::min(a1, p + step);
                        const double cost = (double)(I.pend - I.pbeg) * (2.0 * std::max(la, 1) * bcells[b] + 64.0);
                        cls[class_of(la, P.width)].push_back({cost, I});
                    }
                }
    }
    P.class_off.assign(nc + 1, 0);
    for (int c = 0; c < nc; ++c) {
        std::stable_sort(cls[c].begin(), cls[c].end(),
                         [](const std::pair<double, BatchItem> &a, const std::pair<double, BatchItem> &b) {
                             return a.first > b.first;
                         });
        P.class_off[c] = (uint32_t)P.items.size();
        for (auto &e : cls[c]) P.items.push_back(e.second);
    }
    P.class_off[nc] = (uint32_t)P.items.size();
    uint64_t o2 = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o2;
        o2 = align_up(o2 + (bytes ? bytes : 1), 256);
        return at;
    };
    P.off_vocabs = take(sizeof(DevVocab) * nv);
    P.off_outs = take(8ull * nv);
    P.off_counters = take(4ull * nc);
    P.off_items = take(sizeof(BatchItem) * P.items.size());
    P.ws_bytes = o2;
    return P;
}

std::string device_name(int dev)
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    return std::string(p.name) + "/" + p.gcnArchName;
}

}  // namespace

struct nw_batch {
    std::vector<const nw_vocab *> v;
    std::vector<void *> outs;   // host copies of d_outs
    nw_batch_options opt{};
    Plan plan;
    int out_kind = OUT_I16;
    uint8_t *ws = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int cus = 0;

    // Enqueue the reset and the class kernels on stream s.  The class
    // kernels are independent (own counters, own items), so they are spread
    // over library streams forked from s and joined back into it: in a
    // captured graph they become parallel branches, and one class's tail
    // overlaps the next class's start.
    hipError_t enqueue(hipStream_t s)
    {
        if (plan.width == 0) {
            StreamFork fork(s);
            hipError_t e = fork.begin();
            if (e != hipSuccess) return e;
            for (size_t i = 0; i < v.size(); ++i)
                if ((e = launch_triangle_tiled(v[i]->dev, v[i]->h_maxrp.data(), 0, v[i]->num_pairs, out_kind, outs[i],
                                               s, nullptr, &fork)) != hipSuccess)
                    return e;
            return fork.end();
        }
        const KernelTables &T = kernel_tables();
        const int nc = num_classes(plan.width);
        uint32_t *counters = reinterpret_cast<uint32_t *>(ws + plan.off_counters);
        hipError_t e = launch_reset_counters(counters, nc, s);
        if (e != hipSuccess) return e;
        StreamFork fork(s);
        if ((e = fork.begin()) != hipSuccess) return e;
        const DevVocab *vocabs = reinterpret_cast<const DevVocab *>(ws + plan.off_vocabs);
        const BatchItem *items = reinterpret_cast<const BatchItem *>(ws + plan.off_items);
        void *const *outs = reinterpret_cast<void *const *>(ws + plan.off_outs);
        for (int c = 0; c < nc; ++c) {
            const uint32_t n = plan.class_off[c + 1] - plan.class_off[c];
            if (!n) continue;
            const void *fn = plan.width == 1 ? T.persist1[c] : T.persist8[c];
            const uint32_t grid = std::min<uint32_t>(n, (uint32_t)cus * std::max<uint32_t>(1, opt.wg_per_cu));
            const size_t lds = plan.class_lds[c];
            if (lds > 65536 && (e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
                return e;
            const BatchItem *it = items + plan.class_off[c];
            uint32_t *ctr = counters + c;
            int kind = out_kind;
            int code_es = plan.code_es;
            uint32_t nn = n;
            void *args[] = {&vocabs, &it, &nn, &ctr, &outs, &kind, &code_es};
            if ((e = fork.launch(fn, dim3(grid), dim3(kThreads), lds, args)) != hipSuccess) return e;
        }
        return fork.end();
    }
};

extern "C" {

int nw_all_pairs_scores_batched(const nw_vocab *const *v, uint32_t nv, void *const *d_outs, nw_dtype dt,
                                void *hip_stream)
{
    if (!v || !d_outs) return fail(NW_EINVAL, "NULL argument");
    if (nv == 0) return ok();
    for (uint32_t i = 0; i < nv; ++i) {
        int rc = check_triangle_args(v[i], 0, v[i] ? v[i]->num_pairs : 0, dt, d_outs[i]);
        if (rc) return fail(rc, "dictionary %u: %s", i, nw_last_error());
        if (v[i]->device != v[0]->device) return fail(NW_EINVAL, "dictionary %u is on another device", i);
    }
    DeviceScope scope(v[0]->device);
    hipStream_t st = (hipStream_t)hip_stream;
    const int kind = dt == NW_I8 ? OUT_I8 : OUT_I16;
    // dictionaries with words past the register-row limit first, each on the
    // anti-diagonal kernel's own fork; then the register-row launches of all
    // others share one fork, so one dictionary's tail overlaps the next one's
    // start (forks follow each other, never interleave)
    hipError_t e = hipSuccess;
    for (uint32_t i = 0; i < nv && e == hipSuccess; ++i)
        if (v[i]->max_len > (uint32_t)kMaxLen)
            e = launch_triangle_diag(v[i]->dev, v[i]->h_maxrp.data(), v[i]->h_maxdp, 0, v[i]->num_pairs, kind,
                                     d_outs[i], st);
    if (e != hipSuccess) return dev_fail(e, "launching the batched triangles");
    StreamFork fork(st);
    e = fork.begin();
    for (uint32_t i = 0; i < nv && e == hipSuccess; ++i)
        if (v[i]->max_len <= (uint32_t)kMaxLen)
            e = launch_triangle_tiled(v[i]->dev, v[i]->h_maxrp.data(), 0, v[i]->num_pairs, kind, d_outs[i], st,
                                      nullptr, &fork);
    const hipError_t e2 = fork.end();
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return dev_fail(e, "launching the batched triangles");
    return ok();
}

int nw_batch_workspace_bytes(const nw_vocab *const *v, uint32_t nv, const nw_batch_options *opt, uint64_t *bytes)
{
    if (!v || !nv || !opt || !bytes) return fail(NW_EINVAL, "NULL argument");
    if (nv > 65535) return fail(NW_EINVAL, "at most 65535 dictionaries");
    *bytes = make_plan(v, nv, *opt, 2).ws_bytes;   // the items do not depend on the output type
    return ok();
}

int nw_batch_create(const nw_vocab *const *v, uint32_t nv, void *const *d_outs, nw_dtype dt, const nw_batch_options *opt,
                    void *d_ws, uint64_t ws_bytes, nw_batch **out)
{
    if (!out) return fail(NW_EINVAL, "out is NULL");
    *out = nullptr;
    if (!v || !nv || !d_outs || !opt) return fail(NW_EINVAL, "NULL argument");
    if (dt != NW_I8 && dt != NW_I16) return fail(NW_EINVAL, "dtype must be NW_I8 or NW_I16");
    for (uint32_t i = 0; i < nv; ++i) {
        if (!v[i]) return fail(NW_EINVAL, "dictionary %u is NULL", i);
        if (!v[i]->symmetric) return fail(NW_EINVAL, "all-pairs scoring needs a symmetric similarity matrix");
        if (v[i]->max_len > (uint32_t)kMaxLen) return fail(NW_EINVAL, "batched form supports words of at most %d symbols", kMaxLen);
        if (dt == NW_I8 && (v[i]->lo < -128 || v[i]->hi > 127))
            return fail(NW_ERANGE, "score bounds of dictionary %u do not fit int8", i);
        if (v[i]->num_pairs && !d_outs[i]) return fail(NW_EINVAL, "output %u is NULL", i);
    }
    if (!d_ws || (uintptr_t)d_ws % 256) return fail(NW_EINVAL, "d_ws must be a 256-byte aligned device pointer");
    nw_batch *B = new nw_batch();
    B->v.assign(v, v + nv);
    B->outs.assign(d_outs, d_outs + nv);
    B->opt = *opt;
    B->plan = make_plan(v, nv, *opt, dt == NW_I8 ? 1 : 2);
    B->out_kind = dt == NW_I8 ? OUT_I8 : OUT_I16;
    B->ws = static_cast<uint8_t *>(d_ws);
    if (ws_bytes < B->plan.ws_bytes) {
        const uint64_t need = B->plan.ws_bytes;
        delete B;
        return fail(NW_ENOMEM, "workspace holds %llu bytes; the batch needs %llu", (unsigned long long)ws_bytes,
                    (unsigned long long)need);
    }
    hipError_t e = hipDeviceGetAttribute(&B->cus, hipDeviceAttributeMultiprocessorCount, v[0]->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
    if (B->plan.width != 0) {
        // the persistent plan's device image: dictionary descriptors, outputs,
        // counters, items (the tiled form reads none of it)
        std::vector<uint8_t> img(B->plan.ws_bytes, 0);
        for (uint32_t i = 0; i < nv; ++i)
            std::memcpy(img.data() + B->plan.off_vocabs + i * sizeof(DevVocab), &v[i]->dev, sizeof(DevVocab));
        std::memcpy(img.data() + B->plan.off_outs, d_outs, 8ull * nv);
        std::memcpy(img.data() + B->plan.off_items, B->plan.items.data(), sizeof(BatchItem) * B->plan.items.size());
        if (e == hipSuccess) e = hipMemcpyAsync(B->ws, img.data(), img.size(), hipMemcpyHostToDevice, B->cap);
        if (e == hipSuccess) e = hipStreamSynchronize(B->cap);
    }
    if (e == hipSuccess && opt->use_graph) {
        // one capture of a run; the fork inside it adds its launches to the
        // capture's graph as chains of kernel nodes
        e = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = B->enqueue(B->cap);
            e = hipStreamEndCapture(B->cap, &B->graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
        nw_batch_destroy(B);
        return dev_fail(e, "creating the batch");
    }
    *out = B;
    return ok();
}

int nw_batch_run(nw_batch *B, void *hip_stream)
{
    if (!B) return fail(NW_EINVAL, "batch is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = B->exec ? hipGraphLaunch(B->exec, s) : B->enqueue(s);
    if (e != hipSuccess) return dev_fail(e, "running the batch");
    return ok();
}

int nw_batch_info(const nw_batch *B, uint64_t *items, uint32_t *launches)
{
    if (!B) return fail(NW_EINVAL, "batch is NULL");
    if (items) *items = B->plan.items.size();
    if (launches) {
        uint32_t n = 0;
        if (B->plan.width == 0) {   // as launch_triangle_tiled issues them
            for (const nw_vocab *x : B->v) {
                if (x->n < 2) continue;
                if ((int64_t)x->n <= kClassLaunchMaxWords) {
                    for (size_t c = 0; c < x->h_maxrp.size(); c += 8) {
                        uint32_t rows = 0;
                        for (size_t la = c; la < std::min(c + 8, x->h_maxrp.size()); ++la) rows += x->h_maxrp[la];
                        n += rows > 0;
                    }
                } else {
                    for (uint32_t c : x->h_maxrp) n += c > 0;
                }
            }
        } else {
            for (size_t c = 0; c + 1 < B->plan.class_off.size(); ++c) n += B->plan.class_off[c + 1] > B->plan.class_off[c];
        }
        *launches = n;
    }
    return ok();
}

void nw_batch_destroy(nw_batch *B)
{
    if (!B) return;
    if (B->exec) hipGraphExecDestroy(B->exec);
    if (B->graph) hipGraphDestroy(B->graph);
    if (B->cap) {
        hipStreamSynchronize(B->cap);
        hipStreamDestroy(B->cap);
    }
    delete B;
}

int nw_batch_autotune(const nw_vocab *const *v, uint32_t nv, void *const *d_outs, nw_dtype dt, void *d_ws,
                      uint64_t ws_bytes, void *hip_stream, const char *cache_path, nw_batch_options *best,
                      float *best_ms)
{
    if (!v || !nv || !best) return fail(NW_EINVAL, "NULL argument");
    // workload signature: device, dtype, and per dictionary n, longest word, alphabet, symbols
    std::ostringstream key;
    key << device_name(v[0]->device) << "|dt" << (int)dt;
    for (uint32_t i = 0; i < nv; ++i) {
        uint64_t sl = 0;
        for (uint8_t l : v[i]->h_clen) sl += l;
        key << "|" << v[i]->n << ":" << v[i]->max_len << ":" << v[i]->dev.alphabet << ":" << sl;
    }
    const std::string k = key.str();
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            if (line.find("\"key\": \"" + k + "\"") == std::string::npos) continue;
            nw_batch_options o{};
            float ms = 0;
            const size_t at = line.find("\"class_width\"");
            if (at == std::string::npos) continue;
            if (std::sscanf(line.c_str() + at,
                            "\"class_width\": %u, \"wg_per_cu\": %u, \"pairs_per_item\": %u, \"use_graph\": %u, "
                            "\"ms\": %f",
                            &o.class_width, &o.wg_per_cu, &o.pairs_per_item, &o.use_graph, &ms) == 5) {
                *best = o;
                if (best_ms) *best_ms = ms;
                return ok();
            }
        }
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (int rc = refuse_capture(s, "nw_batch_autotune")) return rc;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return dev_fail(e, "autotune events");
    auto time_one = [&](const nw_batch_options &o, float &ms) -> int {
        nw_batch *B = nullptr;
        int rc = nw_batch_create(v, nv, d_outs, dt, &o, d_ws, ws_bytes, &B);
        if (rc) return rc;
        rc = nw_batch_run(B, s);   // warm-up
        float tot = 0;
        for (int rep = 0; rep < 2 && !rc; ++rep) {
            hipEventRecord(e0, s);
            rc = nw_batch_run(B, s);
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            float t = 0;
            hipEventElapsedTime(&t, e0, e1);
            tot += t;
        }
        hipStreamSynchronize(s);
        nw_batch_destroy(B);
        ms = tot / 2;
        return rc;
    };
    // coordinate search from (width 8, 4 workgroups per CU, 64 pairs per item)
    nw_batch_options cur{8, 4, 64, 1};
    float cur_ms = 0;
    int rc = time_one(cur, cur_ms);
    const uint32_t widths[] = {0, 1, 8}, wgs[] = {2, 4, 8}, ppi[] = {16, 64, 0};
    // the tiled form launched eagerly (its launches overlap on forked
    // library streams; the captured form replays the same chains as a graph)
    if (!rc) {
        const nw_batch_options o{0, 1, 0, 0};
        float ms = 0;
        rc = time_one(o, ms);
        if (!rc && ms < cur_ms) {
            cur = o;
            cur_ms = ms;
        }
    }
    for (int dim = 0; dim < 3 && !rc; ++dim) {
        if (dim > 0 && cur.class_width == 0) break;   // the tiled form has no persistent parameters
        const uint32_t *vals = dim == 0 ? widths : dim == 1 ? wgs : ppi;
        const int nvals = 3;
        for (int t = 0; t < nvals && !rc; ++t) {
            nw_batch_options o = cur;
            (dim == 0 ? o.class_width : dim == 1 ? o.wg_per_cu : o.pairs_per_item) = vals[t];
            if (o.class_width == cur.class_width && o.wg_per_cu == cur.wg_per_cu && o.pairs_per_item == cur.pairs_per_item)
                continue;
            uint64_t need = 0;
            nw_batch_workspace_bytes(v, nv, &o, &need);
            if (need > ws_bytes) continue;
            float ms = 0;
            rc = time_one(o, ms);
            if (!rc && ms < cur_ms) {
                cur = o;
                cur_ms = ms;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    if (cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        out << "{\"key\": \"" << k << "\", \"class_width\": " << cur.class_width << ", \"wg_per_cu\": " << cur.wg_per_cu
            << ", \"pairs_per_item\": " << cur.pairs_per_item << ", \"use_graph\": " << cur.use_graph
            << ", \"ms\": " << cur_ms << "}\n";
    }
    return ok();
}

}  // extern "C"
