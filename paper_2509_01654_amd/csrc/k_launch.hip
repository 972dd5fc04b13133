// k_launch.hip -- launchers of every kernel, and the naive triangle kernel.
//
// Naive kernel (k_tri_naive): the paper's GPU scheme (Section 4.2): one thread
// per pair index, a 1-D grid, idx -> (row, column) through the closed form of
// the row index, and one DP per thread with its scratch in shared memory (one
// row of the score matrix instead of the whole matrix).
#define NW_LAUNCH_TU 1
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "k_batch.h"
#include "k_diag.h"
#include "k_edges.h"
#include "k_probe.h"
#include "k_query.h"
#include "k_topk.h"
#include "k_topk_code.h"
#include "k_tri_code.h"
#include "k_tri_tiled.h"
#include "nw_fork.h"
#include "nw_kernels.h"

namespace nw {

// CAP: scratch row capacity (longest word + 1); NT: threads per block.  The
// score goes to out (OUT_I8 / OUT_I16) or, if it passes the slice, to E.
template <int CAP, int NT>
__global__ __launch_bounds__(NT) void k_tri_naive(DevVocab V, uint64_t idx_begin, uint64_t idx_end, void *out,
                                                  int out_kind, EdgeSink E)
{
    __shared__ int16_t rows[NT][CAP];
    int16_t *row = rows[threadIdx.x];   // this thread's scratch: one row of the score matrix
    const int64_t n = V.n;
    const int gap = V.gap;
    const double z = (double)n - 0.5;
    for (uint64_t idx = idx_begin + (uint64_t)blockIdx.x * NT + threadIdx.x; idx < idx_end;
         idx += (uint64_t)gridDim.x * NT) {
        // r = floor(z - sqrt(z^2 - 2 idx)), z = n - 1/2 (Section 4.2), then an
        // integer fix-up so rounding can never pick the wrong row
        int64_t r = (int64_t)floor(z - sqrt(z * z - 2.0 * (double)idx));
        if (r < 0) r = 0;
        if (r > n - 2) r = n - 2;
        while (r > 0 && row_start_idx(n, r) > idx) --r;
        while (r + 1 < n - 1 && row_start_idx(n, r + 1) <= idx) ++r;
        const int64_t c = r + 1 + (int64_t)(idx - row_start_idx(n, r));
        const int la = V.clen[r], lb = V.clen[c];
        const uint8_t *A = V.csym + r * V.WB;
        const uint8_t *B = V.csym + c * V.WB;
        for (int j = 0; j <= lb; ++j) row[j] = (int16_t)(gap * j);
        for (int i = 1; i <= la; ++i) {
            int diag = row[0];
            row[0] = (int16_t)(gap * i);
            const int a = A[i - 1];
            for (int j = 1; j <= lb; ++j) {
                const int bsym = B[j - 1];
                const int sim = V.has_submat ? (int)V.submat[a * V.alphabet + bsym] : (a == bsym ? V.match : V.mismatch);
                const int up = row[j];
                int v = diag + sim;
                v = max(v, up + gap);
                v = max(v, (int)row[j - 1] + gap);
                diag = up;
                row[j] = (int16_t)v;
            }
        }
        const int score = row[lb];
        if (out_kind == OUT_I8)
            static_cast<int8_t *>(out)[idx - idx_begin] = (int8_t)score;
        else if (out_kind == OUT_I16)
            static_cast<int16_t *>(out)[idx - idx_begin] = (int16_t)score;
        else if (edge_passes(E, score, la, lb))
            edge_direct(E, (int32_t)r, (int32_t)c, score);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
const KernelTables &kernel_tables()
{
    static KernelTables t;
    static bool init = [] {
#define X(lo, hi) nw_fill_##lo(t);
        NW_LA_SPLITS
#undef X
#define X(lo, hi) nw_fill_class_##lo(t);
        NW_CLASS8
#undef X
        return true;
    }();
    (void)init;
    return t;
}

// A launch through a fork (a stream, or a node of the graph being captured).
static hipError_t launch_dyn(const void *fn, dim3 grid, size_t lds, StreamFork &fork, void **args)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return fork.launch(fn, grid, dim3(kThreads), lds, args);
}

// Row of pair index idx in the row-major triangle of n words: the largest u
// with S_{u-1} = (n-1)u - u(u-1)/2 <= idx (Section 4.2), by bisection.
static int64_t row_of_index(int64_t n, uint64_t idx)
{
    auto start = [n](int64_t u) { return (uint64_t)(n - 1) * (uint64_t)u - (uint64_t)u * (uint64_t)(u - 1) / 2u; };
    int64_t lo = 0, hi = n - 2;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (start(mid) <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Grid of a triangle launch over pair indices [idx_begin, idx_end): the whole
// column-major block-pair space, or a row-major window over the block rows
// the range touches when that is smaller.
struct TriGrid {
    uint32_t blocks, rb0, rbn;
};
static TriGrid tri_grid(const DevVocab &V, uint64_t idx_begin, uint64_t idx_end)
{
    const uint64_t all = (uint64_t)V.nb * (V.nb + 1) / 2;
    const uint32_t r0 = (uint32_t)(row_of_index(V.n, idx_begin) / V.CB);
    const uint32_t r1 = (uint32_t)(row_of_index(V.n, idx_end - 1) / V.CB);
    const uint64_t win = (uint64_t)(r1 - r0 + 1) * (uint64_t)V.nb;
    if (win < all) return {(uint32_t)win, r0, r1 - r0 + 1};
    return {(uint32_t)all, 0, 0};
}

// How many runs of row pairs a launch of `tiles` tiles cuts each tile of a
// row length into (at most maxrp row pairs per tile).  A launch with fewer
// tiles than workgroup slots (256 CUs x 6) splits its tiles into runs of at
// least kMinRowPairs row pairs, up to about four workgroups per slot; short
// runs cost more than they balance.
static uint32_t tile_chunks(uint64_t tiles, uint32_t maxrp)
{
    constexpr uint64_t kTargetWorkgroups = 256 * 6 * 4;
    constexpr uint64_t kSplitBelow = 2048;
    constexpr uint32_t kMinRowPairs = 16;
    if (tiles >= kSplitBelow) return 1;
    const uint32_t want = (uint32_t)((kTargetWorkgroups + tiles - 1) / tiles);
    return std::max<uint32_t>(1, std::min(want, maxrp / kMinRowPairs));
}

// NW_EPILOGUE=plain keeps the kernels with the plain integer epilogue where
// the score-code kernels would apply (both are exact; for comparisons).
static bool plain_epilogue_only()
{
    static const bool only = [] {
        const char *e = std::getenv("NW_EPILOGUE");
        return e && std::strcmp(e, "plain") == 0;
    }();
    return only;
}

hipError_t launch_triangle_tiled(const DevVocab &V, const uint32_t *h_maxrp, uint64_t idx_begin, uint64_t idx_end,
                                 int out_kind, void *d_out, hipStream_t stream, const EdgeSink *E, StreamFork *shared)
{
    if (idx_begin >= idx_end || V.n < 2) return hipSuccess;
    const TriGrid G = tri_grid(V, idx_begin, idx_end);
    const KernelTables &tab = kernel_tables();
    StreamFork own(stream);
    if (!shared) {
        hipError_t ef = own.begin();
        if (ef != hipSuccess) return ef;
    }
    StreamFork &fork = shared ? *shared : own;
    if (V.n <= kClassLaunchMaxWords) {
        // small dictionaries: one launch per class of 8 row lengths
        // (k_tri_class; the per-length launches would be bound by launch cost)
        for (int c = 0; c < kNumClass8 && 8 * c <= V.lmax; ++c) {
            const int lo = 8 * c, hi = std::min(8 * c + 7, (int)V.lmax);
            uint32_t rows = 0, maxrp = 0;
            size_t lds = 0;
            for (int LA = lo; LA <= hi; ++LA) {
                rows += h_maxrp[LA];
                maxrp = std::max(maxrp, h_maxrp[LA]);
                lds = std::max<size_t>(lds, tri_lds_bytes(LA, V.alphabet, V.CB));
            }
            if (rows == 0) continue;
            // runs of at least two row pairs, about 2048 workgroups per launch
            const uint64_t ny = (uint64_t)(hi - lo + 1);
            uint32_t chunks = (uint32_t)std::max<uint64_t>(
                1, std::min<uint64_t>((2048 + G.blocks * ny - 1) / (G.blocks * ny), (maxrp + 1) / 2));
            uint32_t rpc = (maxrp + chunks - 1) / chunks;
            DevVocab Vc = V;
            uint64_t ib = idx_begin, ie = idx_end;
            void *po = d_out;
            int ok = out_kind;
            EdgeSink es = E ? *E : EdgeSink{};
            uint32_t rb0 = G.rb0, rbn = G.rbn;
            void *args[] = {&Vc, &ib, &ie, &po, &ok, &es, &rb0, &rbn, &chunks, &rpc};
            hipError_t e = launch_dyn(tab.class8[c], dim3((uint32_t)((uint64_t)G.blocks * chunks), (uint32_t)ny), lds,
                                      fork, args);
            if (e != hipSuccess) return e;
        }
        return shared ? hipSuccess : own.end();
    }
    const bool code_ok = out_kind != OUT_EDGES && !plain_epilogue_only();
    for (int LA = 0; LA <= V.lmax; ++LA) {
        if (h_maxrp[LA] == 0) continue;   // no block has row pairs of this length
        uint32_t chunks = tile_chunks(G.blocks, h_maxrp[LA]);
        uint32_t rpc = (h_maxrp[LA] + chunks - 1) / chunks;
        int esz = out_kind == OUT_I8 ? 1 : 2;
        const int R = code_ok && tab.tri_code2[LA] && tri_code_applies(V, LA, esz, 2)   ? 2
                      : code_ok && tri_code_applies(V, LA, esz, 1) ? 1
                                                                   : 0;
        if (R) {
            // runs of whole steps
            rpc = (rpc + R - 1) / R * R;
            DevVocab Vc = V;
            uint64_t ib = idx_begin, ie = idx_end;
            void *po = d_out;
            uint32_t rb0 = G.rb0, rbn = G.rbn;
            void *args[] = {&Vc, &ib, &ie, &po, &esz, &rb0, &rbn, &chunks, &rpc};
            hipError_t e = launch_dyn(R == 2 ? tab.tri_code2[LA] : tab.tri_code1[LA],
                                      dim3((uint32_t)((uint64_t)G.blocks * chunks)),
                                      tri_code_lds_bytes(LA, V.alphabet, V.CB, esz, R), fork, args);
            if (e != hipSuccess) return e;
            continue;
        }
        DevVocab Vc = V;
        uint64_t ib = idx_begin, ie = idx_end;
        void *po = d_out;
        int ok = out_kind;
        EdgeSink es = E ? *E : EdgeSink{};
        uint32_t rb0 = G.rb0, rbn = G.rbn;
        void *args[] = {&Vc, &ib, &ie, &po, &ok, &es, &rb0, &rbn, &chunks, &rpc};
        hipError_t e = launch_dyn(tab.tri[LA], dim3((uint32_t)((uint64_t)G.blocks * chunks)),
                                  tri_lds_bytes(LA, V.alphabet, V.CB), fork, args);
        if (e != hipSuccess) return e;
    }
    return shared ? hipSuccess : own.end();
}

hipError_t launch_edges_tiled(const DevVocab &V, const uint32_t *h_maxrp, uint64_t idx_begin, uint64_t idx_end,
                              const EdgeSink &E, hipStream_t stream)
{
    if (idx_begin >= idx_end || V.n < 2) return hipSuccess;
    const TriGrid G = tri_grid(V, idx_begin, idx_end);
    const KernelTables &tab = kernel_tables();
    StreamFork fork(stream);
    hipError_t ef = fork.begin();
    if (ef != hipSuccess) return ef;
    for (int LA = 0; LA <= V.lmax; ++LA) {
        if (h_maxrp[LA] == 0) continue;
        uint32_t chunks = tile_chunks(G.blocks, h_maxrp[LA]);
        uint32_t rpc = (h_maxrp[LA] + chunks - 1) / chunks;
        DevVocab Vc = V;
        EdgeSink Ec = E;
        uint64_t ib = idx_begin, ie = idx_end;
        uint32_t rb0 = G.rb0, rbn = G.rbn;
        void *args[] = {&Vc, &Ec, &ib, &ie, &rb0, &rbn, &chunks, &rpc};
        hipError_t e = launch_dyn(tab.edges[LA], dim3((uint32_t)((uint64_t)G.blocks * chunks)),
                                  edges_lds_bytes(LA, V.alphabet, V.CB), fork, args);
        if (e != hipSuccess) return e;
    }
    return fork.end();
}

hipError_t launch_triangle_naive(const DevVocab &V, uint64_t idx_begin, uint64_t idx_end, int out_kind, void *d_out,
                                 hipStream_t stream, const EdgeSink *E)
{
    if (idx_begin >= idx_end) return hipSuccess;
    const uint64_t count = idx_end - idx_begin;
    const bool lng = V.lmax > kMaxLen;
    const uint64_t nt = lng ? 64 : 256;
    const uint64_t blocks = (count + nt - 1) / nt;
    const uint32_t grid = (uint32_t)(blocks < (1u << 20) ? blocks : (1u << 20));
    const EdgeSink es = E ? *E : EdgeSink{};
    if (!lng)
        hipLaunchKernelGGL((k_tri_naive<kMaxLen + 1, 256>), dim3(grid), dim3(256), 0, stream, V, idx_begin, idx_end,
                           d_out, out_kind, es);
    else
        hipLaunchKernelGGL((k_tri_naive<kLongMaxLen + 1, 64>), dim3(grid), dim3(64), 0, stream, V, idx_begin, idx_end,
                           d_out, out_kind, es);
    return hipGetLastError();
}

bool diag_fits(const DevVocab &V)
{
    for (int c = 0; c < kDiagClasses; ++c)
        if (32 * c + 1 <= V.lmax && diag_lds_bytes(diag_rows_per_lane(c), V.alphabet, V.CB) > kMaxLdsBytes) return false;
    return true;
}

hipError_t launch_triangle_diag(const DevVocab &V, const uint32_t *h_maxrp, const uint32_t *h_maxdp,
                                uint64_t idx_begin, uint64_t idx_end, int out_kind, void *d_out, hipStream_t stream,
                                const EdgeSink *E)
{
    if (idx_begin >= idx_end || V.n < 2) return hipSuccess;
    // a class whose profile does not fit in LDS (large alphabets with long
    // words): the whole range goes through the one-thread-per-pair kernel
    if (!diag_fits(V)) return launch_triangle_naive(V, idx_begin, idx_end, out_kind, d_out, stream, E);
    const TriGrid G = tri_grid(V, idx_begin, idx_end);
    const KernelTables &tab = kernel_tables();
    StreamFork fork(stream);
    hipError_t ef = fork.begin();
    if (ef != hipSuccess) return ef;
    DevVocab Vc = V;
    uint64_t ib = idx_begin, ie = idx_end;
    void *po = d_out;
    int ok = out_kind;
    EdgeSink es = E ? *E : EdgeSink{};
    uint32_t rb0 = G.rb0, rbn = G.rbn;
    if (h_maxrp[0] != 0) {   // empty row words: score gap * lb, the register-row kernel of length 0
        uint32_t one = 1, all = 0xFFFFFFFFu;
        void *args[] = {&Vc, &ib, &ie, &po, &ok, &es, &rb0, &rbn, &one, &all};
        hipError_t e = launch_dyn(tab.tri[0], dim3(G.blocks), tri_lds_bytes(0, V.alphabet, V.CB), fork, args);
        if (e != hipSuccess) return e;
    }
    for (int c = 0; c < kDiagClasses; ++c) {
        const int R = diag_rows_per_lane(c);
        const uint32_t maxrp = h_maxdp[c];   // most row pairs of this class in one block
        if (maxrp == 0) continue;
        // runs of row pairs so that a launch has about kDiagWorkgroups workgroups
        constexpr uint64_t kDiagWorkgroups = 2048;
        uint32_t chunks = (uint32_t)std::min<uint64_t>(maxrp, std::max<uint64_t>(1, (kDiagWorkgroups + G.blocks - 1) / G.blocks));
        uint32_t rpc = (maxrp + chunks - 1) / chunks;
        static const void *const kDiag[kDiagClasses] = {
            reinterpret_cast<const void *>(&k_tri_diag<2>),  reinterpret_cast<const void *>(&k_tri_diag<4>),
            reinterpret_cast<const void *>(&k_tri_diag<6>),  reinterpret_cast<const void *>(&k_tri_diag<8>),
            reinterpret_cast<const void *>(&k_tri_diag<10>), reinterpret_cast<const void *>(&k_tri_diag<12>),
            reinterpret_cast<const void *>(&k_tri_diag<14>), reinterpret_cast<const void *>(&k_tri_diag<16>)};
        const void *fn = kDiag[c];
        void *args[] = {&Vc, &ib, &ie, &po, &ok, &es, &rb0, &rbn, &chunks, &rpc};
        const size_t lds = diag_lds_bytes(R, V.alphabet, V.CB);
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        e = fork.launch(fn, dim3((uint32_t)((uint64_t)G.blocks * chunks)), dim3(kDiagThreads), lds, args);
        if (e != hipSuccess) return e;
    }
    return fork.end();
}

hipError_t launch_query(const DevVocab &V, const RowSet &R, const uint32_t *h_off, const ColSet &C, int k,
                        int nsplit, uint64_t *partial, hipStream_t stream, bool fork_streams)
{
    const KernelTables &tab = kernel_tables();
    StreamFork fork(stream);
    if (fork_streams) {
        hipError_t ef = fork.begin();
        if (ef != hipSuccess) return ef;
    }
    int64_t per = (C.nslots + nsplit - 1) / nsplit;
    per = (per + kThreads - 1) / kThreads * kThreads;
    const int rpw = 4;
    for (int LA = 0; LA <= kMaxLen; ++LA) {
        const uint32_t np = h_off[LA + 1] - h_off[LA];
        if (np == 0) continue;
        QueryArgs Q;
        Q.R = R;
        Q.C = C;
        Q.wtab = V.wtab;
        Q.alphabet = V.alphabet;
        Q.gap = V.gap;
        Q.lo = V.lo;
        Q.k = k;
        Q.rpw = rpw;
        Q.per = per;
        Q.nsplit = nsplit;
        Q.partial = partial;
        void *args[] = {&Q};
        const dim3 grid((np + rpw - 1) / rpw, nsplit);
        hipError_t e = launch_dyn(tab.query[LA], grid, query_lds_bytes(LA, V.alphabet, k), fork, args);
        if (e != hipSuccess) return e;
    }
    return fork_streams ? fork.end() : hipSuccess;
}

// NW_PREPASS=lists keeps the list pre-pass (k_query_tiled + merge) where the
// selection would apply (both give the same keys; for comparisons).
static bool list_prepass_only()
{
    static const bool only = [] {
        const char *e = std::getenv("NW_PREPASS");
        return e && std::strcmp(e, "lists") == 0;
    }();
    return only;
}

bool probe_thr_applies(const DevVocab &V)
{
    return !list_prepass_only() && V.hi - V.lo <= kProbeMaxCode && V.pslots <= kProbeMaxSlots &&
           probe_lds_bytes(kMaxLen, V.alphabet, V.pslots) <= 65536u;
}

hipError_t launch_probe_thr(const DevVocab &V, const RowSet &R, const uint32_t *h_off, int m, uint64_t *thr,
                            hipStream_t stream)
{
    if (!probe_thr_applies(V)) return hipErrorNotSupported;
    const KernelTables &tab = kernel_tables();
    StreamFork fork(stream);
    hipError_t ef = fork.begin();
    if (ef != hipSuccess) return ef;
    const int rpw = 1;   // a workgroup per row pair: measured best of 1, 2, 4, 8 and 16
    for (int LA = 0; LA <= kMaxLen; ++LA) {
        const uint32_t np = h_off[LA + 1] - h_off[LA];
        if (np == 0) continue;
        ProbeArgs Q;
        Q.R = R;
        Q.C.sym = V.psym;
        Q.C.len = V.plen;
        Q.C.orig = V.porig;
        Q.C.nslots = V.pslots;
        Q.rank = V.prank;
        Q.wtab = V.wtab;
        Q.alphabet = V.alphabet;
        Q.gap = V.gap;
        Q.lo = V.lo;
        Q.m = m;
        Q.rpw = rpw;
        Q.n = V.n;
        Q.nprobe = V.nprobe;
        Q.thr = thr;
        void *args[] = {&Q};
        hipError_t e = launch_dyn(tab.probe_thr[LA], dim3((np + rpw - 1) / rpw), probe_lds_bytes(LA, V.alphabet, V.pslots),
                                  fork, args);
        if (e != hipSuccess) return e;
    }
    return fork.end();
}

hipError_t launch_merge(const uint64_t *partial, int P, int kin, int64_t rows, int kout, int lo, int16_t *score,
                        int32_t *index, uint64_t *thr, int rank, hipStream_t stream)
{
    if (rows <= 0) return hipSuccess;
    if ((int64_t)P * kin >= 1024) {   // many keys per row: a workgroup each
        hipLaunchKernelGGL(k_merge_lists_wg, dim3((uint32_t)rows), dim3(256), 0, stream, partial, P, kin, rows, kout, lo,
                           score, index, thr, rank);
        return hipGetLastError();
    }
    const uint32_t grid = (uint32_t)((rows + 3) / 4);
    hipLaunchKernelGGL(k_merge_lists, dim3(grid), dim3(256), 0, stream, partial, P, kin, rows, kout, lo, score, index,
                       thr, rank);
    return hipGetLastError();
}

hipError_t launch_topk_main(const DevVocab &V, const TopkArgs &T, hipStream_t stream)
{
    if (V.n < 2) return hipSuccess;
    const uint32_t nblk_pairs = (uint32_t)((uint64_t)V.nb * (V.nb + 1) / 2);
    const KernelTables &tab = kernel_tables();
    StreamFork fork(stream);
    hipError_t ef = fork.begin();
    if (ef != hipSuccess) return ef;
    for (int LA = 0; LA <= V.lmax; ++LA) {
        DevVocab Vc = V;
        TopkArgs Tc = T;
        hipError_t e;
        if (!plain_epilogue_only() && topk_code_applies(V, T, LA)) {
            // score codes within [0, 1024), the histogram in LDS below 64 KiB
            Tc.hist_in_lds = T.hist != nullptr;
            Tc.wt_in_lds = topk_code_wt_in_lds(V, T, LA);
            void *args[] = {&Vc, &Tc};
            e = launch_dyn(tab.topk_code[LA], dim3(nblk_pairs),
                           topk_code_lds_bytes(LA, V.alphabet, T.nbins, Tc.hist_in_lds, V.CB, Tc.wt_in_lds), fork, args);
        } else {
            // the histogram copies go to LDS when they fit beside the profiles
            // (large alphabets with wide score ranges add to global bins instead)
            Tc.hist_in_lds = T.hist != nullptr && T.nbins <= kLdsHistMax &&
                             topk_lds_bytes(LA, V.alphabet, T.nbins, 1, V.CB) <= kMaxLdsBytes;
            void *args[] = {&Vc, &Tc};
            e = launch_dyn(tab.topk[LA], dim3(nblk_pairs), topk_lds_bytes(LA, V.alphabet, T.nbins, Tc.hist_in_lds, V.CB),
                           fork, args);
        }
        if (e != hipSuccess) return e;
    }
    return fork.end();
}

__global__ void k_scatter_lists(const int16_t *qs, const int32_t *qi, const int32_t *words, uint32_t B, int kq, int k,
                                int16_t *score, int32_t *index)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B) return;
    const int32_t w = words[t];
    int o = 0;
    for (int c = 0; c < kq && o < k; ++c) {
        const int32_t j = qi[(size_t)t * kq + c];
        if (j == w) continue;   // no self-loops
        score[(size_t)w * k + o] = qs[(size_t)t * kq + c];
        index[(size_t)w * k + o] = j;
        ++o;
    }
    for (; o < k; ++o) {
        score[(size_t)w * k + o] = (int16_t)-32768;
        index[(size_t)w * k + o] = -1;
    }
}

hipError_t launch_scatter_lists(const int16_t *qs, const int32_t *qi, const int32_t *words, uint32_t B, int kq, int k,
                                int16_t *score, int32_t *index, hipStream_t stream)
{
    if (B == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_lists, dim3((B + 255) / 256), dim3(256), 0, stream, qs, qi, words, B, kq, k, score,
                       index);
    return hipGetLastError();
}

hipError_t launch_reset_counters(uint32_t *counters, int n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_reset_counters, dim3((n + 63) / 64), dim3(64), 0, stream, counters, n);
    return hipGetLastError();
}

hipError_t launch_tighten(const uint32_t *cnt, const uint64_t *lists, uint32_t cap, int64_t n, int k, uint64_t *thr,
                          hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tighten, dim3((uint32_t)((n + 3) / 4)), dim3(256), 0, stream, cnt, lists, cap, n, k, thr);
    return hipGetLastError();
}

hipError_t launch_select(const uint32_t *cnt, const uint64_t *lists, uint32_t cap, int64_t n, int k, int lo,
                         int16_t *score, int32_t *index, uint32_t *ovf_count, int32_t *ovf_list, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const uint32_t grid = (uint32_t)((n + 3) / 4);
    hipLaunchKernelGGL(k_select, dim3(grid), dim3(256), 0, stream, cnt, lists, cap, n, k, lo, score, index, ovf_count,
                       ovf_list);
    return hipGetLastError();
}

}  // namespace nw
