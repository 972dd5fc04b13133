// nw_graph.hip -- the word graph behind Section 5's ego networks: compressed
// rows of an undirected edge list (nw_graph_csr) and breadth-first hop
// distances from a seed set (nw_ego_network).
//
// CSR: per-node degrees with 64-bit atomics (both ends of every edge, which
// also checks the endpoints), an exclusive scan of the degrees into row
// starts (blocks of 1024 nodes scanned in LDS, the block totals scanned by
// one workgroup, then added back), and a fill in which each edge end takes
// the next slot of its row with an atomic cursor.
//
// Ego network: level-synchronous breadth-first search.  Level l expands the
// nodes at distance l; a neighbour still unreached gets l + 1.  Several
// frontier nodes may claim the same neighbour in one level -- they all write
// the same value -- and nodes of the current level are never rewritten, so
// the distances do not depend on the order of the writes.
#include <algorithm>

#include "nw_host.h"

using namespace nw;
using namespace nw::host;

namespace {

constexpr int kGraphThreads = 256;
constexpr int kScanItems = 4;                               // degrees per thread of a scan block
constexpr uint64_t kScanBlock = kGraphThreads * kScanItems;   // degrees per scan block
constexpr int kSeedBatch = 64;                              // seeds per seeding launch (passed by value)

uint32_t stride_grid(uint64_t items)
{
    const uint64_t g = (items + kGraphThreads - 1) / kGraphThreads;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, 256 * 32));
}

__global__ __launch_bounds__(kGraphThreads) void k_graph_degree(const int32_t *ei, const int32_t *ej, uint64_t m,
                                                                uint64_t n, unsigned long long *deg,
                                                                unsigned long long *bad)
{
    const uint64_t step = (uint64_t)gridDim.x * kGraphThreads;
    for (uint64_t e = (uint64_t)blockIdx.x * kGraphThreads + threadIdx.x; e < m; e += step) {
        const uint32_t a = (uint32_t)ei[e], b = (uint32_t)ej[e];   // negative ids wrap past n
        if (a >= n || b >= n) {
            atomicAdd(bad, 1ull);
            continue;
        }
        atomicAdd(&deg[a], 1ull);
        atomicAdd(&deg[b], 1ull);
    }
}

// Inclusive sum over the 64 lanes of a wavefront.
__device__ __forceinline__ unsigned long long wave_inclusive_sum(unsigned long long x, int lane)
{
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long y = __shfl_up(x, (unsigned)d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive prefix of x over the workgroup, and the workgroup total.
__device__ __forceinline__ unsigned long long block_exclusive_sum(unsigned long long x, unsigned long long &total)
{
    __shared__ unsigned long long wtot[kGraphThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long inc = wave_inclusive_sum(x, lane);
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    unsigned long long before = 0;
    total = 0;
    for (int w = 0; w < kGraphThreads / 64; ++w) {
        if (w < wave) before += wtot[w];
        total += wtot[w];
    }
    __syncthreads();   // wtot is reused by the next call
    return before + inc - x;
}

// row_ptr[1 + i] = sum of deg over block-local indices <= i; sums[block] = block total.
__global__ __launch_bounds__(kGraphThreads) void k_scan_block(const unsigned long long *deg, uint64_t n,
                                                              int64_t *row_ptr, unsigned long long *sums)
{
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
    unsigned long long v[kScanItems];
    unsigned long long t = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        t += base + q < n ? deg[base + q] : 0ull;
        v[q] = t;
    }
    unsigned long long total;
    const unsigned long long before = block_exclusive_sum(t, total);
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) row_ptr[1 + base + q] = (int64_t)(before + v[q]);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the block totals in place, by one workgroup.
__global__ __launch_bounds__(kGraphThreads) void k_scan_sums(unsigned long long *sums, uint64_t nblocks)
{
    unsigned long long carry = 0;
    for (uint64_t c = 0; c < nblocks; c += kGraphThreads) {
        const uint64_t i = c + threadIdx.x;
        const unsigned long long x = i < nblocks ? sums[i] : 0ull;
        unsigned long long total;
        const unsigned long long ex = block_exclusive_sum(x, total);
        if (i < nblocks) sums[i] = carry + ex;
        carry += total;
    }
}

// Add each block's offset; row_ptr[0] = 0; the cursor of row i (in place of
// its degree) starts at row_ptr[i].
__global__ __launch_bounds__(kGraphThreads) void k_scan_add(int64_t *row_ptr, uint64_t n,
                                                            const unsigned long long *sums, unsigned long long *deg)
{
    const uint64_t step = (uint64_t)gridDim.x * kGraphThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kGraphThreads + threadIdx.x; i < n; i += step) {
        const int64_t end = row_ptr[1 + i] + (int64_t)sums[i / kScanBlock];
        row_ptr[1 + i] = end;
        deg[i] = (unsigned long long)end - deg[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) row_ptr[0] = 0;
}

__global__ __launch_bounds__(kGraphThreads) void k_graph_fill(const int32_t *ei, const int32_t *ej, uint64_t m,
                                                              unsigned long long *cursor, int32_t *adj)
{
    const uint64_t step = (uint64_t)gridDim.x * kGraphThreads;
    for (uint64_t e = (uint64_t)blockIdx.x * kGraphThreads + threadIdx.x; e < m; e += step) {
        const int32_t a = ei[e], b = ej[e];
        adj[atomicAdd(&cursor[a], 1ull)] = b;
        adj[atomicAdd(&cursor[b], 1ull)] = a;
    }
}

__global__ __launch_bounds__(kGraphThreads) void k_ego_clear(int32_t *dist, uint64_t n)
{
    const uint64_t step = (uint64_t)gridDim.x * kGraphThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kGraphThreads + threadIdx.x; i < n; i += step) dist[i] = -1;
}

struct SeedBatch {
    int32_t v[kSeedBatch];
    int32_t count;
};

__global__ void k_ego_seed(int32_t *dist, SeedBatch s)
{
    if ((int)threadIdx.x < s.count) dist[s.v[threadIdx.x]] = 0;
}

__global__ __launch_bounds__(kGraphThreads) void k_ego_level(const int64_t *row_ptr, const int32_t *adj, uint64_t n,
                                                             int32_t *dist, int32_t level)
{
    const uint64_t step = (uint64_t)gridDim.x * kGraphThreads;
    for (uint64_t v = (uint64_t)blockIdx.x * kGraphThreads + threadIdx.x; v < n; v += step) {
        if (dist[v] != level) continue;
        for (int64_t p = row_ptr[v]; p < row_ptr[v + 1]; ++p) {
            const int32_t u = adj[p];
            if (dist[u] < 0) dist[u] = level + 1;
        }
    }
}

struct GraphWs {
    uint64_t deg, sums, bad, total;
};
GraphWs graph_ws(uint64_t n)
{
    GraphWs w;
    const uint64_t nblocks = (n + kScanBlock - 1) / kScanBlock;
    w.deg = 0;
    w.sums = align_up(8 * std::max<uint64_t>(n, 1), 256);
    w.bad = w.sums + align_up(8 * std::max<uint64_t>(nblocks, 1), 256);
    w.total = w.bad + 256;
    return w;
}

}  // namespace

extern "C" {

int nw_graph_workspace_bytes(uint64_t n, uint64_t *bytes)
{
    if (!bytes) return fail(NW_EINVAL, "bytes is NULL");
    if (n >= (1ull << 31)) return fail(NW_EINVAL, "n must be < 2^31");
    *bytes = graph_ws(n).total;
    return ok();
}

int nw_graph_csr(uint64_t n, const int32_t *d_i, const int32_t *d_j, uint64_t m, int64_t *d_row_ptr, int32_t *d_adj,
                 void *d_ws, uint64_t ws_bytes, void *hip_stream)
{
    if (n >= (1ull << 31)) return fail(NW_EINVAL, "n must be < 2^31");
    if (!d_row_ptr || !d_ws || (m > 0 && (!d_i || !d_j || !d_adj)))
        return fail(NW_EINVAL, "NULL edge, row or workspace pointer");
    if ((uintptr_t)d_ws % 256 || (uintptr_t)d_row_ptr % 8 || (uintptr_t)d_i % 4 || (uintptr_t)d_j % 4 ||
        (uintptr_t)d_adj % 4)
        return fail(NW_EINVAL, "misaligned graph arrays or workspace");
    const GraphWs W = graph_ws(n);
    if (ws_bytes < W.total)
        return fail(NW_ENOMEM, "workspace holds %llu bytes; the graph needs %llu", (unsigned long long)ws_bytes,
                    (unsigned long long)W.total);
    hipStream_t st = (hipStream_t)hip_stream;
    if (int rc = refuse_capture(st, "nw_graph_csr")) return rc;
    uint8_t *ws = static_cast<uint8_t *>(d_ws);
    auto *deg = reinterpret_cast<unsigned long long *>(ws + W.deg);
    auto *sums = reinterpret_cast<unsigned long long *>(ws + W.sums);
    auto *bad = reinterpret_cast<unsigned long long *>(ws + W.bad);
    hipError_t e;
    if ((e = hipMemsetAsync(ws, 0, W.total, st)) != hipSuccess) return dev_fail(e, "clearing the graph workspace");
    if (m > 0) {
        hipLaunchKernelGGL(k_graph_degree, dim3(stride_grid(m)), dim3(kGraphThreads), 0, st, d_i, d_j, m, n, deg, bad);
        if ((e = hipGetLastError()) != hipSuccess) return dev_fail(e, "launching the degree count");
    }
    unsigned long long h_bad = 0;
    if ((e = hipMemcpyAsync(&h_bad, bad, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return dev_fail(e, "reading the endpoint check");
    if (h_bad) return fail(NW_EINVAL, "%llu edges have an endpoint outside [0, %llu)", h_bad, (unsigned long long)n);
    const uint64_t nblocks = (n + kScanBlock - 1) / kScanBlock;
    if (n > 0) {
        hipLaunchKernelGGL(k_scan_block, dim3((uint32_t)nblocks), dim3(kGraphThreads), 0, st, deg, n, d_row_ptr, sums);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kGraphThreads), 0, st, sums, nblocks);
    }
    hipLaunchKernelGGL(k_scan_add, dim3(stride_grid(std::max<uint64_t>(n, 1))), dim3(kGraphThreads), 0, st, d_row_ptr,
                       n, sums, deg);
    if (m > 0)
        hipLaunchKernelGGL(k_graph_fill, dim3(stride_grid(m)), dim3(kGraphThreads), 0, st, d_i, d_j, m, deg, d_adj);
    if ((e = hipGetLastError()) != hipSuccess) return dev_fail(e, "launching the row build");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return dev_fail(e, "building the rows");
    return ok();
}

int nw_ego_network(uint64_t n, const int64_t *d_row_ptr, const int32_t *d_adj, const int32_t *h_seeds,
                   uint32_t n_seeds, uint32_t depth, int32_t *d_dist, void *hip_stream)
{
    if (n >= (1ull << 31)) return fail(NW_EINVAL, "n must be < 2^31");
    if (!d_row_ptr || !d_dist || (n_seeds > 0 && !h_seeds)) return fail(NW_EINVAL, "NULL graph, seed or output pointer");
    if (depth > 1000000) return fail(NW_EINVAL, "depth %u exceeds 1000000", depth);
    for (uint32_t t = 0; t < n_seeds; ++t)
        if (h_seeds[t] < 0 || (uint64_t)h_seeds[t] >= n)
            return fail(NW_EINVAL, "seed %d outside [0, %llu)", h_seeds[t], (unsigned long long)n);
    if (n == 0) return ok();
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_ego_clear, dim3(stride_grid(n)), dim3(kGraphThreads), 0, st, d_dist, n);
    for (uint32_t t0 = 0; t0 < n_seeds; t0 += kSeedBatch) {
        SeedBatch s{};
        s.count = (int32_t)std::min<uint32_t>(kSeedBatch, n_seeds - t0);
        for (int q = 0; q < s.count; ++q) s.v[q] = h_seeds[t0 + q];
        hipLaunchKernelGGL(k_ego_seed, dim3(1), dim3(kSeedBatch), 0, st, d_dist, s);
    }
    // a breadth-first distance never reaches n, so deeper levels find nothing
    const uint32_t levels = (uint32_t)std::min<uint64_t>(depth, n);
    if (n_seeds > 0)
        for (uint32_t l = 0; l < levels; ++l) {
            if (!d_adj) break;
            hipLaunchKernelGGL(k_ego_level, dim3(stride_grid(n)), dim3(kGraphThreads), 0, st, d_row_ptr, d_adj, n,
                               d_dist, (int32_t)l);
        }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return dev_fail(e, "launching the ego-network search");
    return ok();
}

}  // extern "C"
