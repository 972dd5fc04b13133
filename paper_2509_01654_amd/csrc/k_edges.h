// k_edges.h -- the threshold edge emitter as a kernel of its own: every pair
// of a tile is scored in registers and tested against the weight slice right
// after its DP, so no score is staged in LDS or re-read.
//
// Layout and loop are those of the top-k main pass: a workgroup takes a tile
// (block pair r <= b, row length LA, a run of row pairs), stages the column
// block's lengths and columns in LDS once, and deals the length-sorted column
// slots to the wavefronts in groups of 64 (every wavefront gets the same mix
// of lengths).  Lane words are prefetched one ahead into two register sets.
// Passing pairs go to one of two LDS pools (by row-pair parity); a pool is
// moved to the edge arrays between row pairs, with one global atomic per
// flush reserving its slots, so the DP loop never waits on global memory.  A
// full pool sends further edges straight to the arrays (one atomic each).
#pragma once

#include "k_topk.h"
#include "nw_tile_common.h"

namespace nw {

constexpr int kEdgePool = 128;       // entries per pool
constexpr int kEdgePoolFlush = 64;   // a pool is flushed once it holds this many

// LDS: two profiles, the column block's metadata (column | length << 16, 4 B
// per slot), two pools of (i, j, score) and their counters.
__host__ __device__ constexpr uint32_t edges_pool_bytes() { return 2u * kEdgePool * 12u + 16u; }
__host__ __device__ constexpr uint32_t edges_lds_bytes(int LA, int alphabet, int CB)
{
    return 2u * profile_bytes(LA, alphabet) + 4u * (uint32_t)CB + edges_pool_bytes();
}

struct EdgePool {
    int32_t *i;       // [2][kEdgePool]
    int32_t *j;       // [2][kEdgePool]
    int32_t *s;       // [2][kEdgePool]
    uint32_t *n;      // [2] appends so far (may pass kEdgePool)
};

__device__ __forceinline__ void edge_direct(const EdgeSink &E, int32_t i, int32_t j, int s)
{
    const unsigned long long q = atomicAdd(E.count, 1ull);
    if (q < E.cap) {
        E.ei[q] = i;
        E.ej[q] = j;
        E.es[q] = (int16_t)s;
    }
}

__device__ __forceinline__ void edge_offer(const EdgePool &P, int b, const EdgeSink &E, int32_t i, int32_t j, int s)
{
    const uint32_t p = atomicAdd(&P.n[b], 1u);
    if (p < (uint32_t)kEdgePool) {
        P.i[b * kEdgePool + p] = i;
        P.j[b * kEdgePool + p] = j;
        P.s[b * kEdgePool + p] = s;
    } else {
        edge_direct(E, i, j, s);
    }
}

// Move pool b to the edge arrays.  Every thread of the workgroup calls it
// while no thread appends to pool b; count is the pool's counter as every
// thread read it.  Ends with a barrier and the pool empty.
__device__ __forceinline__ void edge_flush(const EdgePool &P, int b, const EdgeSink &E, uint32_t count,
                                           unsigned long long *base_lds)
{
    const uint32_t m = min(count, (uint32_t)kEdgePool);
    if (threadIdx.x == 0) *base_lds = atomicAdd(E.count, (unsigned long long)m);
    __syncthreads();
    const unsigned long long base = *base_lds;
    for (uint32_t t = threadIdx.x; t < m; t += kThreads) {
        const unsigned long long q = base + t;
        if (q < E.cap) {
            E.ei[q] = P.i[b * kEdgePool + t];
            E.ej[q] = P.j[b * kEdgePool + t];
            E.es[q] = (int16_t)P.s[b * kEdgePool + t];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) P.n[b] = 0;
}

template <int LA>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(topk_min_waves<LA>())))
void k_edges_tiled(DevVocab V, EdgeSink E, uint64_t idx_begin, uint64_t idx_end, uint32_t rb0, uint32_t rbn,
                   uint32_t chunks, uint32_t rpc)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ unsigned long long flush_base;
    uint32_t r, b;
    if (!tile_block_pair(blockIdx.x / chunks, rb0, rbn, V.nb, r, b)) return;
    const uint32_t *rpo = V.rp_off + (size_t)r * (V.lmax + 1) + LA;
    const uint64_t pbeg64 = (uint64_t)rpo[0] + (uint64_t)(blockIdx.x % chunks) * rpc;
    if (pbeg64 >= rpo[1]) return;
    const uint32_t pbeg = (uint32_t)pbeg64;
    const uint32_t pend = rpo[1] - pbeg <= rpc ? rpo[1] : pbeg + rpc;

    const int64_t n = V.n, CB = V.CB;
    const int64_t I0 = (int64_t)r * CB, I1 = min(I0 + CB, n);
    const int64_t J0 = (int64_t)b * CB, J1 = min(J0 + CB, n);
    // the tile's pair indices: skip a tile outside [idx_begin, idx_end), and
    // test every pair only when the tile straddles a bound (uniform)
    bool whole;
    {
        const int64_t jlo = (r == b) ? I0 + 1 : J0;
        if (jlo >= J1) return;
        const uint64_t first = row_start_idx(n, I0) + (uint64_t)(jlo - I0 - 1);
        const int64_t ilast = (r == b) ? J1 - 2 : I1 - 1;
        const uint64_t last = row_start_idx(n, ilast) + (uint64_t)(J1 - 1 - ilast - 1);
        if (last < idx_begin || first >= idx_end) return;
        whole = first >= idx_begin && last < idx_end;
    }

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint32_t prof_bytes = profile_bytes(LA, V.alphabet);
    uint32_t *meta = reinterpret_cast<uint32_t *>(lds + 2 * prof_bytes);
    EdgePool pool;
    {
        uint8_t *pb = lds + 2 * prof_bytes + 4u * (uint32_t)CB;
        pool.i = reinterpret_cast<int32_t *>(pb);
        pool.j = reinterpret_cast<int32_t *>(pb + 2 * kEdgePool * 4);
        pool.s = reinterpret_cast<int32_t *>(pb + 2 * kEdgePool * 8);
        pool.n = reinterpret_cast<uint32_t *>(pb + 2 * kEdgePool * 12);
        if (tid < 2) pool.n[tid] = 0;
    }
    for (int t = tid; t < CB; t += kThreads) meta[t] = (uint32_t)V.bcol[J0 + t] | ((uint32_t)V.blen[J0 + t] << 16);
    const ProfileRole role = profile_role(tid, V.alphabet);
    const int CPL = V.CB / kThreads;
    const int lane_base = wave * 64 + lane;   // column word c: slot c*256 + wave*64 + lane
    const int off_a = V.gap * LA;

    for (uint32_t k = pbeg; k < pend; ++k) {
        const int32_t a0 = V.rpairs[2 * k], a1 = V.rpairs[2 * k + 1];
        const uint8_t *prof = lds + (k & 1) * prof_bytes;
        build_profile<LA>(V.wtab, V.alphabet, reinterpret_cast<uint32_t *>(lds + (k & 1) * prof_bytes),
                          V.bsym + (int64_t)a0 * kWordBytes, V.bsym + (int64_t)(a1 >= 0 ? a1 : a0) * kWordBytes, role);
        __syncthreads();
        const int pb = (int)(k & 1);
        {
            const uint32_t other = pool.n[pb ^ 1];
            if (other >= (uint32_t)kEdgePoolFlush) edge_flush(pool, pb ^ 1, E, other, &flush_base);
        }
        const int64_t u0 = I0 + V.bcol[a0];
        const int64_t u1 = a1 >= 0 ? I0 + V.bcol[a1] : -1;
        const uint64_t base0 = row_start_idx(n, u0) - (uint64_t)u0 - 1;   // idx(u0, j) = base0 + j
        const uint64_t base1 = u1 >= 0 ? row_start_idx(n, u1) - (uint64_t)u1 - 1 : 0;

        auto column = [&](const uint32_t(&bw)[kWordBytes / 4], int c) __attribute__((always_inline)) {
            const uint32_t m = meta[lane_base + c * kThreads];
            const int lb = (int)(m >> 16);
            const int col = (int)(m & 0xFFFF);
            const int lbmax_w = __builtin_amdgcn_readlane(lb, 63);
            h2 g;
            if constexpr (LA == 0)
                g = h2{0, 0};
            else
                g = dp_lane<LA, kWordBytes>(bw, lbmax_w, prof, profile_stride_dw<LA>() * 4u);
            if (col == 0xFFFF) return;
            const int off = off_a + __mul24(V.gap, lb);
            const int s0 = (int)g[0] + off, s1 = (int)g[1] + off;
            const int64_t j = J0 + col;
            bool v0 = (r < b) || (j > u0);
            bool v1 = u1 >= 0 && ((r < b) || (j > u1));
            if (!whole) {
                const uint64_t i0 = base0 + (uint64_t)j, i1 = base1 + (uint64_t)j;
                v0 = v0 && i0 >= idx_begin && i0 < idx_end;
                v1 = v1 && i1 >= idx_begin && i1 < idx_end;
            }
            if (v0 && edge_passes(E, s0, LA, lb)) edge_offer(pool, pb, E, (int32_t)u0, (int32_t)j, s0);
            if (v1 && edge_passes(E, s1, LA, lb)) edge_offer(pool, pb, E, (int32_t)u1, (int32_t)j, s1);
        };
        const uint8_t *wbase = V.bsym + (J0 + lane_base) * kWordBytes;
        auto word_at = [&](int c) { return wbase + (int64_t)min(c, CPL - 1) * kThreads * kWordBytes; };
        uint32_t bwA[kWordBytes / 4], bwB[kWordBytes / 4];
        load_word(bwA, word_at(0));
        for (int c = 0; c < CPL; c += 2) {
            load_word(bwB, word_at(c + 1));
            column(bwA, c);
            if (c + 1 >= CPL) break;
            load_word(bwA, word_at(c + 2));
            column(bwB, c + 1);
        }
    }
    __syncthreads();
    for (int bsel = 0; bsel < 2; ++bsel) {
        const uint32_t left = pool.n[bsel];
        if (left) edge_flush(pool, bsel, E, left, &flush_base);
    }
}

}  // namespace nw
