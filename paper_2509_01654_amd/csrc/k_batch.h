// k_batch.h -- batched persistent triangle kernel: many dictionaries in one
// launch sequence.
//
// The host cuts every dictionary's triangle into work items (dictionary, block
// pair (r, b), row length LA, a chunk of that block's row pairs of length LA),
// estimates each item's DP cells, and orders the items of each row-length
// class heaviest first.  One persistent kernel per class runs a fixed grid;
// each workgroup takes the next item from the class counter (one atomic per
// item) until the queue is empty, and runs the same tile code as the
// per-length triangle kernel (tri_tile<LA>) for the item's exact LA.  Every
// workgroup leaves once the counter has passed the last item, so the grid
// always drains.
#pragma once

#include "k_tri_code.h"
#include "k_tri_tiled.h"

namespace nw {

struct BatchItem {
    uint16_t vocab;     // index into the dictionary array
    uint16_t la;        // row length of the item
    uint32_t r, b;      // block pair, r <= b
    uint32_t pbeg, pend;
};

// Dispatch a runtime row length to the tile instance of a class [L, HI].
template <int L, int HI>
__device__ __forceinline__ void tri_tile_dispatch(int la, const DevVocab &V, uint32_t r, uint32_t b, uint32_t pbeg,
                                                  uint32_t pend, uint64_t idx_begin, uint64_t idx_end, void *out,
                                                  int out_kind, const EdgeSink &E, uint8_t *lds)
{
    if constexpr (L <= HI) {
        if (la == L)
            tri_tile<L>(V, r, b, pbeg, pend, idx_begin, idx_end, out, out_kind, E, lds);
        else
            tri_tile_dispatch<L + 1, HI>(la, V, r, b, pbeg, pend, idx_begin, idx_end, out, out_kind, E, lds);
    }
}

// The same for the score-code tile (tri_tile_code, one row pair a step).
template <int L, int HI>
__device__ __forceinline__ void tri_tile_code_dispatch(int la, const DevVocab &V, uint32_t r, uint32_t b,
                                                       uint32_t pbeg, uint32_t pend, void *out, int es, uint8_t *lds)
{
    if constexpr (L <= HI) {
        if (la == L)
            tri_tile_code<L, 1>(V, r, b, pbeg, pend, 0, ~0ull, out, es, lds);
        else
            tri_tile_code_dispatch<L + 1, HI>(la, V, r, b, pbeg, pend, out, es, lds);
    }
}

// code_es = 1 or 2: every dictionary's scores fit the score-code tile, which
// stores es-byte scores; 0: the plain tile with out_kind.
template <int LO, int HI>
__global__ __launch_bounds__(kThreads) void k_tri_persist(const DevVocab *vocabs, const BatchItem *items,
                                                          uint32_t nitems, uint32_t *counter, void *const *outs,
                                                          int out_kind, int code_es)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t it = s_item;
        __syncthreads();
        if (it >= nitems) break;
        const BatchItem I = items[it];
        const DevVocab V = vocabs[I.vocab];
        if (code_es)
            tri_tile_code_dispatch<LO, HI>(I.la, V, I.r, I.b, I.pbeg, I.pend, outs[I.vocab], code_es, lds);
        else
            tri_tile_dispatch<LO, HI>(I.la, V, I.r, I.b, I.pbeg, I.pend, 0, ~0ull, outs[I.vocab], out_kind,
                                      EdgeSink{}, lds);
    }
}

// The triangle of a small dictionary with one launch per class of row
// lengths [LO, HI] instead of one per length: workgroup (x, y) takes run
// x % chunks (at most rpc row pairs) of tile x / chunks, and row length
// LO + y.  Small dictionaries have little work per length, so the per-length
// launches are bound by their host-side launch cost; this form issues a few
// launches instead.
template <int LO, int HI>
__global__ __launch_bounds__(kThreads) void k_tri_class(DevVocab V, uint64_t idx_begin, uint64_t idx_end, void *out,
                                                        int out_kind, EdgeSink E, uint32_t rb0, uint32_t rbn,
                                                        uint32_t chunks, uint32_t rpc)
{
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t r, b;
    if (!tile_block_pair(blockIdx.x / chunks, rb0, rbn, V.nb, r, b)) return;
    const int la = LO + (int)blockIdx.y;
    if (la > V.lmax) return;
    const uint32_t *rpo = V.rp_off + (size_t)r * (V.lmax + 1) + la;
    const uint64_t pbeg64 = (uint64_t)rpo[0] + (uint64_t)(blockIdx.x % chunks) * rpc;
    if (pbeg64 >= rpo[1]) return;
    const uint32_t pbeg = (uint32_t)pbeg64;
    const uint32_t pend = rpo[1] - pbeg <= rpc ? rpo[1] : pbeg + rpc;
    tri_tile_dispatch<LO, HI>(la, V, r, b, pbeg, pend, idx_begin, idx_end, out, out_kind, E, lds);
}

#ifdef NW_LAUNCH_TU
// Zero the class counters (a kernel rather than a memset node, so a captured
// graph replays it like any other kernel).
__global__ void k_reset_counters(uint32_t *counters, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counters[i] = 0;
}
#endif

}  // namespace nw
