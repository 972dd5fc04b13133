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
__device__ __forceinline__ void tri_tile_dispatch(int la, const DevVocab &V, const BatchItem &I, void *out,
                                                  int out_kind, uint8_t *lds)
{
    if constexpr (L <= HI) {
        if (la == L)
            tri_tile<L>(V, I.r, I.b, I.pbeg, I.pend, 0, ~0ull, out, out_kind, EdgeSink{}, lds);
        else
            tri_tile_dispatch<L + 1, HI>(la, V, I, out, out_kind, lds);
    }
}

template <int LO, int HI>
__global__ __launch_bounds__(kThreads) void k_tri_persist(const DevVocab *vocabs, const BatchItem *items,
                                                          uint32_t nitems, uint32_t *counter, void *const *outs,
                                                          int out_kind)
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
        tri_tile_dispatch<LO, HI>(I.la, V, I, outs[I.vocab], out_kind, lds);
    }
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
