// k_inst.hip -- instantiates the tiled kernels (triangle, query, top-k) for
// row lengths LA in [NW_LA_LO, NW_LA_HI]; compiled once per range so the
// instances build in parallel.  Exports their addresses through
// nw_fill_<NW_LA_LO>.
#include <utility>

#include "k_batch.h"
#include "k_edges.h"
#include "k_probe.h"
#include "k_query.h"
#include "k_topk.h"
#include "k_topk_code.h"
#include "k_tri_code.h"
#include "k_tri_tiled.h"
#include "nw_kernels.h"

#define NW_CAT2(a, b) a##b
#define NW_CAT(a, b) NW_CAT2(a, b)

namespace nw {

template <int LA>
static const void *tri_code2_kernel()
{
    if constexpr (LA >= 1 && LA <= kTopkPairMaxLA)
        return reinterpret_cast<const void *>(&k_tri_code<LA, 2>);
    else
        return nullptr;
}

template <int LO, int... Is>
static void fill(KernelTables &t, std::integer_sequence<int, Is...>)
{
    ((t.tri[LO + Is] = reinterpret_cast<const void *>(&k_tri_tiled<LO + Is>)), ...);
    ((t.tri_code1[LO + Is] = reinterpret_cast<const void *>(&k_tri_code<LO + Is, 1>)), ...);
    ((t.tri_code2[LO + Is] = tri_code2_kernel<LO + Is>()), ...);
    ((t.query[LO + Is] = reinterpret_cast<const void *>(&k_query_tiled<LO + Is>)), ...);
    ((t.probe_thr[LO + Is] = reinterpret_cast<const void *>(&k_probe_thr<LO + Is>)), ...);
    ((t.topk[LO + Is] = reinterpret_cast<const void *>(&k_topk_tiled<LO + Is>)), ...);
    ((t.topk_code[LO + Is] = reinterpret_cast<const void *>(&k_topk_code<LO + Is, topk_code_pairs(LO + Is)>)), ...);
    ((t.edges[LO + Is] = reinterpret_cast<const void *>(&k_edges_tiled<LO + Is>)), ...);
    ((t.persist1[LO + Is] = reinterpret_cast<const void *>(&k_tri_persist<LO + Is, LO + Is>)), ...);
}

void NW_CAT(nw_fill_, NW_LA_LO)(KernelTables &t)
{
    fill<NW_LA_LO>(t, std::make_integer_sequence<int, NW_LA_HI - NW_LA_LO + 1>{});
}

}  // namespace nw
