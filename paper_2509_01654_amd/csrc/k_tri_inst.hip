// k_tri_inst.hip -- instantiates k_tri_tiled<LA> for LA in
// [NW_LA_LO, NW_LA_HI]; compiled once per range so the instances build in
// parallel.  Exports the kernel addresses through nw_tri_fill_<NW_LA_LO>.
#include <utility>

#include "k_tri_tiled.h"

#define NW_CAT2(a, b) a##b
#define NW_CAT(a, b) NW_CAT2(a, b)

namespace nw {

template <int LO, int... Is>
static void fill(tri_kernel_t *tab, std::integer_sequence<int, Is...>)
{
    ((tab[LO + Is] = reinterpret_cast<tri_kernel_t>(&k_tri_tiled<LO + Is>)), ...);
}

void NW_CAT(nw_tri_fill_, NW_LA_LO)(tri_kernel_t *tab)
{
    fill<NW_LA_LO>(tab, std::make_integer_sequence<int, NW_LA_HI - NW_LA_LO + 1>{});
}

}  // namespace nw
