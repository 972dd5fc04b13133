// k_batch_inst.hip -- instantiates the persistent batched kernel and the
// small-dictionary class kernel of one row-length class [NW_CLASS_LO,
// NW_CLASS_HI] (width-8 classes), one class per translation unit so they
// build in parallel.  Exports them through nw_fill_class_<NW_CLASS_LO>.
#include "k_batch.h"
#include "nw_kernels.h"

#define NW_CAT2(a, b) a##b
#define NW_CAT(a, b) NW_CAT2(a, b)

namespace nw {

void NW_CAT(nw_fill_class_, NW_CLASS_LO)(KernelTables &t)
{
    t.persist8[NW_CLASS_LO / 8] = reinterpret_cast<const void *>(&k_tri_persist<NW_CLASS_LO, NW_CLASS_HI>);
    t.class8[NW_CLASS_LO / 8] = reinterpret_cast<const void *>(&k_tri_class<NW_CLASS_LO, NW_CLASS_HI>);
}

}  // namespace nw
