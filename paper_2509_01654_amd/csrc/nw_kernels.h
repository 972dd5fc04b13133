// nw_kernels.h -- the per-length kernel instances, compiled in separate
// translation units (k_inst.hip) and collected into one table.
#pragma once

#include "nw_internal.h"

namespace nw {

// Row-length ranges compiled in separate translation units (build time).
#define NW_LA_SPLITS X(0, 14) X(15, 22) X(23, 29) X(30, 35) X(36, 40) X(41, 44) X(45, 48)

struct KernelTables {
    const void *tri[kMaxLen + 1];
    const void *query[kMaxLen + 1];
    const void *topk[kMaxLen + 1];
};

#define X(lo, hi) void nw_fill_##lo(KernelTables &t);
NW_LA_SPLITS
#undef X

const KernelTables &kernel_tables();

}  // namespace nw
