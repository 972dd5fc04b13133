// nw_kernels.h -- the per-length kernel instances, compiled in separate
// translation units (k_inst.hip) and collected into one table.
#pragma once

#include "nw_internal.h"

namespace nw {

// Row-length ranges compiled in separate translation units (build time).
#define NW_LA_SPLITS X(0, 14) X(15, 22) X(23, 29) X(30, 35) X(36, 40) X(41, 44) X(45, 48)

// Row-length classes of the width-8 persistent batched kernels.
#define NW_CLASS8 X(0, 7) X(8, 15) X(16, 23) X(24, 31) X(32, 39) X(40, 47) X(48, 48)
constexpr int kNumClass8 = 7;

struct KernelTables {
    const void *tri[kMaxLen + 1];
    const void *tri_code1[kMaxLen + 1];  // the same with score codes and dword stores, one row pair a step
    const void *tri_code2[kMaxLen + 1];  // two row pairs a step (rows 1 .. 16; else NULL)
    const void *query[kMaxLen + 1];
    const void *probe_thr[kMaxLen + 1];  // threshold pre-pass by selection
    const void *topk[kMaxLen + 1];
    const void *topk_code[kMaxLen + 1];  // the same with the score-code epilogue
    const void *edges[kMaxLen + 1];      // threshold edge emitter
    const void *persist1[kMaxLen + 1];   // persistent batched kernel, one per row length
    const void *persist8[kNumClass8];    // persistent batched kernel, one per class of 8 lengths
    const void *class8[kNumClass8];      // small-dictionary triangle kernel, one per class of 8 lengths
};

#define X(lo, hi) void nw_fill_##lo(KernelTables &t);
NW_LA_SPLITS
#undef X
#define X(lo, hi) void nw_fill_class_##lo(KernelTables &t);
NW_CLASS8
#undef X

const KernelTables &kernel_tables();

}  // namespace nw
