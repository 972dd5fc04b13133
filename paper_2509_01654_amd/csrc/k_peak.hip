// k_peak.hip -- issue-rate microbenchmark of the DP's instruction pair.
//
// A DP cell of the register-row kernels is one packed add and one packed
// three-input max per two cells (nw_dp.h).  k_packed_rate issues exactly that
// pair in eight independent chains per lane, so no instruction waits on the
// one before it, at full occupancy over every CU.  Timed by the caller, the
// launch gives the packed lane-instruction rate the chip sustains at the
// clock it runs during the measurement: the measured counterpart of the
// nominal 256 CUs x 64 lanes x clock, and twice that in 16-bit operations
// (two halves per packed instruction).
#include "nw_host.h"
#include "nw_dp.h"

using namespace nw;
using namespace nw::host;

namespace {

constexpr int kPeakThreads = 256;
constexpr int kPeakChains = 8;    // independent chains per lane
constexpr int kPeakUnroll = 4;    // chain rounds per loop trip

// Each trip issues kPeakUnroll x kPeakChains x 2 packed instructions per lane.
__global__ __launch_bounds__(kPeakThreads) void k_packed_rate(uint32_t trips)
{
    h2 x[kPeakChains], y[kPeakChains];
#pragma unroll
    for (int i = 0; i < kPeakChains; ++i) {
        x[i] = h2{(_Float16)(threadIdx.x & 15), (_Float16)i};
        y[i] = h2{(_Float16)i, (_Float16)(blockIdx.x & 7)};
    }
    const h2 d = h2{(_Float16)-1.0f, (_Float16)-2.0f};
    const h2 z = h2{(_Float16)-8.0f, (_Float16)-8.0f};
    for (uint32_t t = 0; t < trips; ++t) {
#pragma unroll
        for (int u = 0; u < kPeakUnroll; ++u)
#pragma unroll
            for (int i = 0; i < kPeakChains; ++i) x[i] = max3(x[i] + d, y[i], z);
    }
    h2 m = x[0];
#pragma unroll
    for (int i = 1; i < kPeakChains; ++i) m = max3(m, x[i], z);
    // keep the result live (an empty asm that takes it as a VGPR operand), so
    // the compiler cannot drop the chains; nothing is stored
    asm volatile("" ::"v"(__builtin_bit_cast(uint32_t, m)));
}

}  // namespace

extern "C" {

int nw_packed_issue_rate(uint32_t blocks, uint32_t trips, uint64_t *lane_instructions, void *hip_stream)
{
    if (blocks == 0 || trips == 0) return fail(NW_EINVAL, "blocks and trips must be at least 1");
    if (!lane_instructions) return fail(NW_EINVAL, "lane_instructions is NULL");
    hipLaunchKernelGGL(k_packed_rate, dim3(blocks), dim3(kPeakThreads), 0, (hipStream_t)hip_stream, trips);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return dev_fail(e, "launching the packed-rate microbenchmark");
    *lane_instructions = (uint64_t)blocks * kPeakThreads * trips * kPeakUnroll * kPeakChains * 2;
    return ok();
}

}  // extern "C"
