// k_tri_tiled.h -- the tiled all-pairs kernel that writes the row-major upper
// triangle (Section 4.1 of the paper) in the caller's word order.
//
// The caller-order words are cut into blocks of CB words; a workgroup takes
// one block pair (r, b), r <= b, and one exact row length LA.  It walks the
// row pairs (u, u') of block r whose words both have length LA; for each pair
// it builds the similarity profile in LDS, and every lane runs the DP of the
// pair against CB/256 column words of block b (slots sorted by length, so the
// 64 lanes of a wavefront have near-equal column lengths).  Scores land in an
// LDS staging row in caller column order and leave as two contiguous row
// segments out[idx(u, jstart) ..], so the HBM writes are coalesced even though
// the DP ran in length-sorted order.
//
// Pipelining inside the workgroup: one barrier per row pair.  Iteration k
// builds the profile of pair k (double-buffered) and stores the staged scores
// of pair k-2 (triple-buffered), then, after the barrier, runs the DP of pair k.
#pragma once

#include "nw_dp.h"
#include "nw_internal.h"

namespace nw {

// Row-length ranges compiled in separate translation units (build time).
#define NW_TRI_SPLITS X(0, 16) X(17, 24) X(25, 31) X(32, 37) X(38, 43) X(44, 48)

typedef void (*tri_kernel_t)(DevVocab, uint64_t, uint64_t, void *, int);

__device__ __forceinline__ uint64_t row_start_idx(int64_t n, int64_t r)
{
    // S_{r-1} = (n-1) r - (r-1) r / 2 : pairs before row r (Section 4.2)
    return (uint64_t)(n - 1) * (uint64_t)r - ((uint64_t)(r - 1) * (uint64_t)r) / 2u;
}

__device__ __forceinline__ void decode_block_pair(uint32_t t, uint32_t &r, uint32_t &b)
{
    // t enumerates pairs (r, b), 0 <= r <= b, column-major: t = b(b+1)/2 + r
    uint32_t bb = (uint32_t)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((bb + 1) * (bb + 2) / 2 <= t) ++bb;
    while (bb * (bb + 1) / 2 > t) --bb;
    b = bb;
    r = t - bb * (bb + 1) / 2;
}

// Dwords per profile row: LA rounded up to whole 16-byte reads, plus one
// 16-byte pad so consecutive symbol rows start on different LDS banks.
__host__ __device__ constexpr uint32_t profile_stride_dw_rt(int LA) { return (uint32_t)(((LA + 3) / 4) * 4 + 4); }
template <int LA>
__host__ __device__ constexpr uint32_t profile_stride_dw()
{
    return profile_stride_dw_rt(LA);
}
// Bytes of one profile buffer (alphabet rows plus the sentinel row); none for LA = 0.
__host__ __device__ constexpr uint32_t profile_bytes(int LA, int alphabet)
{
    return LA == 0 ? 0u : (uint32_t)(alphabet + 1) * profile_stride_dw_rt(LA) * 4u;
}
// Dynamic LDS of k_tri_tiled: two profile buffers and three int16 staging rows pairs.
__host__ __device__ constexpr uint32_t tri_lds_bytes(int LA, int alphabet, int CB)
{
    return 2u * profile_bytes(LA, alphabet) + 3u * 2u * (uint32_t)CB * 2u;
}

// Build the profile of the row pair (slot_u, slot_u2) into prof (LDS): rows
// c = 0 .. alphabet-1 hold (w(u_i, c), w(u'_i, c)); row `alphabet` is the
// sentinel row (-2048, -2048) read past the end of a lane word.
// Thread (c, i0) fills dwords i = i0, i0+G, ... of row c.
template <int LA>
__device__ __forceinline__ void build_profile(const DevVocab &V, uint32_t *prof, int32_t slot_u, int32_t slot_u2,
                                              int c, int i0, int G)
{
    constexpr uint32_t S = profile_stride_dw<LA>();
    if (c < 0) return;
    const uint8_t *su = V.bsym + (int64_t)slot_u * V.WB;
    const uint8_t *su2 = V.bsym + (int64_t)(slot_u2 >= 0 ? slot_u2 : slot_u) * V.WB;
    const int A = V.alphabet;
    if (c == A) {
        for (int i = i0; i < LA; i += G) prof[c * S + i] = kSentinelPair;
        return;
    }
    for (int i = i0; i < LA; i += G) {
        const uint32_t lo = V.wtab[(int)su[i] * A + c];
        const uint32_t hi = V.wtab[(int)su2[i] * A + c];
        prof[c * S + i] = lo | (hi << 16);
    }
}

template <int LA>
__global__ __launch_bounds__(kThreads) void k_tri_tiled(DevVocab V, uint64_t idx_begin, uint64_t idx_end, void *out,
                                                        int out_kind)
{
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr int WB = kWordBytes;
    constexpr int LBMAX = WB;          // a padded word holds at most WB symbols
    constexpr int NWD = WB / 4;
    constexpr uint32_t S = profile_stride_dw<LA>();

    uint32_t r, b;
    decode_block_pair(blockIdx.x, r, b);
    const uint32_t *rpo = V.rp_off + (size_t)r * (V.lmax + 1) + LA;
    const uint32_t pbeg = rpo[0], pend = rpo[1];
    if (pbeg >= pend) return;

    const int64_t n = V.n, CB = V.CB;
    const int64_t I0 = (int64_t)r * CB, I1 = min(I0 + CB, n);
    const int64_t J0 = (int64_t)b * CB, J1 = min(J0 + CB, n);
    {
        // skip the block pair if none of its pairs falls in [idx_begin, idx_end)
        const int64_t jlo = (r == b) ? I0 + 1 : J0;
        if (jlo >= J1) return;
        const uint64_t first = row_start_idx(n, I0) + (uint64_t)(jlo - I0 - 1);
        const int64_t ilast = (r == b) ? J1 - 2 : I1 - 1;
        const uint64_t last = row_start_idx(n, ilast) + (uint64_t)(J1 - 1 - ilast - 1);
        if (last < idx_begin || first >= idx_end) return;
    }

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint32_t prof_bytes = profile_bytes(LA, V.alphabet);
    int16_t *stg = reinterpret_cast<int16_t *>(lds + 2 * prof_bytes);   // [3][2][CB]

    // profile-build role of this thread
    const int rows = V.alphabet + 1;
    const int G = kThreads / rows;
    const int pc = (tid / rows) < G ? tid % rows : -1;
    const int pi0 = tid / rows;
    const int CPL = V.CB / kThreads;

    for (uint32_t k = pbeg; k < pend + 2; ++k) {
        if (k < pend)
            build_profile<LA>(V, reinterpret_cast<uint32_t *>(lds + (k & 1) * prof_bytes), V.rpairs[2 * k], V.rpairs[2 * k + 1], pc,
                              pi0, G);
        if (k >= pbeg + 2) {
            // store the staged scores of pair k-2 as contiguous row segments
            const uint32_t kk = k - 2;
            const int16_t *srow = stg + (size_t)(kk % 3) * 2 * CB;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int32_t slot = V.rpairs[2 * kk + h];
                if (slot < 0) continue;
                const int64_t u = I0 + V.bcol[slot];
                const int64_t jstart = (r == b) ? u + 1 : J0;
                const uint64_t base = row_start_idx(n, u) + (uint64_t)(jstart - u - 1);
                for (int64_t t = tid; t < J1 - jstart; t += kThreads) {
                    const uint64_t idx = base + (uint64_t)t;
                    if (idx >= idx_begin && idx < idx_end) {
                        const int16_t s = srow[h * CB + (jstart - J0) + t];
                        if (out_kind == OUT_I8)
                            static_cast<int8_t *>(out)[idx - idx_begin] = (int8_t)s;
                        else
                            static_cast<int16_t *>(out)[idx - idx_begin] = s;
                    }
                }
            }
        }
        __syncthreads();
        if (k < pend) {
            const int32_t su = V.rpairs[2 * k];
            const int32_t su2 = V.rpairs[2 * k + 1];
            (void)su;
            int16_t *sdst = stg + (size_t)(k % 3) * 2 * CB;
            for (int c = 0; c < CPL; ++c) {
                const int64_t slot = J0 + (int64_t)(wave * 64 * CPL + c * 64 + lane);
                const int lb = V.blen[slot];
                const int lbmax_w = __builtin_amdgcn_readlane(lb, 63);
                int s0, s1;
                if constexpr (LA == 0) {
                    s0 = s1 = V.gap * lb;
                } else {
                    uint32_t bw[NWD];
                    const u32x4 *src = reinterpret_cast<const u32x4 *>(V.bsym + slot * WB);
#pragma unroll
                    for (int q = 0; q < NWD / 4; ++q) {
                        const u32x4 x = src[q];
                        bw[4 * q + 0] = x[0];
                        bw[4 * q + 1] = x[1];
                        bw[4 * q + 2] = x[2];
                        bw[4 * q + 3] = x[3];
                    }
                    const h2 g = dp_lane<LA, LBMAX>(bw, lbmax_w, lds + (k & 1) * prof_bytes, S * 4u);
                    const int off = V.gap * (LA + lb);
                    s0 = (int)g[0] + off;
                    s1 = (int)g[1] + off;
                }
                const int col = V.bcol[slot];
                if (col != 0xFFFF) {
                    sdst[col] = (int16_t)s0;
                    if (su2 >= 0) sdst[CB + col] = (int16_t)s1;
                }
            }
        }
    }
}

}  // namespace nw
