// nw_tile_common.h -- pieces shared by the tiled kernels: the row-major pair
// index, block-pair decoding, the LDS similarity profile of a row pair, and
// the scores of a row pair against one lane word.
#pragma once

#include "nw_dp.h"
#include "nw_internal.h"

namespace nw {

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

// Dwords per profile row: LA rounded up to whole 16-byte reads, then to an
// odd number of 16-byte units.  Lanes read the rows of different symbols at
// the same offset in one ds_read_b128; with an odd row stride two rows share
// an LDS bank group only when their symbols are congruent modulo the number
// of bank groups, while an even stride makes many more rows collide.
__host__ __device__ constexpr uint32_t profile_stride_dw_rt(int LA)
{
    return (uint32_t)((((LA + 3) / 4) | 1) * 4);
}
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

// The profile row/positions a thread fills: rows c = tid mod (A+1) for the
// first G*(A+1) threads, positions i0, i0+G, ... (G = threads / (A+1)).
struct ProfileRole {
    int c, i0, G;
};
__device__ __forceinline__ ProfileRole profile_role(int tid, int alphabet)
{
    const int rows = alphabet + 1;
    ProfileRole r;
    r.G = kThreads / rows;
    r.i0 = tid / rows;
    r.c = r.i0 < r.G ? tid % rows : -1;
    return r;
}

// Build the profile of the row pair (slot_u, slot_u2) into prof (LDS): rows
// c = 0 .. alphabet-1 hold (w(u_i, c), w(u'_i, c)); row `alphabet` is the
// sentinel row (-2048, -2048) read past the end of a lane word.
// Thread (c, i0) fills dwords i = i0, i0+G, ... of row c.
template <int LA>
__device__ __forceinline__ void build_profile(const uint16_t *wtab, int A, uint32_t *prof, const uint8_t *su,
                                              const uint8_t *su2, const ProfileRole &role)
{
    constexpr uint32_t S = profile_stride_dw<LA>();
    const int c = role.c;
    if (c < 0) return;
    if (c == A) {
        for (int i = role.i0; i < LA; i += role.G) prof[c * S + i] = kSentinelPair;
        return;
    }
    for (int i = role.i0; i < LA; i += role.G) {
        const uint32_t lo = wtab[(int)su[i] * A + c];
        const uint32_t hi = wtab[(int)su2[i] * A + c];
        prof[c * S + i] = lo | (hi << 16);
    }
}

// The symbols of a padded word as 32-bit registers.
__device__ __forceinline__ void load_word(uint32_t (&bw)[kWordBytes / 4], const uint8_t *p)
{
    const u32x4 *src = reinterpret_cast<const u32x4 *>(p);
#pragma unroll
    for (int q = 0; q < kWordBytes / 16; ++q) {
        const u32x4 x = src[q];
        bw[4 * q + 0] = x[0];
        bw[4 * q + 1] = x[1];
        bw[4 * q + 2] = x[2];
        bw[4 * q + 3] = x[3];
    }
}

// Scores of the two row words (u, u') against a lane word already in registers.
template <int LA>
__device__ __forceinline__ void pair_scores_regs(const uint32_t (&bw)[kWordBytes / 4], int lb, int lbmax_w,
                                                 const uint8_t *prof, int gap, int &s0, int &s1)
{
    if constexpr (LA == 0) {
        s0 = s1 = gap * lb;
    } else {
        const h2 g = dp_lane<LA, kWordBytes>(bw, lbmax_w, prof, profile_stride_dw<LA>() * 4u);
        const int off = gap * (LA + lb);
        s0 = (int)g[0] + off;
        s1 = (int)g[1] + off;
    }
}

// Scores of the two row words (u, u') against the lane word of length lb:
// the DP of nw_dp.h plus the change of variables back to Algorithm 1.
template <int LA>
__device__ __forceinline__ void pair_scores(const uint8_t *lane_word, int lb, int lbmax_w, const uint8_t *prof,
                                            int gap, int &s0, int &s1)
{
    if constexpr (LA == 0) {
        s0 = s1 = gap * lb;
    } else {
        uint32_t bw[kWordBytes / 4];
        load_word(bw, lane_word);
        const h2 g = dp_lane<LA, kWordBytes>(bw, lbmax_w, prof, profile_stride_dw<LA>() * 4u);
        const int off = gap * (LA + lb);
        s0 = (int)g[0] + off;
        s1 = (int)g[1] + off;
    }
}

}  // namespace nw
