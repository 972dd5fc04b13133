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

// The block pair of tile t.  rbn == 0: column-major over all pairs
// r <= b (decode_block_pair).  rbn > 0: row-major over block rows rb0 ..
// rb0+rbn-1 and every column block, grid rbn*nb; returns false for b < r
// (no such tile).  The window keeps launches for a narrow pair-index range
// from spanning the whole triangle.
__device__ __forceinline__ bool tile_block_pair(uint32_t t, uint32_t rb0, uint32_t rbn, int nb, uint32_t &r, uint32_t &b)
{
    if (rbn == 0) {
        decode_block_pair(t, r, b);
        return true;
    }
    r = rb0 + t / (uint32_t)nb;
    b = t % (uint32_t)nb;
    return b >= r;
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

// Two-pair profile: row c holds the first pair's LA dwords (padded to whole
// 16-byte units), then the second pair's, then one spare unit, so rows are an
// odd number of 16-byte units apart as in the one-pair layout.
__host__ __device__ constexpr uint32_t profile2_stride_dw(int LA) { return (uint32_t)(((LA + 3) / 4) * 8 + 4); }
__host__ __device__ constexpr uint32_t profile2_off_b(int LA) { return (uint32_t)((LA + 3) / 4) * 16u; }
__host__ __device__ constexpr uint32_t profile2_bytes(int LA, int alphabet)
{
    return LA == 0 ? 0u : (uint32_t)(alphabet + 1) * profile2_stride_dw(LA) * 4u;
}

// Build the two-pair profile of row pairs (su, su2) and (sv, sv2).
template <int LA>
__device__ __forceinline__ void build_profile2(const uint16_t *wtab, int A, uint32_t *prof, const uint8_t *su,
                                               const uint8_t *su2, const uint8_t *sv, const uint8_t *sv2,
                                               const ProfileRole &role)
{
    constexpr uint32_t S = profile2_stride_dw(LA);
    constexpr uint32_t OB = profile2_off_b(LA) / 4;
    const int c = role.c;
    if (c < 0) return;
    if (c == A) {
        for (int i = role.i0; i < 2 * LA; i += role.G) prof[c * S + (i < LA ? i : OB + i - LA)] = kSentinelPair;
        return;
    }
    for (int i = role.i0; i < 2 * LA; i += role.G) {
        const bool second = i >= LA;
        const int p = second ? i - LA : i;
        const uint32_t lo = wtab[(int)(second ? sv : su)[p] * A + c];
        const uint32_t hi = wtab[(int)(second ? sv2 : su2)[p] * A + c];
        prof[c * S + (second ? OB + p : p)] = lo | (hi << 16);
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

// Does the pair with raw score s and word lengths la, lb pass the slice of E?
__device__ __forceinline__ bool edge_passes(const EdgeSink &E, int s, int la, int lb)
{
    if (!E.normalised) return s >= E.lo && s <= E.hi;
    const int64_t m = max(max(la, lb), 1);
    const int64_t w = 100ll * (int64_t)s * (int64_t)E.den;
    return w >= (int64_t)E.lo * m && w <= (int64_t)E.hi * m;
}

// Store the staged scores of row word u (caller index, length la) against
// the columns jstart .. J1-1, srow[t] = score(u, jstart + t), restricted to
// pair indices in [idx_begin, idx_end): as triangle entries out[idx -
// idx_begin] (int8 / int16), or as edges into E (OUT_EDGES).  Edges take one
// atomic per wavefront and row that has any: the wavefront counts its passing
// pairs with ballots, reserves that many slots, then writes them in the same
// order.  Every thread of the workgroup (NT threads) calls this with the same
// arguments.
template <int NT = kThreads>
__device__ __forceinline__ void store_row(const DevVocab &V, int64_t u, int la, int64_t jstart, int64_t J1,
                                          const int16_t *srow, uint64_t idx_begin, uint64_t idx_end, void *out,
                                          int out_kind, const EdgeSink &E)
{
    const uint64_t base = row_start_idx(V.n, u) + (uint64_t)(jstart - u - 1);
    const int64_t len = J1 - jstart;
    const int tid = threadIdx.x;
    if (out_kind != OUT_EDGES) {
        for (int64_t t = tid; t < len; t += NT) {
            const uint64_t idx = base + (uint64_t)t;
            if (idx >= idx_begin && idx < idx_end) {
                const int16_t s = srow[t];
                if (out_kind == OUT_I8)
                    static_cast<int8_t *>(out)[idx - idx_begin] = (int8_t)s;
                else
                    static_cast<int16_t *>(out)[idx - idx_begin] = s;
            }
        }
        return;
    }
    const int wave = tid >> 6, lane = tid & 63;
    auto passes = [&](int64_t t) {
        if (t >= len) return false;
        const uint64_t idx = base + (uint64_t)t;
        return idx >= idx_begin && idx < idx_end && edge_passes(E, srow[t], la, V.clen[jstart + t]);
    };
    // the trip count is uniform over the wavefront, so every ballot sees all 64 lanes
    uint32_t cnt = 0;
    for (int64_t t0 = (int64_t)wave * 64; t0 < len; t0 += NT) cnt += (uint32_t)__popcll(__ballot(passes(t0 + lane)));
    if (cnt == 0) return;
    uint32_t plo = 0, phi = 0;
    if (lane == 0) {
        const unsigned long long p = atomicAdd(E.count, (unsigned long long)cnt);
        plo = (uint32_t)p;
        phi = (uint32_t)(p >> 32);
    }
    uint64_t pos = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)plo) |
                   ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)phi) << 32);
    for (int64_t t0 = (int64_t)wave * 64; t0 < len; t0 += NT) {
        const int64_t t = t0 + lane;
        const bool p = passes(t);
        const uint64_t m = __ballot(p);
        if (p) {
            const uint64_t q = pos + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (q < E.cap) {
                E.ei[q] = (int32_t)u;
                E.ej[q] = (int32_t)(jstart + t);
                E.es[q] = srow[t];
            }
        }
        pos += (uint64_t)__popcll(m);
    }
}

}  // namespace nw
