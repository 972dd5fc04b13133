// k_query.h -- per-row top-k of a set of row words against a column set.
//
// Used for served queries (rows = query words, columns = the dictionary) and
// for the threshold pre-pass of the all-pairs top-k (rows = every dictionary
// word, columns = the probe subset).  A neighbour list is the first k of
// {(score(q, d), d)} sorted by (score descending, index ascending); there is
// no self-exclusion here (the all-pairs path accounts for it).
//
// k_query_tiled<LA>: a workgroup takes `rpw` row pairs of length LA (the two
// words of a pair fill the two binary16 halves of the DP) and one split of the
// column slots.  Per row pair it builds the LDS profile, then each wavefront
// walks its share of the split (64 length-sorted column words per step) and
// keeps a sorted wave list of the best k keys for each of the two rows.  Each
// wave writes its two lists to `partial`, row-major [row][split*4 + wave][k].
//
// k_merge_lists: one wavefront per row merges its P partial lists into the
// final top-k (and optionally reports the key of a given rank).
#pragma once

#include "nw_tile_common.h"
#include "nw_topk.h"

namespace nw {

struct QueryArgs {
    RowSet R;
    ColSet C;
    const uint16_t *wtab;
    int alphabet;
    int gap;
    int lo;                 // lower score bound (key origin)
    int k;                  // list length, 1..64
    int rpw;                // row pairs per workgroup
    int64_t per;            // column slots per split (multiple of 256)
    int nsplit;
    uint64_t *partial;      // [rows][nsplit*4][k]
};

__host__ __device__ constexpr uint32_t query_lds_bytes(int LA, int alphabet) { return 2u * profile_bytes(LA, alphabet); }

template <int LA>
__global__ __launch_bounds__(kThreads) void k_query_tiled(QueryArgs Q)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t off0 = Q.R.off[LA], off1 = Q.R.off[LA + 1];
    const uint32_t pbeg = off0 + blockIdx.x * (uint32_t)Q.rpw;
    if (pbeg >= off1) return;
    const uint32_t pend = min(pbeg + (uint32_t)Q.rpw, off1);
    const int split = blockIdx.y;
    const int64_t c0 = (int64_t)split * Q.per;
    const int64_t c1 = min(c0 + Q.per, Q.C.nslots);

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint32_t prof_bytes = profile_bytes(LA, Q.alphabet);
    const ProfileRole role = profile_role(tid, Q.alphabet);
    const int P = Q.nsplit * 4;

    for (uint32_t p = pbeg; p < pend; ++p) {
        const int32_t a0 = Q.R.pairs[2 * p], a1 = Q.R.pairs[2 * p + 1];
        const uint8_t *prof = lds + (p & 1) * prof_bytes;
        build_profile<LA>(Q.wtab, Q.alphabet, reinterpret_cast<uint32_t *>(lds + (p & 1) * prof_bytes),
                          Q.R.sym + (int64_t)a0 * kWordBytes, Q.R.sym + (int64_t)(a1 >= 0 ? a1 : a0) * kWordBytes,
                          role);
        __syncthreads();
        uint64_t list0 = 0, list1 = 0, thr0 = 0, thr1 = 0;
        for (int64_t base = c0 + wave * 64; base < c1; base += kThreads) {
            const int64_t slot = base + lane;
            const int lb = Q.C.len[slot];
            const int lbmax_w = __builtin_amdgcn_readlane(lb, 63);
            const int32_t d = Q.C.orig[slot];
            int s0, s1;
            pair_scores<LA>(Q.C.sym + slot * kWordBytes, lb, lbmax_w, prof, Q.gap, s0, s1);
            const uint64_t key0 = d >= 0 ? nb_key(s0, Q.lo, (uint32_t)d) : 0;
            const uint64_t key1 = d >= 0 ? nb_key(s1, Q.lo, (uint32_t)d) : 0;
            wl_offer(list0, thr0, key0, Q.k, lane);
            if (a1 >= 0) wl_offer(list1, thr1, key1, Q.k, lane);
        }
        if (lane < Q.k) {
            const int32_t r0 = Q.R.orig[a0];
            Q.partial[((int64_t)r0 * P + split * 4 + wave) * Q.k + lane] = list0;
            if (a1 >= 0) {
                const int32_t r1 = Q.R.orig[a1];
                Q.partial[((int64_t)r1 * P + split * 4 + wave) * Q.k + lane] = list1;
            }
        }
    }
}

#ifdef NW_LAUNCH_TU   // non-template kernels: compiled in the launcher unit only
// One wavefront per row: merge P sorted lists of kin keys into the top kout.
// Writes scores/indices (padding INT16_MIN / -1) when score != NULL and the
// key of rank `rank` (0 when the list is shorter) to thr when thr != NULL.
__global__ __launch_bounds__(256) void k_merge_lists(const uint64_t *partial, int P, int kin, int64_t rows, int kout,
                                                     int lo, int16_t *score, int32_t *index, uint64_t *thr, int rank)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= rows) return;
    const uint64_t *src = partial + row * (int64_t)P * kin;
    const int total = P * kin;
    uint64_t list = 0, t = 0;
    for (int base = 0; base < total; base += 64) {
        const int i = base + lane;
        const uint64_t key = i < total ? src[i] : 0;
        wl_offer(list, t, key, kout, lane);
    }
    if (score != nullptr && lane < kout) {
        score[row * kout + lane] = list ? (int16_t)key_score(list, lo) : (int16_t)-32768;
        index[row * kout + lane] = list ? key_index(list) : -1;
    }
    if (thr != nullptr) {
        const uint64_t v = readlane64(list, rank - 1);
        if (lane == 0) thr[row] = v;
    }
}

#endif

}  // namespace nw
