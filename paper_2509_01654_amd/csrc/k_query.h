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
// keeps a sorted wave list of the best k keys for each of the two rows.  With
// several splits the four wave lists of a row are merged in LDS (wavefront 0
// for the first row, 1 for the second) into the split's list, written to
// `partial`, row-major [row][split][k]; with one split (many rows, nothing to
// spread) the four wave lists go out as they are, [row][wave][k].  Either
// way a row has query_lists(nsplit) lists of k keys.
//
// k_merge_lists: one wavefront per row merges its P partial lists into the
// final top-k (and optionally reports the key of a given rank);
// k_merge_lists_wg does the same with a workgroup per row, for rows with many
// partial keys (a few queries spread over many splits).
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
    uint64_t *partial;      // [rows][nsplit][k]
};

// LDS: two profiles, then the wave lists of both rows of a pair (2 x 4 x k keys).
__host__ __device__ constexpr uint32_t query_lds_bytes(int LA, int alphabet, int k)
{
    return 2u * profile_bytes(LA, alphabet) + 2u * 4u * 8u * (uint32_t)k;
}

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
    uint64_t *wl = reinterpret_cast<uint64_t *>(lds + 2 * prof_bytes);   // [2 rows][4 waves][k]

    for (uint32_t p = pbeg; p < pend; ++p) {
        const int32_t a0 = Q.R.pairs[2 * p], a1 = Q.R.pairs[2 * p + 1];
        const uint8_t *prof = lds + (p & 1) * prof_bytes;
        build_profile<LA>(Q.wtab, Q.alphabet, reinterpret_cast<uint32_t *>(lds + (p & 1) * prof_bytes),
                          Q.R.sym + (int64_t)a0 * kWordBytes, Q.R.sym + (int64_t)(a1 >= 0 ? a1 : a0) * kWordBytes,
                          role);
        __syncthreads();
        uint64_t list0 = 0, list1 = 0, thr0 = 0, thr1 = 0;
        // the next step's column word is loaded while this step's DP and
        // list offers run (a split is a few steps, so load latency would
        // otherwise dominate a lightly loaded GPU)
        int64_t base = c0 + wave * 64;
        int lb_n = 0;
        int32_t d_n = -1;
        uint32_t bw_n[kWordBytes / 4];
        if (base < c1) {
            lb_n = Q.C.len[base + lane];
            d_n = Q.C.orig[base + lane];
            load_word(bw_n, Q.C.sym + (base + lane) * kWordBytes);
        }
        for (; base < c1; base += kThreads) {
            const int lb = lb_n;
            const int32_t d = d_n;
            uint32_t bw[kWordBytes / 4];
#pragma unroll
            for (int q = 0; q < kWordBytes / 4; ++q) bw[q] = bw_n[q];
            const int64_t nx = base + kThreads + lane;
            if (base + kThreads < c1) {
                lb_n = Q.C.len[nx];
                d_n = Q.C.orig[nx];
                load_word(bw_n, Q.C.sym + nx * kWordBytes);
            }
            const int lbmax_w = __builtin_amdgcn_readlane(lb, 63);
            int s0, s1;
            pair_scores_regs<LA>(bw, lb, lbmax_w, prof, Q.gap, s0, s1);
            const uint64_t key0 = d >= 0 ? nb_key(s0, Q.lo, (uint32_t)d) : 0;
            const uint64_t key1 = d >= 0 ? nb_key(s1, Q.lo, (uint32_t)d) : 0;
            wl_offer(list0, thr0, key0, Q.k, lane);
            if (a1 >= 0) wl_offer(list1, thr1, key1, Q.k, lane);
        }
        if (Q.nsplit == 1) {   // uniform: the wave lists are the row's partial lists
            if (lane < Q.k) {
                Q.partial[((int64_t)Q.R.orig[a0] * 4 + wave) * Q.k + lane] = list0;
                if (a1 >= 0) Q.partial[((int64_t)Q.R.orig[a1] * 4 + wave) * Q.k + lane] = list1;
            }
            continue;
        }
        if (lane < Q.k) {
            wl[(0 * 4 + wave) * Q.k + lane] = list0;
            wl[(1 * 4 + wave) * Q.k + lane] = list1;
        }
        __syncthreads();
        // wavefront h merges the four wave lists of row h of the pair
        if (wave < 2 && (wave == 0 || a1 >= 0)) {
            const uint64_t *src = wl + wave * 4 * Q.k;
            uint64_t list = 0, t = 0;
            for (int base = 0; base < 4 * Q.k; base += 64) {
                const int i = base + lane;
                wl_offer(list, t, i < 4 * Q.k ? src[i] : 0, Q.k, lane);
            }
            const int32_t row = Q.R.orig[wave == 0 ? a0 : a1];
            if (lane < Q.k) Q.partial[((int64_t)row * Q.nsplit + split) * Q.k + lane] = list;
        }
        __syncthreads();   // the wave lists are rewritten by the next row pair
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
    offer_range(list, t, src, 0, total, kout, lane);
    if (score != nullptr && lane < kout) {
        score[row * kout + lane] = list ? (int16_t)key_score(list, lo) : (int16_t)-32768;
        index[row * kout + lane] = list ? key_index(list) : -1;
    }
    if (thr != nullptr) {
        const uint64_t v = readlane64(list, rank - 1);
        if (lane == 0) thr[row] = v;
    }
}

// The same with one workgroup per row: wavefront w merges the w-th quarter of
// the row's P * kin keys, then wavefront 0 merges the four lists (LDS).
__global__ __launch_bounds__(256) void k_merge_lists_wg(const uint64_t *partial, int P, int kin, int64_t rows, int kout,
                                                        int lo, int16_t *score, int32_t *index, uint64_t *thr, int rank)
{
    __shared__ uint64_t quarter[4 * 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row = blockIdx.x;
    if (row >= rows) return;   // uniform over the workgroup
    const uint64_t *src = partial + row * (int64_t)P * kin;
    const int total = P * kin;
    const int per = (total + 3) / 4;
    const int b0 = min(total, wave * per), b1 = min(total, b0 + per);
    uint64_t list = 0, t = 0;
    offer_range(list, t, src, b0, b1, kout, lane);
    if (lane < kout) quarter[wave * kout + lane] = list;
    __syncthreads();
    if (wave != 0) return;
    uint64_t fin = 0, tf = 0;
    for (int base = 0; base < 4 * kout; base += 64) {
        const int i = base + lane;
        wl_offer(fin, tf, i < 4 * kout ? quarter[i] : 0, kout, lane);
    }
    if (score != nullptr && lane < kout) {
        score[row * kout + lane] = fin ? (int16_t)key_score(fin, lo) : (int16_t)-32768;
        index[row * kout + lane] = fin ? key_index(fin) : -1;
    }
    if (thr != nullptr) {
        const uint64_t v = readlane64(fin, rank - 1);
        if (lane == 0) thr[row] = v;
    }
}

#endif

}  // namespace nw
