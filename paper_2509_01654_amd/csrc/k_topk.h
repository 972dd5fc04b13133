// k_topk.h -- fused all-pairs top-k neighbour lists and score histogram.
//
// Every unordered pair {u, j} is scored once (block pairs (r, b), r <= b, as
// in the triangle kernel) and offered to both endpoints: j to u's list and u
// to j's list.  Each word w carries a threshold key thr[w] that is a lower
// bound of its true k-th best key (the pre-pass computes it from the probe
// subset), so only keys >= thr[w] can belong to w's answer; those are
// appended to w's candidate list (cnt[w] counts every append, including any
// past the capacity, so an overflow is detected).  The histogram counts every
// unordered pair once, per integer score, in LDS and then globally.
//
// k_select: one wavefront per word keeps the best k of its candidates with a
// wave list and writes the final (score, index) list; words whose candidate
// count exceeded the capacity are reported for an exact recomputation.
#pragma once

#include "nw_tile_common.h"
#include "nw_topk.h"

namespace nw {

struct TopkArgs {
    uint64_t *thr;              // [n] threshold keys
    uint32_t *cnt;              // [n] candidate counters (zeroed)
    uint64_t *lists;            // [n][cap]
    uint32_t cap;
    unsigned long long *hist;   // [nbins] or NULL
    int lo;                     // lowest score (key and bin origin)
    int nbins;
    int hist_in_lds;            // 1: per-workgroup LDS histogram copies; 0: global atomics
    int wt_in_lds;              // score-code kernel: 1 stages the similarity table in LDS
    // block pairs of this launch: (b - r) mod phase_mod in [phase_lo, phase_hi]
    int phase_mod, phase_lo, phase_hi;
};

// The LDS histogram is kept in kHistCopies copies (copy = lane mod
// kHistCopies) so that lanes adding to the same popular bin in one
// instruction mostly hit different addresses; the copies are summed at the end.
#ifndef NW_TOPK_OCC6_MAX_LA
#define NW_TOPK_OCC6_MAX_LA 10
#endif
constexpr int kHistCopies = 16;
constexpr int kLdsHistMax = 1024;

__host__ __device__ constexpr uint32_t hist_stride(int nbins) { return (uint32_t)(nbins | 1); }
__host__ __device__ constexpr uint32_t topk_hist_bytes(int nbins, int in_lds)
{
    return in_lds ? 4u * kHistCopies * hist_stride(nbins) : 0u;
}
// Candidates are first appended to one of two LDS pools (by row-pair parity)
// and moved to the global lists between row pairs, many at a time, so the DP
// loop never waits on a global atomic.  A pool that is full sends further
// candidates straight to the global lists.
constexpr int kPool = 96;          // entries per pool
constexpr int kPoolFlush = 48;     // a pool is flushed once it holds this many

// LDS: two profile buffers, the histogram copies, the column block's per-slot
// metadata (length, column, threshold score; 8 bytes per slot), and the two
// candidate pools (keys, words, counters).
__host__ __device__ constexpr uint32_t topk_pool_bytes() { return 2u * kPool * 12u + 16u; }
__host__ __device__ constexpr uint32_t topk_lds_bytes(int LA, int alphabet, int nbins, int hist_in_lds, int CB)
{
    return 2u * profile_bytes(LA, alphabet) + topk_hist_bytes(nbins, hist_in_lds) + 8u * (uint32_t)CB +
           topk_pool_bytes();
}

__device__ __forceinline__ void emit_candidate(const TopkArgs &T, int64_t w, uint64_t key)
{
    const uint32_t p = atomicAdd(&T.cnt[w], 1u);
    if (p < T.cap) T.lists[w * (int64_t)T.cap + p] = key;
}

// The LDS candidate pools of one workgroup.
struct CandPool {
    uint64_t *key;    // [2][kPool]
    int32_t *word;    // [2][kPool]
    uint32_t *n;      // [2] appends so far (may pass kPool)
};

// Offer (w, key) through pool b; the key has passed the score test only, the
// full key test against thr[w] happens when it is moved to the global list.
__device__ __forceinline__ void pool_offer(const CandPool &P, int b, const TopkArgs &T, int64_t w, uint64_t key)
{
    const uint32_t p = atomicAdd(&P.n[b], 1u);
    if (p < (uint32_t)kPool) {
        P.key[b * kPool + p] = key;
        P.word[b * kPool + p] = (int32_t)w;
    } else if (key >= T.thr[w]) {
        emit_candidate(T, w, key);
    }
}

// Move pool b to the global lists.  Every thread of the workgroup calls it
// while no thread appends to pool b; ends with a barrier and the pool empty
// (the reset is ordered before later appends by the caller's next barrier).
__device__ __forceinline__ void pool_flush(const CandPool &P, int b, const TopkArgs &T, uint32_t count)
{
    const uint32_t m = min(count, (uint32_t)kPool);
    for (uint32_t i = threadIdx.x; i < m; i += kThreads) {
        const int32_t w = P.word[b * kPool + i];
        const uint64_t key = P.key[b * kPool + i];
        if (key >= T.thr[w]) emit_candidate(T, w, key);
    }
    __syncthreads();
    if (threadIdx.x == 0) P.n[b] = 0;
}

// Waves per SIMD the main pass asks the compiler for: short rows fit six
// waves in registers (the LDS holds six workgroups per CU) once the compiler
// is asked; longer rows keep the compiler's own allocation (a tighter limit
// would spill the DP column).
template <int LA>
constexpr int topk_min_waves() { return LA <= NW_TOPK_OCC6_MAX_LA ? 6 : 1; }

template <int LA>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(topk_min_waves<LA>())))
void k_topk_tiled(DevVocab V, TopkArgs T)
{
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t r, b;
    decode_block_pair(blockIdx.x, r, b);
    const int ph = (int)((b - r) % (uint32_t)T.phase_mod);
    if (ph < T.phase_lo || ph > T.phase_hi) return;
    const uint32_t *rpo = V.rp_off + (size_t)r * (V.lmax + 1) + LA;
    const uint32_t pbeg = rpo[0], pend = rpo[1];
    if (pbeg >= pend) return;

    const int64_t n = V.n, CB = V.CB;
    const int64_t I0 = (int64_t)r * CB;
    const int64_t J0 = (int64_t)b * CB;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint32_t prof_bytes = profile_bytes(LA, V.alphabet);
    const bool lds_hist = T.hist != nullptr && T.hist_in_lds;
    const uint32_t hs = hist_stride(T.nbins);
    uint32_t *hist_all = reinterpret_cast<uint32_t *>(lds + 2 * prof_bytes);
    // this lane's copy, indexed by the score itself (biased by lo)
    uint32_t *hist = hist_all + (lane & (kHistCopies - 1)) * hs - T.lo;
    const int off_a = V.gap * LA;   // score = G + gap * (LA + lb), Section 4 change of variables
    if (lds_hist)
        for (int i = tid; i < kHistCopies * (int)hs; i += kThreads) hist_all[i] = 0;
    // The column block's slots are the same for every row pair: stage their
    // metadata once -- x = column | length << 16, y = score of the column
    // word's threshold (a pair can only enter that word's list at or above it)
    uint2 *meta = reinterpret_cast<uint2 *>(lds + 2 * prof_bytes + topk_hist_bytes(T.nbins, lds_hist));
    CandPool pool;
    {
        uint8_t *pb = lds + 2 * prof_bytes + topk_hist_bytes(T.nbins, lds_hist) + 8u * (uint32_t)CB;
        pool.key = reinterpret_cast<uint64_t *>(pb);
        pool.word = reinterpret_cast<int32_t *>(pb + 2 * kPool * 8);
        pool.n = reinterpret_cast<uint32_t *>(pb + 2 * kPool * 12);
        if (tid < 2) pool.n[tid] = 0;
    }
    for (int i = tid; i < CB; i += kThreads) {
        const int64_t slot = J0 + i;
        const uint32_t col = V.bcol[slot];
        const uint32_t lb = V.blen[slot];
        const int ts = col != 0xFFFF ? key_score(T.thr[J0 + col], T.lo) : 0x7FFFFFFF;
        meta[i] = make_uint2(col | (lb << 16), (uint32_t)ts);
    }
    const ProfileRole role = profile_role(tid, V.alphabet);
    const int CPL = V.CB / kThreads;
    // Column word c of this lane is slot c*256 + wave*64 + lane: each wavefront
    // takes every fourth group of 64 consecutive (length-sorted) slots, so the
    // four wavefronts get the same mix of lengths and reach the per-row-pair
    // barrier together, while each group's lanes still have near-equal lengths.
    const int lane_base = wave * 64 + lane;

    for (uint32_t k = pbeg; k < pend; ++k) {
        const int32_t a0 = V.rpairs[2 * k], a1 = V.rpairs[2 * k + 1];
        const uint8_t *prof = lds + (k & 1) * prof_bytes;
        build_profile<LA>(V.wtab, V.alphabet, reinterpret_cast<uint32_t *>(lds + (k & 1) * prof_bytes),
                          V.bsym + (int64_t)a0 * kWordBytes, V.bsym + (int64_t)(a1 >= 0 ? a1 : a0) * kWordBytes, role);
        __syncthreads();
        // This row pair appends to pool pb; the other pool took the previous
        // row pair's candidates, which every wavefront has finished (barrier
        // above), so its count is the same for all threads.
        const int pb = (int)(k & 1);
        {
            const uint32_t other = pool.n[pb ^ 1];
            if (other >= (uint32_t)kPoolFlush) pool_flush(pool, pb ^ 1, T, other);
        }
        const int64_t u0 = I0 + V.bcol[a0];
        const int64_t u1 = a1 >= 0 ? I0 + V.bcol[a1] : -1;
        const uint64_t thr_u0 = T.thr[u0];
        const uint64_t thr_u1 = u1 >= 0 ? T.thr[u1] : ~0ull;
        // a key >= thr needs score >= the threshold's score: test that first
        const int ts_u0 = key_score(thr_u0, T.lo);
        const int ts_u1 = key_score(thr_u1, T.lo);
        // One column word of this lane: its DP against the row pair, then the
        // histogram and both endpoints' candidate tests.
        auto column = [&](const uint32_t(&bw)[kWordBytes / 4], int c) __attribute__((always_inline)) {
            const uint2 m = meta[lane_base + c * kThreads];
            const int lb = (int)(m.x >> 16);
            const int col = (int)(m.x & 0xFFFF);
            const int ts_j = (int)m.y;
            const int lbmax_w = __builtin_amdgcn_readlane(lb, 63);
            h2 g;
            if constexpr (LA == 0)
                g = h2{0, 0};
            else
                g = dp_lane<LA, kWordBytes>(bw, lbmax_w, prof, profile_stride_dw<LA>() * 4u);
            if (col == 0xFFFF) return;
            const int off = off_a + __mul24(V.gap, lb);
            const int s0 = (int)g[0] + off, s1 = (int)g[1] + off;
            const int64_t j = J0 + col;
            // each unordered pair once: in a diagonal block only j > u
            const bool v0 = (r < b) || (j > u0);
            const bool v1 = u1 >= 0 && ((r < b) || (j > u1));
            if (lds_hist) {
                if (v0) atomicAdd(&hist[s0], 1u);
                if (v1) atomicAdd(&hist[s1], 1u);
            } else if (T.hist) {
                if (v0) atomicAdd(&T.hist[s0 - T.lo], 1ull);
                if (v1) atomicAdd(&T.hist[s1 - T.lo], 1ull);
            }
            // A pair enters a list only at or above the owner's threshold
            // score.  One test covers all four lists; the few lanes that pass
            // it (about one pair in a thousand) take the detailed tests.
            const bool c0 = v0 && s0 >= min(ts_u0, ts_j);
            const bool c1 = v1 && s1 >= min(ts_u1, ts_j);
            if (__builtin_expect(c0 || c1, 0)) {
                if (c0 && s0 >= ts_u0) pool_offer(pool, pb, T, u0, nb_key(s0, T.lo, (uint32_t)j));
                if (c0 && s0 >= ts_j) pool_offer(pool, pb, T, j, nb_key(s0, T.lo, (uint32_t)u0));
                if (c1 && s1 >= ts_u1) pool_offer(pool, pb, T, u1, nb_key(s1, T.lo, (uint32_t)j));
                if (c1 && s1 >= ts_j) pool_offer(pool, pb, T, j, nb_key(s1, T.lo, (uint32_t)u1));
            }
        };
        // Lane words are prefetched one ahead into two alternating register
        // sets (the loop handles two column words per trip), so no word is
        // copied between registers; the fetch past the last word re-reads the
        // last one.
        const uint8_t *wbase = V.bsym + (J0 + lane_base) * kWordBytes;
        auto word_at = [&](int c) { return wbase + (int64_t)min(c, CPL - 1) * kThreads * kWordBytes; };
        uint32_t bwA[kWordBytes / 4], bwB[kWordBytes / 4];
        load_word(bwA, word_at(0));
        for (int c = 0; c < CPL; c += 2) {
            load_word(bwB, word_at(c + 1));
            column(bwA, c);
            if (c + 1 >= CPL) break;
            load_word(bwA, word_at(c + 2));
            column(bwB, c + 1);
        }
    }
    // the candidates still pooled
    __syncthreads();
    for (int b = 0; b < 2; ++b) {
        const uint32_t left = pool.n[b];
        if (left) pool_flush(pool, b, T, left);
    }
    if (lds_hist) {
        __syncthreads();
        for (int i = tid; i < T.nbins; i += kThreads) {
            uint32_t sum = 0;
            for (int c = 0; c < kHistCopies; ++c) sum += hist_all[c * hs + i];
            if (sum) atomicAdd(&T.hist[i], (unsigned long long)sum);
        }
    }
}

#ifdef NW_LAUNCH_TU   // non-template kernels: compiled in the launcher unit only
// One wavefront per word: raise thr[w] to the k-th best key among the
// candidates collected so far (real keys of real partners, so it stays a
// lower bound of the final k-th key).
__global__ __launch_bounds__(256) void k_tighten(const uint32_t *cnt, const uint64_t *lists, uint32_t cap, int64_t n,
                                                 int k, uint64_t *thr)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n) return;
    const uint32_t c = cnt[w];
    const int m = (int)(c < cap ? c : cap);
    if (m < k) return;
    const uint64_t *src = lists + w * (int64_t)cap;
    uint64_t list = 0, t = 0;
    offer_range(list, t, src, 0, m, k, lane);
    const uint64_t kth = readlane64(list, k - 1);
    if (lane == 0 && kth > thr[w]) thr[w] = kth;
}

// One wavefront per word: the best k of its (at most cap) candidates.
// Words with more than cap candidates are appended to ovf_list.
__global__ __launch_bounds__(256) void k_select(const uint32_t *cnt, const uint64_t *lists, uint32_t cap, int64_t n,
                                                int k, int lo, int16_t *score, int32_t *index, uint32_t *ovf_count,
                                                int32_t *ovf_list)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n) return;
    const uint32_t c = cnt[w];
    if (c > cap && lane == 0) {
        const uint32_t p = atomicAdd(ovf_count, 1u);
        ovf_list[p] = (int32_t)w;
    }
    const int m = (int)(c < cap ? c : cap);
    const uint64_t *src = lists + w * (int64_t)cap;
    uint64_t list = 0, t = 0;
    offer_range(list, t, src, 0, m, k, lane);
    if (lane < k) {
        score[w * k + lane] = list ? (int16_t)key_score(list, lo) : (int16_t)-32768;
        index[w * k + lane] = list ? key_index(list) : -1;
    }
}

#endif

}  // namespace nw
