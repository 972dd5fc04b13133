// k_topk_code.h -- main pass of the fused top-k with a score-code epilogue.
//
// The same computation as k_topk_tiled (every unordered pair of the block
// pair scored once by the same DP, offered to both endpoints' candidate lists
// when it reaches their thresholds, counted once in the histogram), with the
// per-pair work after the DP done on binary16 bit patterns:
//
//   Adding K = 1024 - lo + gap (LA + lb) to the DP result G gives the
//   binary16 value 1024 + (s - lo), whose bits are 0x6400 + (s - lo)
//   (binary16 spacing is 1 on [1024, 2048), and every term is an integer of
//   magnitude <= 2048, so the sum is exact).
//
// One packed add therefore turns both pairs' results into score codes, two
// packed 16-bit ops give both histogram addresses, and the threshold tests
// compare codes as 16-bit integers: about 9 vector instructions per column
// word instead of about 21.  It applies when every score code lies in
// [0, 1024) and the histogram fits in LDS below 64 KiB.
//
// A tile takes the short epilogue unless it is a diagonal block pair (only
// pairs j > u count there), holds the padding slots of the last block, or
// the row pair is half empty; those take the general one.
#pragma once

#include "k_topk.h"

namespace nw {

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
typedef int16_t i16x2 __attribute__((ext_vector_type(2)));

// Binary16 bits of 1024 + x for integers 0 <= x < 1024.
constexpr uint32_t kCodeOrigin = 0x6400u;
// A threshold code no score reaches.
constexpr uint32_t kCodeNever = 0x7FFFu;
constexpr int kCodeMaxBins = 256;

// Row pairs per step of k_topk_code<LA, R>: two for the short rows, whose
// per-column address and per-column-word work weigh most; one where the two
// DP columns would not fit beside the other registers.
constexpr int kTopkPairMaxLA = 16;
__host__ __device__ constexpr int topk_code_pairs(int LA) { return LA >= 1 && LA <= kTopkPairMaxLA ? 2 : 1; }
__host__ __device__ constexpr uint32_t topk_code_profile_bytes(int LA, int R, int alphabet)
{
    return R == 2 ? profile2_bytes(LA, alphabet) : profile_bytes(LA, alphabet);
}
// Row pairs staged in LDS at a time (their words' symbols, caller indices and
// threshold codes), so the per-step profile build and threshold reads wait on
// LDS only; the staging itself costs one more barrier per chunk.
constexpr int kChunkPairs = 32;
__host__ __device__ constexpr uint32_t chunk_sym_bytes(int LA) { return (uint32_t)((LA + 3) / 4) * 4u; }
__host__ __device__ constexpr uint32_t chunk_bytes(int LA)
{
    return 2u * kChunkPairs * (chunk_sym_bytes(LA) + 8u);
}
// The similarity table w(x, y) may be staged in LDS for alphabets up to 48
// symbols (4.5 KiB), where the build of the row-pair profiles reads it; the
// launcher stages it only when that costs no workgroup per CU (topk_code_wt_in_lds).
// Otherwise it is read from global memory, where it stays cached.
constexpr int kLdsWtabMaxAlphabet = 48;
__host__ __device__ constexpr uint32_t wtab_lds_bytes(int alphabet, int in_lds)
{
    return in_lds && alphabet <= kLdsWtabMaxAlphabet ? (((uint32_t)alphabet * (uint32_t)alphabet * 2u + 15u) & ~15u)
                                                     : 0u;
}
// LDS of k_topk_code: two profile buffers, the histogram copies, 4 bytes of
// metadata per column slot, the longest length of each group of 64 slots, the
// similarity table, two row-pair chunks and the candidate pools.
__host__ __device__ constexpr uint32_t topk_code_lds_bytes(int LA, int alphabet, int nbins, int has_hist, int CB,
                                                        int wt_in_lds)
{
    return 2u * topk_code_profile_bytes(LA, topk_code_pairs(LA), alphabet) + topk_hist_bytes(nbins, has_hist) +
           4u * (uint32_t)CB + (((uint32_t)CB / 64u + 15u) & ~15u) + wtab_lds_bytes(alphabet, wt_in_lds) +
           2u * chunk_bytes(LA) + topk_pool_bytes();
}

// Does the main pass of this dictionary with these arguments take
// k_topk_code<LA>?  Every score code lies in [0, 1024), and the histogram
// copies (placed after the two profiles) end below 64 KiB.
__host__ __device__ inline bool topk_code_applies(const DevVocab &V, const TopkArgs &T, int LA)
{
    return T.lo <= V.lo && V.hi - T.lo < 1024 && (T.hist == nullptr || T.nbins <= kCodeMaxBins) &&
           2u * topk_code_profile_bytes(LA, topk_code_pairs(LA), V.alphabet) +
                   topk_hist_bytes(T.nbins, T.hist != nullptr) <= 65536u &&
           topk_code_lds_bytes(LA, V.alphabet, T.nbins, T.hist != nullptr, V.CB, 0) <= kMaxLdsBytes;
}

// Stage the similarity table in LDS when the alphabet allows it and the LDS
// of a workgroup then still admits as many workgroups per CU as without it.
__host__ __device__ inline bool topk_code_wt_in_lds(const DevVocab &V, const TopkArgs &T, int LA)
{
    if (V.alphabet > kLdsWtabMaxAlphabet) return false;
    const int h = T.hist != nullptr;
    return kMaxLdsBytes / topk_code_lds_bytes(LA, V.alphabet, T.nbins, h, V.CB, 1) ==
           kMaxLdsBytes / topk_code_lds_bytes(LA, V.alphabet, T.nbins, h, V.CB, 0);
}

// The code of threshold score ts: kCodeOrigin + ts - lo, clamped to [0, kCodeNever].
__device__ __forceinline__ uint32_t threshold_code(int ts, int lo)
{
    const int c = (int)kCodeOrigin + ts - lo;
    return (uint32_t)min(max(c, 0), (int)kCodeNever);
}

// R row pairs per step (1 or 2): with two, the profile holds both pairs
// (build_profile2) and one address per column serves both (dp_lane2), so
// the per-column address, the per-column-word metadata, the barrier and the
// column word loads are shared by twice the cells.
// Waves per SIMD the compiler is asked to fit in registers: as many as the
// LDS of the 40-symbol workload admits (six workgroups per CU up to LA = 8
// with two pairs per step, five up to 12); longer rows keep the compiler's
// own allocation.
template <int LA, int R>
constexpr int topk_code_min_waves()
{
    return R == 1 ? topk_min_waves<LA>() : LA <= 8 ? 6 : LA <= 12 ? 5 : 1;
}

template <int LA, int R>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(topk_code_min_waves<LA, R>())))
void k_topk_code(DevVocab V, TopkArgs T)
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
    const int A = V.alphabet;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint32_t prof_bytes = topk_code_profile_bytes(LA, R, A);
    const bool has_hist = T.hist != nullptr;
    const uint32_t hs = hist_stride(T.nbins);
    const uint32_t lds0 = lds_addr_of(lds);
    const uint32_t hist_off = 2 * prof_bytes;
    uint32_t *hist_all = reinterpret_cast<uint32_t *>(lds + hist_off);
    // this lane's histogram copy: by score (general epilogue), and the
    // address of bin (code - kCodeOrigin) as code * 4 + hb modulo 2^16
    const uint32_t my_hist = hist_off + (uint32_t)(lane & (kHistCopies - 1)) * hs * 4u;
    uint32_t *hist = reinterpret_cast<uint32_t *>(lds + my_hist) - T.lo;
    const uint16_t hb = (uint16_t)(lds0 + my_hist - kCodeOrigin * 4u);
    if (has_hist)
        for (int i = tid; i < kHistCopies * (int)hs; i += kThreads) hist_all[i] = 0;
    // per column slot: K | threshold code << 16 (K = binary16 of 1024 - lo + gap (LA + lb));
    // per group of 64 slots: the longest length (the last slot's: slots are length-sorted)
    const uint32_t meta_off = hist_off + topk_hist_bytes(T.nbins, has_hist);
    uint32_t *meta = reinterpret_cast<uint32_t *>(lds + meta_off);
    uint8_t *gmax = lds + meta_off + 4u * (uint32_t)CB;
    uint16_t *wt_lds = reinterpret_cast<uint16_t *>(gmax + (((uint32_t)CB / 64u + 15u) & ~15u));
    uint8_t *chunks = reinterpret_cast<uint8_t *>(wt_lds) + wtab_lds_bytes(A, T.wt_in_lds);
    constexpr uint32_t SW = chunk_sym_bytes(LA);
    CandPool pool;
    {
        uint8_t *pb = chunks + 2u * chunk_bytes(LA);
        pool.key = reinterpret_cast<uint64_t *>(pb);
        pool.word = reinterpret_cast<int32_t *>(pb + 2 * kPool * 8);
        pool.n = reinterpret_cast<uint32_t *>(pb + 2 * kPool * 12);
        if (tid < 2) pool.n[tid] = 0;
    }
    for (int i = tid; i < CB; i += kThreads) {
        const int64_t slot = J0 + i;
        const uint32_t col = V.bcol[slot];
        const uint32_t lb = V.blen[slot];
        const _Float16 kf = (_Float16)(float)(1024 - T.lo + V.gap * (LA + (int)lb));
        const uint32_t kbits = __builtin_bit_cast(uint16_t, kf);
        const uint32_t tj = col != 0xFFFF ? threshold_code(key_score(T.thr[J0 + col], T.lo), T.lo) : kCodeNever;
        meta[i] = kbits | (tj << 16);
        if ((i & 63) == 63) gmax[i >> 6] = (uint8_t)lb;
    }
    const bool wt_staged = T.wt_in_lds && A <= kLdsWtabMaxAlphabet;
    if (wt_staged)
        for (int i = tid; i < A * A; i += kThreads) wt_lds[i] = V.wtab[i];
    const uint16_t *wt = wt_staged ? wt_lds : V.wtab;
    const bool diag = r == b;
    const bool padded = (int64_t)(b + 1) * CB > n;   // the last block holds padding slots
    const ProfileRole role = profile_role(tid, A);
    const int CPL = V.CB / kThreads;
    const int lane_base = wave * 64 + lane;

    for (uint32_t k = pbeg, it = 0; k < pend; k += R, ++it) {
        // row-pair chunk: words' symbols, caller indices and threshold codes
        const uint32_t kc = (k - pbeg) % kChunkPairs;
        uint8_t *chunk = chunks + ((k - pbeg) / kChunkPairs & 1) * chunk_bytes(LA);
        uint8_t *csym = chunk;
        int32_t *cu = reinterpret_cast<int32_t *>(chunk + 2 * kChunkPairs * SW);
        uint32_t *ctu = reinterpret_cast<uint32_t *>(cu + 2 * kChunkPairs);
        if (kc == 0) {
            if (tid < 2 * kChunkPairs) {
                const uint32_t kk = k + (uint32_t)(tid >> 1);
                const int32_t slot = kk < pend ? V.rpairs[2 * kk + (tid & 1)] : -1;
                const int64_t uu = slot >= 0 ? I0 + V.bcol[slot] : -1;
                cu[tid] = (int32_t)uu;
                ctu[tid] = uu >= 0 ? threshold_code(key_score(T.thr[uu], T.lo), T.lo) : kCodeNever;
                // an absent word takes symbol 0 throughout: any valid profile, never counted
                const uint32_t *src = reinterpret_cast<const uint32_t *>(V.bsym + (int64_t)(slot >= 0 ? slot : 0) * kWordBytes);
#pragma unroll
                for (uint32_t q = 0; q < SW / 4; ++q)
                    reinterpret_cast<uint32_t *>(csym + tid * SW)[q] = slot >= 0 ? src[q] : 0u;
            }
            __syncthreads();
        }
        const uint8_t *prof = lds + (it & 1) * prof_bytes;
        {
            auto wp = [&](int h) { return csym + (2 * kc + h) * SW; };
            if constexpr (R == 1)
                build_profile<LA>(wt, A, reinterpret_cast<uint32_t *>(lds + (it & 1) * prof_bytes), wp(0), wp(1), role);
            else
                build_profile2<LA>(wt, A, reinterpret_cast<uint32_t *>(lds + (it & 1) * prof_bytes), wp(0), wp(1),
                                   wp(2), wp(3), role);
        }
        __syncthreads();
        const int pb = (int)(it & 1);
        {
            const uint32_t other = pool.n[pb ^ 1];
            if (other >= (uint32_t)kPoolFlush) pool_flush(pool, pb ^ 1, T, other);
        }
        int64_t u[2 * R];
        uint32_t tu[2 * R];
        bool all = true;
#pragma unroll
        for (int h = 0; h < 2 * R; ++h) {
            u[h] = cu[2 * kc + h];
            tu[h] = ctu[2 * kc + h];
            all = all && u[h] >= 0;
        }
        // the short epilogue: every pair of the tile counts, every half real
        const bool fast = !diag && !padded && all;

        // the detailed tests of one pair whose code passed the combined test
        auto offer = [&](uint32_t code, uint32_t tu_h, uint32_t tj, int64_t uu, int64_t j) {
            if (uu < 0) return;
            const int s = (int)code - (int)kCodeOrigin + T.lo;
            if (code >= tu_h) pool_offer(pool, pb, T, uu, nb_key(s, T.lo, (uint32_t)j));
            if (code >= tj) pool_offer(pool, pb, T, j, nb_key(s, T.lo, (uint32_t)uu));
        };
        // general epilogue of one half: validity, histogram, thresholds
        auto general = [&](uint32_t c, int h, uint32_t tj, int64_t j) {
            // each unordered pair once: in a diagonal block only j > u
            if (u[h] < 0 || (diag && j <= u[h])) return;
            if (has_hist) atomicAdd(&hist[(int)c - (int)kCodeOrigin + T.lo], 1u);
            if (c >= min(tu[h], tj)) offer(c, tu[h], tj, u[h], j);
        };
        auto column = [&](const uint32_t(&bw)[kWordBytes / 4], int c) __attribute__((always_inline)) {
            const int sl = lane_base + c * kThreads;   // local column slot
            const uint32_t mt = meta[sl];
            const int lbmax_w = __builtin_amdgcn_readfirstlane((int)gmax[sl >> 6]);
            h2 g[R];
            if constexpr (LA == 0) {
                g[0] = h2{0, 0};
            } else if constexpr (R == 1) {
                g[0] = dp_lane<LA, kWordBytes>(bw, lbmax_w, prof, profile_stride_dw<LA>() * 4u);
            } else {
                dp_lane2<LA, kWordBytes, profile2_off_b(LA)>(bw, lbmax_w, prof, profile2_stride_dw(LA) * 4u, g[0],
                                                            g[1]);
            }
            uint32_t code[R];
#pragma unroll
            for (int q = 0; q < R; ++q) code[q] = __builtin_bit_cast(uint32_t, g[q] + as_h2(mt).xx);
            const uint32_t tj = mt >> 16;
            if (fast) {
                if (has_hist) {
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        const uint32_t ha = __builtin_bit_cast(
                            uint32_t, __builtin_bit_cast(u16x2, code[q]) * u16x2{4, 4} + u16x2{hb, hb});
                        __atomic_fetch_add(lds_ptr(ha & 0xFFFFu), 1u, __ATOMIC_RELAXED);
                        __atomic_fetch_add(lds_ptr(ha >> 16), 1u, __ATOMIC_RELAXED);
                    }
                }
                // any half at or above min(its row threshold, the column threshold)?
                uint32_t all_neg = 0x80008000u;
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const u16x2 mn = __builtin_elementwise_min(u16x2{(uint16_t)tu[2 * q], (uint16_t)tu[2 * q + 1]},
                                                               u16x2{(uint16_t)tj, (uint16_t)tj});
                    all_neg &= __builtin_bit_cast(uint32_t, __builtin_bit_cast(i16x2, code[q]) -
                                                                 __builtin_bit_cast(i16x2, mn));
                }
                if (__builtin_expect(all_neg != 0x80008000u, 0)) {
                    const int64_t j = J0 + (int64_t)V.bcol[J0 + sl];
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        offer(code[q] & 0xFFFFu, tu[2 * q], tj, u[2 * q], j);
                        offer(code[q] >> 16, tu[2 * q + 1], tj, u[2 * q + 1], j);
                    }
                }
                return;
            }
            const uint32_t col = V.bcol[J0 + sl];
            if (col == 0xFFFF) return;
            const int64_t j = J0 + col;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                general(code[q] & 0xFFFFu, 2 * q, tj, j);
                general(code[q] >> 16, 2 * q + 1, tj, j);
            }
        };
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
    __syncthreads();
    for (int bb = 0; bb < 2; ++bb) {
        const uint32_t left = pool.n[bb];
        if (left) pool_flush(pool, bb, T, left);
    }
    if (has_hist) {
        __syncthreads();
        for (int i = tid; i < T.nbins; i += kThreads) {
            uint32_t sum = 0;
            for (int c = 0; c < kHistCopies; ++c) sum += hist_all[c * hs + i];
            if (sum) atomicAdd(&T.hist[i], (unsigned long long)sum);
        }
    }
}

}  // namespace nw
