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

__host__ __device__ constexpr uint32_t topk_code_lds_bytes(int LA, int alphabet, int nbins, int has_hist, int CB)
{
    return 2u * profile_bytes(LA, alphabet) + topk_hist_bytes(nbins, has_hist) + 8u * (uint32_t)CB +
           topk_pool_bytes();
}

// Does the main pass of this dictionary with these arguments take
// k_topk_code<LA>?  Every score code lies in [0, 1024), and the histogram
// copies (placed after the two profiles) end below 64 KiB.
__host__ __device__ inline bool topk_code_applies(const DevVocab &V, const TopkArgs &T, int LA)
{
    return T.lo <= V.lo && V.hi - T.lo < 1024 && (T.hist == nullptr || T.nbins <= kCodeMaxBins) &&
           2u * profile_bytes(LA, V.alphabet) + topk_hist_bytes(T.nbins, T.hist != nullptr) <= 65536u &&
           topk_code_lds_bytes(LA, V.alphabet, T.nbins, T.hist != nullptr, V.CB) <= kMaxLdsBytes;
}

// The code of threshold score ts: kCodeOrigin + ts - lo, clamped to [0, kCodeNever].
__device__ __forceinline__ uint32_t threshold_code(int ts, int lo)
{
    const int c = (int)kCodeOrigin + ts - lo;
    return (uint32_t)min(max(c, 0), (int)kCodeNever);
}

template <int LA>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(topk_min_waves<LA>())))
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
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint32_t prof_bytes = profile_bytes(LA, V.alphabet);
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
    // column metadata: x = column | K << 16 (K = binary16 of 1024 - lo + gap (LA + lb)),
    // y = threshold code of the column word | lb << 16
    const uint32_t meta_off = hist_off + topk_hist_bytes(T.nbins, has_hist);
    uint2 *meta = reinterpret_cast<uint2 *>(lds + meta_off);
    CandPool pool;
    {
        uint8_t *pb = lds + meta_off + 8u * (uint32_t)CB;
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
        meta[i] = make_uint2(col | (kbits << 16), tj | (lb << 16));
    }
    const bool diag = r == b;
    const bool padded = (int64_t)(b + 1) * CB > n;   // the last block holds padding slots
    const ProfileRole role = profile_role(tid, V.alphabet);
    const int CPL = V.CB / kThreads;
    const int lane_base = wave * 64 + lane;

    for (uint32_t k = pbeg; k < pend; ++k) {
        const int32_t a0 = V.rpairs[2 * k], a1 = V.rpairs[2 * k + 1];
        const uint8_t *prof = lds + (k & 1) * prof_bytes;
        build_profile<LA>(V.wtab, V.alphabet, reinterpret_cast<uint32_t *>(lds + (k & 1) * prof_bytes),
                          V.bsym + (int64_t)a0 * kWordBytes, V.bsym + (int64_t)(a1 >= 0 ? a1 : a0) * kWordBytes, role);
        __syncthreads();
        const int pb = (int)(k & 1);
        {
            const uint32_t other = pool.n[pb ^ 1];
            if (other >= (uint32_t)kPoolFlush) pool_flush(pool, pb ^ 1, T, other);
        }
        const int64_t u0 = I0 + V.bcol[a0];
        const int64_t u1 = a1 >= 0 ? I0 + V.bcol[a1] : -1;
        const uint32_t tu0 = threshold_code(key_score(T.thr[u0], T.lo), T.lo);
        const uint32_t tu1 = u1 >= 0 ? threshold_code(key_score(T.thr[u1], T.lo), T.lo) : kCodeNever;
        const u16x2 tu = u16x2{(uint16_t)tu0, (uint16_t)tu1};
        // the short epilogue: every pair of the tile counts, both halves real
        const bool fast = !diag && !padded && a1 >= 0;

        // the detailed tests of one pair whose code passed the combined test
        auto offer = [&](uint32_t code, uint32_t tu_h, uint32_t tj, int64_t u, int64_t j) {
            const int s = (int)code - (int)kCodeOrigin + T.lo;
            if (code >= tu_h) pool_offer(pool, pb, T, u, nb_key(s, T.lo, (uint32_t)j));
            if (code >= tj) pool_offer(pool, pb, T, j, nb_key(s, T.lo, (uint32_t)u));
        };
        auto column = [&](const uint32_t(&bw)[kWordBytes / 4], int c) __attribute__((always_inline)) {
            const uint2 m = meta[lane_base + c * kThreads];
            const int lbmax_w = (int)((uint32_t)__builtin_amdgcn_readlane((int)m.y, 63) >> 16);
            h2 g;
            if constexpr (LA == 0)
                g = h2{0, 0};
            else
                g = dp_lane<LA, kWordBytes>(bw, lbmax_w, prof, profile_stride_dw<LA>() * 4u);
            const uint32_t code = __builtin_bit_cast(uint32_t, g + as_h2(m.x).yy);
            const u16x2 cv = __builtin_bit_cast(u16x2, code);
            const uint32_t tj = m.y & 0xFFFFu;
            if (fast) {
                if (has_hist) {
                    const uint32_t ha = __builtin_bit_cast(uint32_t, cv * u16x2{4, 4} + u16x2{hb, hb});
                    __atomic_fetch_add(lds_ptr(ha & 0xFFFFu), 1u, __ATOMIC_RELAXED);
                    __atomic_fetch_add(lds_ptr(ha >> 16), 1u, __ATOMIC_RELAXED);
                }
                // either half at or above min(its row threshold, the column threshold)?
                const u16x2 mn = __builtin_elementwise_min(tu, u16x2{(uint16_t)tj, (uint16_t)tj});
                const uint32_t d =
                    __builtin_bit_cast(uint32_t, __builtin_bit_cast(i16x2, cv) - __builtin_bit_cast(i16x2, mn));
                if (__builtin_expect((d & 0x80008000u) != 0x80008000u, 0)) {
                    const int64_t j = J0 + (int64_t)(m.x & 0xFFFFu);
                    offer(code & 0xFFFFu, tu0, tj, u0, j);
                    offer(code >> 16, tu1, tj, u1, j);
                }
                return;
            }
            const uint32_t col = m.x & 0xFFFFu;
            if (col == 0xFFFF) return;
            const int64_t j = J0 + col;
            const uint32_t c0 = code & 0xFFFFu, c1 = code >> 16;
            // each unordered pair once: in a diagonal block only j > u
            const bool v0 = !diag || j > u0;
            const bool v1 = u1 >= 0 && (!diag || j > u1);
            if (has_hist) {
                if (v0) atomicAdd(&hist[(int)c0 - (int)kCodeOrigin + T.lo], 1u);
                if (v1) atomicAdd(&hist[(int)c1 - (int)kCodeOrigin + T.lo], 1u);
            }
            if (v0 && c0 >= min(tu0, tj)) offer(c0, tu0, tj, u0, j);
            if (v1 && c1 >= min(tu1, tj)) offer(c1, tu1, tj, u1, j);
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
