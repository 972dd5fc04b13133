// k_probe.h -- the threshold pre-pass of the all-pairs top-k as a selection.
//
// Every word u needs one key from the pre-pass: its key of rank m = k + 1
// (rank 1 is the best) against the probe subset, the M words at caller
// indices floor(i n / M), i = 0 .. M-1 (keys as in nw_topk.h: score
// descending, then index ascending; the word itself counts when it is a
// probe).  When every score code s - lo fits in a byte below 0xFF, a
// workgroup finds that key for a pair of equal-length words without keeping
// sorted lists:
//   1. the DP of the pair against every probe slot (length-sorted, as the
//      query kernel walks them) adds each word's code to an LDS histogram
//      and stores it at the probe's rank i in an LDS byte array, so the
//      array is in caller-index order;
//   2. one wavefront per word walks the histogram from the best code down to
//      the code c that holds rank m, and the place r of the wanted key among
//      the keys of code c;
//   3. keys of equal score rank by index ascending and floor(i n / M) rises
//      with i, so the wanted probe is the r-th rank i (ascending) whose code
//      is c: a scan of the byte array, 256 ranks a step.
// A word with fewer than m probe keys gets key 0, as a short list would.
#pragma once

#include "nw_tile_common.h"
#include "nw_topk.h"

namespace nw {

constexpr int kProbeMaxCode = 254;      // codes 0 .. 254; 0xFF fills the tail of the byte arrays
constexpr int kProbeMaxSlots = 65536;   // ranks are 16-bit

struct ProbeArgs {
    RowSet R;                   // the dictionary's words in pairs of equal length
    ColSet C;                   // probe slots, length-sorted, padding slots first
    const uint16_t *rank;       // [C.nslots] rank i of each probe slot (padding: unused)
    const uint16_t *wtab;
    int alphabet;
    int gap;
    int lo;                     // key origin: code = score - lo, at most kProbeMaxCode
    int m;                      // rank of the wanted key, >= 1
    int rpw;                    // row pairs per workgroup
    int64_t n;                  // dictionary size
    int64_t nprobe;             // M, 1 .. C.nslots
    uint64_t *thr;              // [n] the key of each word, by caller index
};

__host__ __device__ constexpr uint32_t probe_prof_bytes(int LA, int alphabet)
{
    return (profile_bytes(LA, alphabet) + 15u) & ~15u;
}
// LDS: one profile, two 256-bin histograms, two byte arrays of nslots codes.
__host__ __device__ constexpr uint32_t probe_lds_bytes(int LA, int alphabet, int64_t nslots)
{
    return probe_prof_bytes(LA, alphabet) + 2u * 256u * 4u + 2u * (uint32_t)nslots;
}

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)x, d);
        if (lane >= d) x += t;
    }
    return x;
}

// The key of rank m of one word from its histogram and its rank-ordered codes
// (one whole wavefront).  Clears the histogram for the next word.
__device__ uint64_t probe_select(uint32_t *hist, const uint8_t *codes, int64_t nslots, const ProbeArgs &Q, int lane)
{
    // lane l holds bins 4(63-l) .. 4(63-l)+3: lane 0 the best codes
    lds_u32x4 *h4 = reinterpret_cast<lds_u32x4 *>(lds_ptr(lds_addr_of(hist))) + (63 - lane);
    const u32x4 h = *h4;
    *h4 = u32x4{0u, 0u, 0u, 0u};
    const uint32_t m = (uint32_t)Q.m;
    const uint32_t cnt = h[0] + h[1] + h[2] + h[3];
    const uint32_t incl = wave_inclusive_sum(cnt, lane);
    if ((uint32_t)__builtin_amdgcn_readlane((int)incl, 63) < m) return 0;
    const int L = __builtin_ctzll(__ballot(incl >= m));
    // in lane L, bins from the best down: the code c holding rank m and the
    // place r of the wanted key among the keys of code c
    int c = 0;
    uint32_t r = 0, before = incl - cnt;
#pragma unroll
    for (int q = 3; q >= 0; --q)
        if (r == 0) {
            if (before + h[q] >= m) {
                c = 4 * (63 - lane) + q;
                r = m - before;
            }
            before += h[q];
        }
    c = __builtin_amdgcn_readlane(c, L);
    r = (uint32_t)__builtin_amdgcn_readlane((int)r, L);

    const uint32_t c4 = (uint32_t)c * 0x01010101u;
    const uint32_t base_addr = lds_addr_of(codes) + 4u * (uint32_t)lane;
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t need = r;   // wave-uniform, 1-based
    for (int64_t base = 0; base < nslots; base += 256) {
        const uint32_t x = *lds_ptr(base_addr + (uint32_t)base) ^ c4;
        // 0x80 in each byte of x that is zero (a code equal to c), exactly
        const uint32_t z = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);
        const uint32_t k4 = (uint32_t)__popc(z);   // 0 .. 4
        const uint64_t b0 = __ballot(k4 & 1u), b1 = __ballot(k4 & 2u), b2 = __ballot(k4 & 4u);
        const uint32_t tot = (uint32_t)(__popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2));
        if (need > tot) {
            need -= tot;
            continue;
        }
        const uint32_t excl = (uint32_t)(__popcll(b0 & lt) + 2 * __popcll(b1 & lt) + 4 * __popcll(b2 & lt));
        const bool here = excl < need && need <= excl + k4;
        const int W = __builtin_ctzll(__ballot(here));
        uint32_t zz = z;
        for (uint32_t q = excl + 1; here && q < need; ++q) zz &= zz - 1u;
        const int byte = here ? (int)(__builtin_ctz(zz) >> 3) : 0;
        const int64_t i = base + 4 * W + __builtin_amdgcn_readlane(byte, W);
        const uint64_t j = (uint64_t)i * (uint64_t)Q.n / (uint64_t)Q.nprobe;
        return ((uint64_t)(uint32_t)c << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)j);
    }
    return 0;   // not reached: the histogram counted at least r codes c
}

template <int LA>
__global__ __launch_bounds__(kThreads) void k_probe_thr(ProbeArgs Q)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t off0 = Q.R.off[LA], off1 = Q.R.off[LA + 1];
    const uint32_t pbeg = off0 + blockIdx.x * (uint32_t)Q.rpw;
    if (pbeg >= off1) return;
    const uint32_t pend = min(pbeg + (uint32_t)Q.rpw, off1);
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t ns = Q.C.nslots;
    const uint32_t pb = probe_prof_bytes(LA, Q.alphabet);
    uint8_t *prof = lds;
    uint32_t *hist = reinterpret_cast<uint32_t *>(lds + pb);   // [2 words][256]
    uint8_t *codes = lds + pb + 2 * 256 * 4;                     // [2 words][ns]
    const uint32_t hist_a = lds_addr_of(hist), codes_a = lds_addr_of(codes);
    const ProfileRole role = profile_role(tid, Q.alphabet);
    for (int i = tid; i < 2 * 256; i += kThreads) *lds_ptr(hist_a + 4u * (uint32_t)i) = 0u;
    for (int64_t i = Q.nprobe + tid; i < ns; i += kThreads) {
        *lds_ptr8(codes_a + (uint32_t)i) = 0xFF;
        *lds_ptr8(codes_a + (uint32_t)(ns + i)) = 0xFF;
    }
    for (uint32_t p = pbeg; p < pend; ++p) {
        const int32_t a0 = Q.R.pairs[2 * p], a1 = Q.R.pairs[2 * p + 1];
        build_profile<LA>(Q.wtab, Q.alphabet, reinterpret_cast<uint32_t *>(prof), Q.R.sym + (int64_t)a0 * kWordBytes,
                          Q.R.sym + (int64_t)(a1 >= 0 ? a1 : a0) * kWordBytes, role);
        // the profile is in, and the previous pair's selections (which clear
        // the histograms) are done
        __syncthreads();
        for (int64_t base = wave * 64; base < ns; base += kThreads) {
            const int64_t slot = base + lane;
            const int lb = Q.C.len[slot];
            const int lbmax_w = __builtin_amdgcn_readlane(lb, 63);
            const int32_t d = Q.C.orig[slot];
            const uint32_t i = Q.rank[slot];
            int s0, s1;
            pair_scores<LA>(Q.C.sym + slot * kWordBytes, lb, lbmax_w, prof, Q.gap, s0, s1);
            if (d >= 0) {
                const uint32_t c0 = (uint32_t)(s0 - Q.lo);
                __atomic_fetch_add(lds_ptr(hist_a + 4u * c0), 1u, __ATOMIC_RELAXED);
                *lds_ptr8(codes_a + i) = (uint8_t)c0;
                if (a1 >= 0) {
                    const uint32_t c1 = (uint32_t)(s1 - Q.lo);
                    __atomic_fetch_add(lds_ptr(hist_a + 4u * (256u + c1)), 1u, __ATOMIC_RELAXED);
                    *lds_ptr8(codes_a + (uint32_t)ns + i) = (uint8_t)c1;
                }
            }
        }
        __syncthreads();   // every probe's code is in
        if (wave < 2 && (wave == 0 || a1 >= 0)) {
            const uint64_t key = probe_select(hist + wave * 256, codes + wave * ns, ns, Q, lane);
            if (lane == 0) Q.thr[Q.R.orig[wave == 0 ? a0 : a1]] = key;
        }
    }
}

}  // namespace nw
