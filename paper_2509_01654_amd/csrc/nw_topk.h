// nw_topk.h -- neighbour-list helpers shared by the top-k and query kernels.
//
// A neighbour of word u is ranked by (score descending, index ascending).  Both
// are folded into one 64-bit key that compares the same way:
//     key(s, j) = (s - lo) << 32 | (0xFFFFFFFF - j),   lo <= s, 0 <= j < 2^31,
// so a larger key is a better neighbour and keys of distinct indices differ.
// Key 0 never occurs (the low word is >= 2^31) and marks an empty entry.
//
// Wave list: a wavefront keeps a sorted top-k (k <= 64) of keys in one 64-bit
// value per lane; lane i holds the i-th best key.  A new key is inserted by
// counting the lanes holding better keys (a prefix, since the list is sorted)
// and shifting the rest down by one lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nw {

__device__ __forceinline__ uint64_t nb_key(int s, int lo, uint32_t j)
{
    return ((uint64_t)(uint32_t)(s - lo) << 32) | (uint64_t)(0xFFFFFFFFu - j);
}
__host__ __device__ __forceinline__ int key_score(uint64_t key, int lo) { return (int)(key >> 32) + lo; }
__host__ __device__ __forceinline__ int32_t key_index(uint64_t key) { return (int32_t)(0xFFFFFFFFu - (uint32_t)key); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// value of lane-1 (lane 0 receives lane 63's value, which the caller ignores)
__device__ __forceinline__ uint64_t shift_down_lanes(uint64_t v, int lane)
{
    const int src = ((lane + 63) & 63) << 2;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Insert wave-uniform key x into the sorted wave list (lanes 0..63).
__device__ __forceinline__ void wl_insert(uint64_t &list, uint64_t x, int lane)
{
    const uint64_t better = __ballot(list > x);
    const int pos = __popcll(better);
    const uint64_t sh = shift_down_lanes(list, lane);
    list = lane < pos ? list : (lane == pos ? x : sh);
}

// Offer every lane's key to the wave list (all lanes of the wave must call).
// thr is the list's current k-th key (wave-uniform) and is kept up to date.
__device__ __forceinline__ void wl_offer(uint64_t &list, uint64_t &thr, uint64_t key, int k, int lane)
{
    uint64_t mask = __ballot(key > thr);
    while (mask) {
        const int l = __builtin_ctzll(mask);
        mask &= mask - 1;
        const uint64_t x = readlane64(key, l);
        if (x > thr) {
            wl_insert(list, x, lane);
            thr = readlane64(list, k - 1);
        }
    }
}

// Offer the keys src[b0 .. b1) to a wave list (whole wavefront), loading them
// eight per lane at a time so that one load latency covers 512 keys.
__device__ __forceinline__ void offer_range(uint64_t &list, uint64_t &t, const uint64_t *src, int b0, int b1, int kout,
                                            int lane)
{
    constexpr int kBatch = 8;
    for (int base = b0; base < b1; base += 64 * kBatch) {
        uint64_t key[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            const int i = base + q * 64 + lane;
            key[q] = i < b1 ? src[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q)
            if (base + q * 64 < b1) wl_offer(list, t, key[q], kout, lane);
    }
}

// Dictionary (or probe) words in blocked, length-sorted slot order.
struct ColSet {
    const uint8_t *sym;     // [nslots * kWordBytes], sentinel-padded
    const uint8_t *len;     // [nslots]
    const int32_t *orig;    // [nslots] caller index, -1 for padding slots
    int64_t nslots;         // multiple of 256
};

// Row words (queries) grouped in pairs of equal length: the pairs of length L
// are pairs[off[L] .. off[L+1]) (second slot -1 when unpaired).
struct RowSet {
    const uint8_t *sym;     // [slots * kWordBytes]
    const int32_t *pairs;   // [npairs][2] slots
    const uint32_t *off;    // [kMaxLen + 2]
    const int32_t *orig;    // [slots] output row of the word
};

}  // namespace nw
