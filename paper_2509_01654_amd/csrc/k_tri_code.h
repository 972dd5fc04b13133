// k_tri_code.h -- the tiled triangle kernel (int8 / int16 scores of the
// row-major upper triangle, Section 4.1 of the paper) with score codes and
// dword-wide segment stores.
//
// Same tiling and pipelining as k_tri_tiled: a workgroup takes a block pair
// (r, b) and a run of block r's row pairs of one length LA, builds each row
// pair's profile (double-buffered), runs every lane's column words against
// it, stages the scores in LDS in caller column order (triple-buffered) and
// writes each row's segment of the triangle two row pairs later.  The
// differences:
//
// * score codes: adding K = 1280 + gap (LA + lb) to the DP result G gives the
//   binary16 value 1280 + s, whose bits are 0x6500 + s for -256 <= s < 768
//   (binary16 spacing is 1 on [1024, 2048)).  The low byte of a code is the
//   int8 score, and code - 0x6500 the int16 score, so one packed add (and, for
//   int16, one packed subtract) turns both pairs' results into their stored
//   form;
// * segments leave as aligned dwords: each dword of the output is assembled
//   from two staged dwords with one byte-align, and only the up to three
//   elements before the first and after the last whole dword are written
//   singly.
//
// Padding slots of the last block stage into a spare slot past the row
// (column CB), so no lane branches on them.  Scores are exact in the same way
// as in k_tri_tiled (nw_dp.h); the kernel applies while every score lies in
// [-256, 768).
#pragma once

#include "k_topk_code.h"
#include "k_tri_tiled.h"

namespace nw {

constexpr int kTriCodeBias = 1280;
constexpr uint32_t kTriCodeOrigin = 0x6500u;

// Bytes of one staged row: CB scores, the spare slot, and slack for the
// second dword a segment's last aligned read touches.
__host__ __device__ constexpr uint32_t tri_code_stage_row(int CB, int es) { return (uint32_t)(CB + 8) * (uint32_t)es; }
// Row pairs per step: two for the short rows (one column address serves
// both, and the barrier and column loads are shared) while the buffers leave
// at least four workgroups per CU; one otherwise.
constexpr uint32_t kTriPairLdsBudget = 40u * 1024u;
// Dynamic LDS: two profile buffers, 4 bytes of metadata per column slot, the
// longest length of each group of 64 slots, two row-pair chunks (symbols and
// caller indices) and three staged steps of 2R rows each.
__host__ __device__ constexpr uint32_t tri_chunk_bytes(int LA) { return 2u * kChunkPairs * (chunk_sym_bytes(LA) + 4u); }
__host__ __device__ constexpr uint32_t tri_code_lds_bytes(int LA, int alphabet, int CB, int es, int R)
{
    return 2u * topk_code_profile_bytes(LA, R, alphabet) + 4u * (uint32_t)CB + (((uint32_t)CB / 64u + 15u) & ~15u) +
           2u * tri_chunk_bytes(LA) + 3u * 2u * (uint32_t)R * tri_code_stage_row(CB, es);
}

// Does a triangle call on this dictionary take k_tri_code<LA, R>?  Every
// score lies in [-256, 768) and the buffers fit.
__host__ __device__ inline bool tri_code_applies(const DevVocab &V, int LA, int es, int R)
{
    return V.lo >= -256 && V.hi < 768 &&
           tri_code_lds_bytes(LA, V.alphabet, V.CB, es, R) <= (R == 1 ? kMaxLdsBytes : kTriPairLdsBudget);
}

// Write a staged row segment of len elements (es bytes each) at LDS address
// sl to global memory at g.  Every thread of the workgroup calls it.
__device__ __forceinline__ void store_segment(uint8_t *g, uint32_t sl, int64_t len, int es)
{
    const int tid = threadIdx.x;
    const uint64_t nbytes = (uint64_t)len * (uint64_t)es;
    const uint32_t head = (uint32_t)((4u - ((uintptr_t)g & 3u)) & 3u);
    if ((uint64_t)head >= nbytes || (head % (uint32_t)es) != 0) {
        // a short segment (or a misaligned int16 one): element by element
        for (int64_t t = tid; t < len; t += kThreads) {
            if (es == 1)
                g[t] = *lds_ptr8(sl + (uint32_t)t);
            else
                reinterpret_cast<uint16_t *>(g)[t] = *lds_ptr16(sl + 2u * (uint32_t)t);
        }
        return;
    }
    const uint64_t nfull = (nbytes - head) / 4u;
    uint32_t *gd = reinterpret_cast<uint32_t *>(g + head);
    const uint32_t s0 = sl + head;
    const uint32_t sh = s0 & 3u;   // the same byte shift for every dword of the segment
    for (uint64_t d = tid; d < nfull; d += kThreads) {
        const uint32_t a = (s0 & ~3u) + 4u * (uint32_t)d;
        const uint32_t x0 = *lds_ptr(a), x1 = *lds_ptr(a + 4);
        gd[d] = __builtin_amdgcn_alignbyte(x1, x0, sh);
    }
    // the bytes before the first and after the last whole dword (whole elements)
    const uint64_t tail = head + 4u * nfull;
    const uint32_t nedge = head + (uint32_t)(nbytes - tail);
    if ((uint32_t)tid < nedge / (uint32_t)es) {
        const uint64_t byte = (uint32_t)tid * es < head ? (uint64_t)tid * es : tail + ((uint64_t)tid * es - head);
        if (es == 1)
            g[byte] = *lds_ptr8(sl + (uint32_t)byte);
        else
            *reinterpret_cast<uint16_t *>(g + byte) = *lds_ptr16(sl + (uint32_t)byte);
    }
}

// One tile: row pairs [pbeg, pend) of block r (all of length LA) against the
// columns of block b, scores of pair indices in [idx_begin, idx_end) stored
// to out (es bytes each).  Every thread of the workgroup calls it; it ends
// with a barrier, so the caller may reuse the LDS afterwards.
template <int LA, int R>
__device__ __forceinline__ void tri_tile_code(const DevVocab &V, uint32_t r, uint32_t b, uint32_t pbeg, uint32_t pend,
                                              uint64_t idx_begin, uint64_t idx_end, void *out, int es, uint8_t *lds)
{
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

    const int A = V.alphabet;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint32_t PB = topk_code_profile_bytes(LA, R, A);
    const uint32_t lds0 = lds_addr_of(lds);
    // per column slot: staging column (CB for padding slots) | K << 16; per
    // group of 64 slots: the longest length
    uint32_t *meta = reinterpret_cast<uint32_t *>(lds + 2 * PB);
    uint8_t *gmax = reinterpret_cast<uint8_t *>(meta + CB);
    uint8_t *chunks_lds = gmax + (((uint32_t)CB / 64u + 15u) & ~15u);
    const uint32_t stage_off = (uint32_t)(chunks_lds - lds) + 2u * tri_chunk_bytes(LA);
    const uint32_t SR = tri_code_stage_row((int)CB, es);
    constexpr uint32_t SW = chunk_sym_bytes(LA);
    for (int i = tid; i < CB; i += kThreads) {
        const int64_t slot = J0 + i;
        const uint32_t col = V.bcol[slot];
        const uint32_t lb = V.blen[slot];
        const _Float16 kf = (_Float16)(float)(kTriCodeBias + V.gap * (LA + (int)lb));
        const uint32_t kbits = __builtin_bit_cast(uint16_t, kf);
        meta[i] = (col == 0xFFFF ? (uint32_t)CB : col) | (kbits << 16);
        if ((i & 63) == 63) gmax[i >> 6] = (uint8_t)lb;
    }
    // the weight table stays in global memory (cached): in LDS it would cost
    // a workgroup per CU, which the triangle's short steps need more
    const uint16_t *wt = V.wtab;
    const ProfileRole role = profile_role(tid, A);
    const int CPL = V.CB / kThreads;
    const int lane_base = wave * 64 + lane;
    auto chunk_of = [&](uint32_t k) { return chunks_lds + ((k - pbeg) / kChunkPairs & 1) * tri_chunk_bytes(LA); };

    // step s covers row pairs pbeg + R s .. + R - 1; its rows are stored two steps later
    const uint32_t nsteps = (pend - pbeg + R - 1) / R;
    for (uint32_t st = 0; st < nsteps + 2; ++st) {
        const uint32_t k = pbeg + R * st;
        if (st < nsteps) {
            const uint32_t kc = (k - pbeg) % kChunkPairs;
            uint8_t *chunk = chunk_of(k);
            uint8_t *csym = chunk;
            int32_t *cu = reinterpret_cast<int32_t *>(chunk + 2 * kChunkPairs * SW);
            if (kc == 0) {
                if (tid < 2 * kChunkPairs) {
                    const uint32_t kk = k + (uint32_t)(tid >> 1);
                    const int32_t slot = kk < pend ? V.rpairs[2 * kk + (tid & 1)] : -1;
                    cu[tid] = slot >= 0 ? (int32_t)(I0 + V.bcol[slot]) : -1;
                    const uint32_t *src =
                        reinterpret_cast<const uint32_t *>(V.bsym + (int64_t)(slot >= 0 ? slot : 0) * kWordBytes);
#pragma unroll
                    for (uint32_t q = 0; q < SW / 4; ++q)
                        reinterpret_cast<uint32_t *>(csym + tid * SW)[q] = slot >= 0 ? src[q] : 0u;
                }
                __syncthreads();
            }
            auto wp = [&](int h) { return csym + (2 * kc + h) * SW; };
            if constexpr (R == 1)
                build_profile<LA>(wt, A, reinterpret_cast<uint32_t *>(lds + (st & 1) * PB), wp(0), wp(1), role);
            else
                build_profile2<LA>(wt, A, reinterpret_cast<uint32_t *>(lds + (st & 1) * PB), wp(0), wp(1), wp(2),
                                   wp(3), role);
        }
        if (st >= 2) {
            // store the staged rows of step st - 2 as contiguous row segments
            const uint32_t ks = pbeg + R * (st - 2);
            const uint32_t kc = (ks - pbeg) % kChunkPairs;
            const int32_t *cu = reinterpret_cast<const int32_t *>(chunk_of(ks) + 2 * kChunkPairs * SW);
#pragma unroll
            for (int h = 0; h < 2 * R; ++h) {
                const int64_t u = cu[2 * kc + h];
                if (u < 0) continue;
                const int64_t jstart = (r == b) ? u + 1 : J0;
                const int64_t len = J1 - jstart;
                if (len <= 0) continue;
                const uint32_t sl = lds0 + stage_off + (((st - 2) % 3) * 2 * R + h) * SR + (uint32_t)(jstart - J0) * es;
                const uint64_t base = row_start_idx(n, u) + (uint64_t)(jstart - u - 1);
                if (base >= idx_begin && base + (uint64_t)len <= idx_end) {
                    store_segment(static_cast<uint8_t *>(out) + (base - idx_begin) * es, sl, len, es);
                } else {
                    for (int64_t t = tid; t < len; t += kThreads) {
                        const uint64_t idx = base + (uint64_t)t;
                        if (idx < idx_begin || idx >= idx_end) continue;
                        uint8_t *g = static_cast<uint8_t *>(out) + (idx - idx_begin) * es;
                        if (es == 1)
                            *g = *lds_ptr8(sl + (uint32_t)t);
                        else
                            *reinterpret_cast<uint16_t *>(g) = *lds_ptr16(sl + 2u * (uint32_t)t);
                    }
                }
            }
        }
        __syncthreads();
        if (st < nsteps) {
            const uint8_t *prof = lds + (st & 1) * PB;
            const uint32_t st0 = lds0 + stage_off + (st % 3) * 2 * R * SR;
            const uint8_t *wbase = V.bsym + (J0 + lane_base) * kWordBytes;
            for (int c = 0; c < CPL; ++c) {
                const int sl = lane_base + c * kThreads;
                const uint32_t m = meta[sl];
                const int lbmax_w = __builtin_amdgcn_readfirstlane((int)gmax[sl >> 6]);
                uint32_t bw[kWordBytes / 4];
                load_word(bw, wbase + (int64_t)c * kThreads * kWordBytes);
                h2 g[R];
                if constexpr (LA == 0) {
                    g[0] = h2{0, 0};
                } else if constexpr (R == 1) {
                    g[0] = dp_lane<LA, kWordBytes>(bw, lbmax_w, prof, profile_stride_dw<LA>() * 4u);
                } else {
                    dp_lane2<LA, kWordBytes, profile2_off_b(LA)>(bw, lbmax_w, prof, profile2_stride_dw(LA) * 4u,
                                                                g[0], g[1]);
                }
                const uint32_t col = m & 0xFFFFu;
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const uint32_t code = __builtin_bit_cast(uint32_t, g[q] + as_h2(m).yy);
                    const uint32_t row = st0 + 2 * q * SR;   // the staged rows of this pair
                    // absent rows stage like present ones and are never stored
                    if (es == 1) {
                        *lds_ptr8(row + col) = (uint8_t)code;
                        *lds_ptr8(row + SR + col) = (uint8_t)(code >> 16);
                    } else {
                        const uint32_t sc = __builtin_bit_cast(
                            uint32_t, __builtin_bit_cast(u16x2, code) -
                                          u16x2{(uint16_t)kTriCodeOrigin, (uint16_t)kTriCodeOrigin});
                        *lds_ptr16(row + 2 * col) = (uint16_t)sc;
                        *lds_ptr16(row + SR + 2 * col) = (uint16_t)(sc >> 16);
                    }
                }
            }
        }
    }
}

// Workgroup = tile * chunks + chunk: a tile's row pairs of length LA are
// split into `chunks` runs of at most rpc row pairs (rpc a multiple of R).
template <int LA, int R>
__global__ __launch_bounds__(kThreads) void k_tri_code(DevVocab V, uint64_t idx_begin, uint64_t idx_end, void *out,
                                                       int es, uint32_t rb0, uint32_t rbn, uint32_t chunks,
                                                       uint32_t rpc)
{
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t r, b;
    if (!tile_block_pair(blockIdx.x / chunks, rb0, rbn, V.nb, r, b)) return;
    const uint32_t *rpo = V.rp_off + (size_t)r * (V.lmax + 1) + LA;
    const uint64_t pbeg64 = (uint64_t)rpo[0] + (uint64_t)(blockIdx.x % chunks) * rpc;
    if (pbeg64 >= rpo[1]) return;
    const uint32_t pbeg = (uint32_t)pbeg64;
    const uint32_t pend = rpo[1] - pbeg <= rpc ? rpo[1] : pbeg + rpc;
    tri_tile_code<LA, R>(V, r, b, pbeg, pend, idx_begin, idx_end, out, es, lds);
}

}  // namespace nw
