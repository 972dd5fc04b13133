// k_tri_tiled.h -- the tiled all-pairs kernel that writes the row-major upper
// triangle (Section 4.1 of the paper) in the caller's word order.
//
// The caller-order words are cut into blocks of CB words; a workgroup takes
// one block pair (r, b), r <= b, and one exact row length LA.  It walks the
// row pairs (u, u') of block r whose words both have length LA; for each pair
// it builds the similarity profile in LDS, and every lane runs the DP of the
// pair against CB/256 column words of block b (slots sorted by length, so the
// 64 lanes of a wavefront have near-equal column lengths).  Scores land in an
// LDS staging row in caller column order and leave as two contiguous row
// segments out[idx(u, jstart) ..], so the HBM writes are coalesced even though
// the DP ran in length-sorted order.
//
// Pipelining inside the workgroup: one barrier per row pair.  Iteration k
// builds the profile of pair k (double-buffered) and stores the staged scores
// of pair k-2 (triple-buffered), then, after the barrier, runs the DP of pair k.
#pragma once

#include "nw_tile_common.h"

namespace nw {

// One tile: row pairs [pbeg, pend) of block r (all of length LA) against the
// columns of block b, scores of pair indices in [idx_begin, idx_end) stored to
// `out` (int8 or int16) or, for OUT_EDGES, filtered into the edge sink E.  All threads of the workgroup must call it; it ends
// with a barrier, so the caller may reuse the LDS afterwards.
template <int LA>
__device__ __forceinline__ void tri_tile(const DevVocab &V, uint32_t r, uint32_t b, uint32_t pbeg, uint32_t pend,
                                         uint64_t idx_begin, uint64_t idx_end, void *out, int out_kind,
                                         const EdgeSink &E, uint8_t *lds)
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
        if (last < idx_begin || first >= idx_end) return;   // uniform: the whole workgroup skips
    }

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint32_t prof_bytes = profile_bytes(LA, V.alphabet);
    int16_t *stg = reinterpret_cast<int16_t *>(lds + 2 * prof_bytes);   // [3][2][CB]

    const ProfileRole role = profile_role(tid, V.alphabet);
    const int CPL = V.CB / kThreads;

    for (uint32_t k = pbeg; k < pend + 2; ++k) {
        if (k < pend) {
            const int32_t a0 = V.rpairs[2 * k], a1 = V.rpairs[2 * k + 1];
            build_profile<LA>(V.wtab, V.alphabet, reinterpret_cast<uint32_t *>(lds + (k & 1) * prof_bytes),
                              V.bsym + (int64_t)a0 * kWordBytes, V.bsym + (int64_t)(a1 >= 0 ? a1 : a0) * kWordBytes,
                              role);
        }
        if (k >= pbeg + 2) {
            // store the staged scores of pair k-2 as contiguous row segments
            const uint32_t kk = k - 2;
            const int16_t *srow = stg + (size_t)(kk % 3) * 2 * CB;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int32_t slot = V.rpairs[2 * kk + h];
                if (slot < 0) continue;
                const int64_t u = I0 + V.bcol[slot];
                const int64_t jstart = (r == b) ? u + 1 : J0;
                store_row(V, u, LA, jstart, J1, srow + h * CB + (jstart - J0), idx_begin, idx_end, out, out_kind, E);
            }
        }
        __syncthreads();
        if (k < pend) {
            const int32_t su2 = V.rpairs[2 * k + 1];
            int16_t *sdst = stg + (size_t)(k % 3) * 2 * CB;
            for (int c = 0; c < CPL; ++c) {
                // groups of 64 length-sorted slots dealt round-robin to the
                // wavefronts, so all four carry the same mix of lengths
                const int64_t slot = J0 + (int64_t)(c * kThreads + wave * 64 + lane);
                const int lb = V.blen[slot];
                const int lbmax_w = __builtin_amdgcn_readlane(lb, 63);
                int s0, s1;
                pair_scores<LA>(V.bsym + slot * kWordBytes, lb, lbmax_w, lds + (k & 1) * prof_bytes, V.gap, s0, s1);
                const int col = V.bcol[slot];
                if (col != 0xFFFF) {
                    sdst[col] = (int16_t)s0;
                    if (su2 >= 0) sdst[CB + col] = (int16_t)s1;
                }
            }
        }
    }
}


// Workgroup = tile * chunks + chunk: a tile's row pairs of length LA are
// split into `chunks` runs of at most rpc row pairs, so that launches over few
// tiles (small dictionaries) still fill the GPU.
template <int LA>
__global__ __launch_bounds__(kThreads) void k_tri_tiled(DevVocab V, uint64_t idx_begin, uint64_t idx_end, void *out,
                                                        int out_kind, EdgeSink E, uint32_t rb0, uint32_t rbn,
                                                        uint32_t chunks, uint32_t rpc)
{
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t r, b;
    if (!tile_block_pair(blockIdx.x / chunks, rb0, rbn, V.nb, r, b)) return;
    const uint32_t *rpo = V.rp_off + (size_t)r * (V.lmax + 1) + LA;
    const uint64_t pbeg64 = (uint64_t)rpo[0] + (uint64_t)(blockIdx.x % chunks) * rpc;
    if (pbeg64 >= rpo[1]) return;
    const uint32_t pbeg = (uint32_t)pbeg64;
    const uint32_t pend = rpo[1] - pbeg <= rpc ? rpo[1] : pbeg + rpc;
    tri_tile<LA>(V, r, b, pbeg, pend, idx_begin, idx_end, out, out_kind, E, lds);
}

}  // namespace nw
