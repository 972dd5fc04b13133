// k_diag.h -- intra-pair anti-diagonal triangle kernel for long words.
//
// The stencil the paper points to as the way to parallelise inside one score
// matrix (Section 6: each cell depends on its up, left and up-left
// neighbours, Section 4.2).  A group of 16 lanes shares one column word; lane
// t owns the R consecutive rows t*R+1 .. t*R+R of the DP (the same binary16
// recurrence G of nw_dp.h, two row words in the two halves).  At step s lane
// t processes column s - t, so the 16 lanes work on one anti-diagonal band:
// the cell above a lane's first row is the last row of lane t-1 one step
// earlier, and the diagonal neighbour is that value one step before, passed
// down the group with a DPP row shift (lane 0 of each 16-lane row receives
// 0, the G[0][j] boundary).  Columns before the start (s - t < 0) and past the
// end of the word read the sentinel symbol, whose profile row leaves a DP
// column unchanged (nw_dp.h), so every lane runs every step with no branch.
//
// Rows per lane R is a template parameter (16*R rows cover words up to 16*R
// symbols); a row pair of length LA <= 16*R runs in class R, and the score is
// read from row LA of the final column.  The similarity profile of the row
// pair spans 16*R positions (positions >= LA are never read into rows <= LA).
#pragma once

#include "nw_tile_common.h"

namespace nw {

constexpr int kDiagLanes = 16;        // lanes per pair
constexpr int kDiagMaxLen = 255;      // longest word of the anti-diagonal path
constexpr int kDiagBuf = 16 + kDiagMaxLen + 16 + 16;   // sentinel | word | sentinel (+ pad)

__host__ __device__ constexpr uint32_t diag_stride_dw(int R) { return (uint32_t)((((kDiagLanes * R) / 4) | 1) * 4); }
__host__ __device__ constexpr uint32_t diag_prof_bytes(int R, int alphabet)
{
    return (uint32_t)(alphabet + 1) * diag_stride_dw(R) * 4u;
}
// LDS: one profile, three int16 staging row pairs, 16 group word buffers.
__host__ __device__ constexpr uint32_t diag_lds_bytes(int R, int alphabet, int CB)
{
    return diag_prof_bytes(R, alphabet) + 3u * 2u * (uint32_t)CB * 2u + 16u * kDiagBuf;
}

__device__ __forceinline__ uint32_t dpp_row_shr1(uint32_t v)
{
    // row_shr:1 within rows of 16 lanes; lane 0 of a row reads 0 (bound_ctrl)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
}

template <int R>
__global__ __launch_bounds__(kThreads) void k_tri_diag(DevVocab V, uint64_t idx_begin, uint64_t idx_end, void *out,
                                                       int out_kind, EdgeSink E, int LA, uint32_t rb0, uint32_t rbn)
{
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr uint32_t S = diag_stride_dw(R);
    constexpr int ROWS = kDiagLanes * R;

    uint32_t r, b;
    if (!tile_block_pair(blockIdx.x, rb0, rbn, V.nb, r, b)) return;
    const uint32_t *rpo = V.rp_off + (size_t)r * (V.lmax + 1) + LA;
    const uint32_t pbeg = rpo[0], pend = rpo[1];
    if (pbeg >= pend) return;
    const int64_t n = V.n, CB = V.CB;
    const int64_t I0 = (int64_t)r * CB, I1 = min(I0 + CB, n);
    const int64_t J0 = (int64_t)b * CB, J1 = min(J0 + CB, n);
    {
        const int64_t jlo = (r == b) ? I0 + 1 : J0;
        if (jlo >= J1) return;
        const uint64_t first = row_start_idx(n, I0) + (uint64_t)(jlo - I0 - 1);
        const int64_t ilast = (r == b) ? J1 - 2 : I1 - 1;
        const uint64_t last = row_start_idx(n, ilast) + (uint64_t)(J1 - 1 - ilast - 1);
        if (last < idx_begin || first >= idx_end) return;
    }

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int t = tid & (kDiagLanes - 1);          // position in the group
    const int g = tid / kDiagLanes;                // group 0..15 of the workgroup
    const int A = V.alphabet;
    uint32_t *prof = reinterpret_cast<uint32_t *>(lds);
    int16_t *stg = reinterpret_cast<int16_t *>(lds + diag_prof_bytes(R, A));   // [3][2][CB]
    uint8_t *gbuf = lds + diag_prof_bytes(R, A) + 3 * 2 * CB * 2 + g * kDiagBuf;
    const int tstar = (LA - 1) / R;                // lane holding row LA
    const int istar = (LA - 1) % R;

    for (uint32_t k = pbeg; k < pend + 2; ++k) {
        __syncthreads();   // the previous pair's DP has finished reading the profile
        if (k < pend) {
            const int32_t a0 = V.rpairs[2 * k], a1 = V.rpairs[2 * k + 1];
            const uint8_t *su = V.bsym + (int64_t)a0 * V.WB;
            const uint8_t *su2 = V.bsym + (int64_t)(a1 >= 0 ? a1 : a0) * V.WB;
            for (int e = tid; e < (A + 1) * ROWS; e += kThreads) {
                const int c = e / ROWS, i = e - c * ROWS;
                uint32_t val;
                if (c == A)
                    val = kSentinelPair;
                else if (i < LA)
                    val = (uint32_t)V.wtab[(int)su[i] * A + c] | ((uint32_t)V.wtab[(int)su2[i] * A + c] << 16);
                else
                    val = 0;
                prof[c * S + i] = val;
            }
        }
        if (k >= pbeg + 2) {
            const uint32_t kk = k - 2;
            const int16_t *srow = stg + (size_t)(kk % 3) * 2 * CB;
            for (int h = 0; h < 2; ++h) {
                const int32_t slot = V.rpairs[2 * kk + h];
                if (slot < 0) continue;
                const int64_t u = I0 + V.bcol[slot];
                const int64_t jstart = (r == b) ? u + 1 : J0;
                store_row(V, u, LA, jstart, J1, srow + h * CB + (jstart - J0), idx_begin, idx_end, out, out_kind, E);
            }
        }
        __syncthreads();
        if (k >= pend) continue;
        const int32_t a1 = V.rpairs[2 * k + 1];
        int16_t *sdst = stg + (size_t)(k % 3) * 2 * CB;
        for (int64_t c0 = 0; c0 < CB; c0 += kThreads / kDiagLanes) {
            const int64_t slot = J0 + c0 + g;
            const int lb = V.blen[slot];
            const int lbmax_w = __builtin_amdgcn_readlane(lb, 63);   // slots ascend in length
            // the group's word between sentinels: gbuf[16 + j] = B[j]
            for (int q = t; q < kDiagBuf; q += kDiagLanes) {
                const int j = q - 16;
                gbuf[q] = (j >= 0 && j < lb) ? V.bsym[slot * V.WB + j] : (uint8_t)A;
            }
            h2 col[R];
#pragma unroll
            for (int i = 0; i < R; ++i) col[i] = h2{0, 0};
            uint32_t last = 0, diag_in = 0;
            const int steps = lbmax_w + kDiagLanes - 1;
            for (int s = 0; s < steps; ++s) {
                const uint32_t sym = gbuf[16 + s - t];
                const u32x4 *row = reinterpret_cast<const u32x4 *>(prof + sym * S + t * R);
                u32x4 w[(R + 3) / 4];
#pragma unroll
                for (int q = 0; q < (R + 3) / 4; ++q) w[q] = row[q];
                const uint32_t up_in = dpp_row_shr1(last);
                h2 d = as_h2(diag_in);
                h2 up = as_h2(up_in);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const h2 v = max3(d + as_h2(w[i >> 2][i & 3]), col[i], up);
                    d = col[i];
                    col[i] = v;
                    up = v;
                }
                last = __builtin_bit_cast(uint32_t, col[R - 1]);
                diag_in = up_in;
            }
            // row LA of the final column lives in lane tstar, register istar
            h2 res = col[0];
#pragma unroll
            for (int i = 1; i < R; ++i) res = (i == istar) ? col[i] : res;
            const int col_idx = V.bcol[slot];
            if (t == tstar && col_idx != 0xFFFF) {
                const int off = V.gap * (LA + lb);
                sdst[col_idx] = (int16_t)((int)res[0] + off);
                if (a1 >= 0) sdst[CB + col_idx] = (int16_t)((int)res[1] + off);
            }
        }
    }
    (void)lane;
}

}  // namespace nw
