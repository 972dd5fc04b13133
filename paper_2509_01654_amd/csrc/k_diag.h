// k_diag.h -- intra-pair anti-diagonal triangle kernel for long words.
//
// The stencil the paper points to as the way to parallelise inside one score
// matrix (Section 6: each cell depends on its up, left and up-left
// neighbours, Section 4.2).  A group of 16 lanes (one DPP row) shares one
// column word; lane t owns the R consecutive rows t*R+1 .. t*R+R of the DP
// (the binary16 recurrence G of nw_dp.h, two row words in the two halves).
// At step s lane t processes column s - t, so the 16 lanes work on one
// anti-diagonal band: the cell above a lane's first row is the last row of
// lane t-1 one step earlier, and the diagonal neighbour is that value one step
// before, passed down the group with a DPP row shift (lane 0 of each row
// receives 0, the G[0][j] boundary).  Columns before the start (s - t < 0) and
// past the end of the word read the sentinel symbol, whose profile row leaves
// a DP column unchanged (nw_dp.h), so every lane runs every step with no
// branch.  The column symbols flow down the group the same way: lane t needs
// at step s the symbol lane t-1 had at step s-1, so one DPP row shift per step
// hands them on, and lane 0 takes the next symbol of the word from an aligned
// dword of LDS read once per four steps.
//
// One launch per class R (rows per lane, even): the class takes the row
// lengths LA with 16(R-2) < LA <= 16R, and a workgroup takes a tile
// (block pair r <= b) and a run of the block's row pairs of that class.  The
// two row words of a pair are consecutive words of the class (their lengths
// may differ: each half reads its score at its own row), so a block leaves at
// most one half-empty pair per class.  1024 threads = 64 groups share one
// similarity profile of the current row pair in LDS, laid out so that the
// lanes' reads never meet in an LDS bank whatever symbols they look up (see
// diag_load); profile entries are read one step ahead of the DP.  The score of a pair is row LA of the final
// column.
#pragma once

#include "nw_tile_common.h"

namespace nw {

constexpr int kDiagLanes = 16;                          // lanes per pair
constexpr int kDiagThreads = 1024;                      // threads per workgroup
constexpr int kDiagGroups = kDiagThreads / kDiagLanes;  // column words in flight per workgroup
constexpr int kDiagMaxLen = 255;                        // longest word of the anti-diagonal path
// Group word buffer: the padded word (at most 256 bytes) | 32 sentinels.
constexpr int kDiagBuf = 256 + 32;

// Profile of a class with R rows per lane (R even, 2..16): the first R & ~3
// rows of every lane in 16-byte units (main part), the last two rows of an
// R = 4m+2 class in 8-byte units (tail).  Dwords per symbol:
__host__ __device__ constexpr uint32_t diag_main_dw(int R) { return (uint32_t)(kDiagLanes * (R & ~3)); }
__host__ __device__ constexpr uint32_t diag_tail_dw(int R) { return (R & 2) ? 4u * kDiagLanes : 0u; }
__host__ __device__ constexpr uint32_t diag_prof_bytes(int R, int alphabet)
{
    return (uint32_t)(alphabet + 1) * (diag_main_dw(R) + diag_tail_dw(R)) * 4u;
}
// LDS: one profile, two int16 staging row pairs, the group word buffers.
__host__ __device__ constexpr uint32_t diag_lds_bytes(int R, int alphabet, int CB)
{
    return diag_prof_bytes(R, alphabet) + 2u * 2u * (uint32_t)CB * 2u + (uint32_t)kDiagGroups * kDiagBuf;
}
// Row-length class c (0 <= c < kDiagClasses) takes lengths 32c+1 .. 32c+32 with R = 2(c+1).
__host__ __device__ constexpr int diag_rows_per_lane(int c) { return 2 * (c + 1); }

__device__ __forceinline__ uint32_t dpp_row_shr1(uint32_t v)
{
    // row_shr:1 within rows of 16 lanes; lane 0 of a row reads 0 (bound_ctrl)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t dpp_row_shr1_or(uint32_t first, uint32_t v)
{
    // row_shr:1 within rows of 16 lanes; lane 0 of a row keeps `first`
    return (uint32_t)__builtin_amdgcn_update_dpp((int)first, (int)v, 0x111, 0xF, 0xF, false);
}

// Profile reads of one step.  Main part: the entry of lane t, its row 4q + e
// (0 <= e < 4), symbol c, is dword c*16(R & ~3) + 64q + 4t + e, so the 16
// lanes of a group read 16 consecutive 16-byte units (the 64 banks once) for
// any symbols.  Tail (rows R-2, R-1): symbol c holds two copies of 32 dwords,
// lane t's pair at 2t (+e); group g reads copy g & 1, so the two groups that
// share an 8-byte read pass use opposite halves of the banks.
template <int R>
struct DiagW {
    static constexpr int Q = R / 4;
    u32x4 q[Q > 0 ? Q : 1];
    uint2 tail;
    __device__ __forceinline__ uint32_t operator[](int i) const
    {
        return i < 4 * Q ? q[i >> 2][i & 3] : (i - 4 * Q == 0 ? tail.x : tail.y);
    }
};

template <int R>
__device__ __forceinline__ void diag_load(DiagW<R> &w, const uint32_t *prof_t, const uint32_t *tail_t, uint32_t sym)
{
    const u32x4 *row = reinterpret_cast<const u32x4 *>(prof_t + sym * diag_main_dw(R));
#pragma unroll
    for (int q = 0; q < R / 4; ++q) w.q[q] = row[q * kDiagLanes];
    if constexpr ((R & 2) != 0) w.tail = *reinterpret_cast<const uint2 *>(tail_t + sym * diag_tail_dw(R));
    // issue the reads here, one step before their use: keep the scheduler
    // from sinking them next to the DP that consumes them
    __builtin_amdgcn_sched_barrier(0);
}

template <int R>
__global__ __launch_bounds__(kDiagThreads) void k_tri_diag(DevVocab V, uint64_t idx_begin, uint64_t idx_end,
                                                           void *out, int out_kind, EdgeSink E, uint32_t rb0,
                                                           uint32_t rbn, uint32_t chunks, uint32_t rpc)
{
    static_assert(R % 2 == 0 && R >= 2 && R <= 16, "rows per lane");
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr uint32_t SM = diag_main_dw(R), ST = diag_tail_dw(R);
    constexpr int ROWS = kDiagLanes * R;
    constexpr int R4 = R & ~3;   // rows of a lane in the main part

    uint32_t r, b;
    if (!tile_block_pair(blockIdx.x / chunks, rb0, rbn, V.nb, r, b)) return;
    // the row pairs of block r in this class, cut into runs of rpc
    const uint32_t *dpo = V.dp_off + (size_t)r * kDiagClasses + (R / 2 - 1);
    const uint32_t cbeg = dpo[0], cend = dpo[1];
    const uint64_t pbeg64 = (uint64_t)cbeg + (uint64_t)(blockIdx.x % chunks) * rpc;
    if (pbeg64 >= cend) return;
    const uint32_t pbeg = (uint32_t)pbeg64;
    const uint32_t pend = cend - pbeg <= rpc ? cend : pbeg + rpc;

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
    const int t = tid & (kDiagLanes - 1);   // position in the group
    const int g = tid / kDiagLanes;         // group of the workgroup
    const int A = V.alphabet;
    uint32_t *prof = reinterpret_cast<uint32_t *>(lds);
    int16_t *stg = reinterpret_cast<int16_t *>(lds + diag_prof_bytes(R, A));   // [2][2][CB]
    uint8_t *gbuf_all = lds + diag_prof_bytes(R, A) + 2 * 2 * CB * 2;
    uint8_t *gbuf = gbuf_all + g * kDiagBuf;
    uint32_t *ptail = prof + (size_t)(A + 1) * SM;
    const uint32_t *prof_t = prof + t * 4;
    const uint32_t *tail_t = ptail + (g & 1) * (ST / 2) + 2 * t;
    const uint32_t *gword = reinterpret_cast<const uint32_t *>(gbuf);
    const int wq = V.WB / 16;               // 16-byte units of a padded word

    // every group buffer starts as sentinels; a column only rewrites its word
    {
        const uint32_t sent4 = (uint32_t)A * 0x01010101u;
        uint32_t *p = reinterpret_cast<uint32_t *>(gbuf_all);
        for (int e = tid; e < kDiagGroups * kDiagBuf / 4; e += kDiagThreads) p[e] = sent4;
    }

    for (uint32_t k = pbeg; k <= pend; ++k) {
        __syncthreads();   // the previous DP has finished with the profile and its staging rows
        if (k < pend) {
            const int32_t a0 = V.dpairs[2 * k], a1 = V.dpairs[2 * k + 1];
            const int LA0 = V.blen[a0], LA1 = a1 >= 0 ? V.blen[a1] : 0;
            const uint8_t *su = V.bsym + (int64_t)a0 * V.WB;
            const uint8_t *su2 = V.bsym + (int64_t)(a1 >= 0 ? a1 : a0) * V.WB;
            for (int e = tid; e < (A + 1) * ROWS; e += kDiagThreads) {
                const int c = e / ROWS, i = e - c * ROWS;
                const int lt = i / R, ri = i - lt * R;
                uint32_t val;
                if (c == A) {
                    val = kSentinelPair;
                } else {
                    // rows past a word's length never reach its score row
                    val = i < LA0 ? (uint32_t)V.wtab[(int)su[i] * A + c] : 0u;
                    if (i < LA1) val |= (uint32_t)V.wtab[(int)su2[i] * A + c] << 16;
                }
                if (ri < R4) {
                    prof[c * SM + (ri >> 2) * (4 * kDiagLanes) + lt * 4 + (ri & 3)] = val;
                } else {
                    uint32_t *tp = ptail + c * ST + 2 * lt + (ri - R4);
                    tp[0] = val;
                    tp[ST / 2] = val;
                }
            }
        }
        if (k > pbeg) {
            const uint32_t kk = k - 1;
            const int16_t *srow = stg + (size_t)(kk & 1) * 2 * CB;
            for (int h = 0; h < 2; ++h) {
                const int32_t slot = V.dpairs[2 * kk + h];
                if (slot < 0) continue;
                const int64_t u = I0 + V.bcol[slot];
                const int64_t jstart = (r == b) ? u + 1 : J0;
                store_row<kDiagThreads>(V, u, V.blen[slot], jstart, J1, srow + h * CB + (jstart - J0), idx_begin,
                                        idx_end, out, out_kind, E);
            }
        }
        __syncthreads();
        if (k == pend) break;

        const int32_t a1 = V.dpairs[2 * k + 1];
        const int LA0 = V.blen[V.dpairs[2 * k]], LA1 = a1 >= 0 ? V.blen[a1] : LA0;
        const int tstar0 = (LA0 - 1) / R, istar0 = (LA0 - 1) % R;   // lane and register of row LA0
        const int tstar1 = (LA1 - 1) / R, istar1 = (LA1 - 1) % R;
        int16_t *sdst = stg + (size_t)(k & 1) * 2 * CB;
        // Column words: chunk c holds the 64 slots c*64 .. c*64+63; the four
        // groups of a wavefront take 4 consecutive slots (similar lengths), and
        // the wavefront's quad rotates with c, so that every wavefront meets
        // the same mix of lengths before the next barrier.
        auto slot_of = [&](int64_t c) { return J0 + c * kDiagGroups + (((g >> 2) + c) & 15) * 4 + (g & 3); };
        const int64_t nchunks = CB / kDiagGroups;
        u32x4 wnext = u32x4{0, 0, 0, 0};   // the first column word of this group, prefetched
        if (t < wq) wnext = *reinterpret_cast<const u32x4 *>(V.bsym + slot_of(0) * V.WB + 16 * t);
        for (int64_t c = 0; c < nchunks; ++c) {
            const int64_t slot = slot_of(c);
            if (t < wq) *reinterpret_cast<u32x4 *>(gbuf + 16 * t) = wnext;
            {
                // next column word of the group (clamped to the block: always a valid slot)
                const int64_t ns = slot_of(min(c + 1, nchunks - 1));
                if (t < wq) wnext = *reinterpret_cast<const u32x4 *>(V.bsym + ns * V.WB + 16 * t);
            }
            const int lb = V.blen[slot];
            const int lbmax_w = __builtin_amdgcn_readlane(lb, 63);   // slots of a quad ascend in length
            h2 col[R];
#pragma unroll
            for (int i = 0; i < R; ++i) col[i] = h2{0, 0};
            uint32_t last = 0, diag_in = 0;
            // one step: row i takes its diagonal sum from the old value of row
            // i-1 before the max3 chain overwrites it, so the column updates in place
            auto step = [&](const DiagW<R> &w) __attribute__((always_inline)) {
                const uint32_t up_in = dpp_row_shr1(last);
                h2 a = as_h2(diag_in) + as_h2(w[0]);
                h2 up = as_h2(up_in);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    h2 an = h2{0, 0};
                    if (i + 1 < R) an = col[i] + as_h2(w[i + 1]);
                    col[i] = max3(a, col[i], up);
                    up = col[i];
                    a = an;
                }
                last = __builtin_bit_cast(uint32_t, col[R - 1]);
                diag_in = up_in;
            };
            // symbol of lane t at step s: B[s - t], the sentinel before the word
            // (and past it, from the padding); gword[m] holds B[4m .. 4m+3],
            // read up to byte 4*(steps/4 + 1) + 3 < 256 + 32.  The next dword
            // is read after the second step's profile reads, so that fewer LDS
            // reads than the wait counter tracks separate it from its use.
            const int steps = lbmax_w + kDiagLanes - 1;
            uint32_t dw = gword[0];
            uint32_t sym = t == 0 ? (dw & 0xFFu) : (uint32_t)A;
            DiagW<R> wa, wb;
            diag_load<R>(wa, prof_t, tail_t, sym);
            for (int s = 0; s < steps; s += 4) {
                sym = dpp_row_shr1_or((dw >> 8) & 0xFFu, sym);
                diag_load<R>(wb, prof_t, tail_t, sym);
                step(wa);
                if (s + 1 >= steps) break;
                sym = dpp_row_shr1_or((dw >> 16) & 0xFFu, sym);
                diag_load<R>(wa, prof_t, tail_t, sym);
                const uint32_t dn = gword[(s >> 2) + 1];
                step(wb);
                if (s + 2 >= steps) break;
                sym = dpp_row_shr1_or(dw >> 24, sym);
                diag_load<R>(wb, prof_t, tail_t, sym);
                step(wa);
                if (s + 3 >= steps) break;
                sym = dpp_row_shr1_or(dn & 0xFFu, sym);
                diag_load<R>(wa, prof_t, tail_t, sym);
                step(wb);
                dw = dn;
            }
            // row LA of the final column lives in lane tstar, register istar (per half)
            h2 res0 = col[0], res1 = col[0];
#pragma unroll
            for (int i = 1; i < R; ++i) {
                res0 = (i == istar0) ? col[i] : res0;
                res1 = (i == istar1) ? col[i] : res1;
            }
            const int col_idx = V.bcol[slot];
            if (col_idx != 0xFFFF) {
                if (t == tstar0) sdst[col_idx] = (int16_t)((int)res0[0] + V.gap * (LA0 + lb));
                if (a1 >= 0 && t == tstar1) sdst[CB + col_idx] = (int16_t)((int)res1[1] + V.gap * (LA1 + lb));
            }
        }
    }
}

}  // namespace nw
