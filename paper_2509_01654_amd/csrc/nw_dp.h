// nw_dp.h -- the inner Needleman-Wunsch recurrence used by every tiled kernel.
//
// Algorithm 1 of the paper (Section 2) fills M[i][j] = max(M[i-1][j-1] +
// sim(A_{i-1}, B_{j-1}), M[i-1][j] + p, M[i][j-1] + p) with M[i][0] = p*i and
// M[0][j] = p*j, and returns M[len A][len B].
//
// The kernels run the same recurrence on G[i][j] = M[i][j] - p*(i+j):
//   G[i][0] = G[0][j] = 0,
//   G[i][j] = max(G[i-1][j-1] + w(A_{i-1}, B_{j-1}), G[i-1][j], G[i][j-1]),
//   w(x, y) = sim(x, y) - 2p,
//   score   = G[len A][len B] + p*(len A + len B).
// Substituting M = G + p(i+j) into the three candidates shows they are the
// same three candidates shifted by the same amount p(i+j), so the maxima agree
// cell by cell.  The up and left candidates no longer need an add, and one
// three-input max finishes a cell: one packed add and one packed max3 per two
// cells.
//
// Every G value is an integer in [0, L * max(w)] (a path adds w on diagonal
// steps only, and at most L of those), so the cells are held as binary16:
// every integer of magnitude <= 2048 is exact in binary16, sums of two such
// integers whose result stays <= 2048 in magnitude are exact, and max is
// exact.  The host refuses a dictionary whose bound exceeds 2048 (NW_ERANGE),
// so no cell is ever rounded.  Two independent pairs share one 32-bit
// register: the low half belongs to the pair (u, v), the high half to (u', v),
// where u and u' are two row words of equal length LA and v is the lane's word.
//
// Similarity comes from a profile in LDS: row c (one per symbol of the
// alphabet) holds LA dwords, dword i = (w(u_i, c), w(u'_i, c)) as two binary16.
// A lane whose word has symbol c in column j reads row c -- ceil(LA/4) 16-byte
// LDS reads per column -- instead of computing LA comparisons.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace nw {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ h2 as_h2(uint32_t x) { return __builtin_bit_cast(h2, x); }

__device__ __forceinline__ h2 max3(h2 a, h2 b, h2 c)
{
    // lowers to v_pk_maximum3_f16 on gfx950
    return __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), c);
}

// Symbol j of a word held as little-endian bytes in 32-bit registers.
template <int NW>
__device__ __forceinline__ uint32_t sym_at(const uint32_t (&bw)[NW], int j)
{
    return __builtin_amdgcn_ubfe(bw[j >> 2], (j & 3) * 8, 8);
}

// LDS byte addresses as plain integers: the address of a __shared__ object,
// and typed pointers at an address.
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) u32x4 lds_u32x4;
__device__ __forceinline__ uint32_t lds_addr_of(const void *p)
{
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint8_t *)p;
}
__device__ __forceinline__ lds_u32 *lds_ptr(uint32_t addr) { return (lds_u32 *)(uintptr_t)addr; }
__device__ __forceinline__ lds_u16 *lds_ptr16(uint32_t addr) { return (lds_u16 *)(uintptr_t)addr; }
__device__ __forceinline__ lds_u8 *lds_ptr8(uint32_t addr) { return (lds_u8 *)(uintptr_t)addr; }

// A wave-uniform value kept in a vector register: the profile base then
// enters the per-column address multiply-add as its vector operand, beside
// the row stride in a scalar register (one multiply-add per column, with no
// copy of the base into a vector register each time).
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// The NQ 16-byte units of the profile row at LDS address `row`, QS bytes apart.
template <int NQ, int QS = 16>
__device__ __forceinline__ void load_row(u32x4 (&dst)[NQ], uint32_t row)
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) dst[q] = *(const lds_u32x4 *)(uintptr_t)(row + q * QS);
}

// Run the DP of two row words (profile `prof`, LA symbols each) against the
// lane's word (bytes in bw, lb symbols) and return G[LA][lb] for both halves.
// lbmin_w / lbmax_w are wave-uniform bounds on lb over the wave's lanes.
// Every lane runs lbmax_w columns (a lane past its own length computes
// columns it ignores); a lane's result is captured when its last column is
// done, which only has to be tested for columns >= lbmin_w.  Keeping the
// column sequence free of divergent branches lets the compiler rotate the
// registers of col[] freely instead of moving values back every column.
// Compile-time loop: f(integral_constant<int, J>) for J = J0 .. N-1 while f
// returns true.  Keeps every column index a constant after inlining, so the
// word bytes and the two profile buffers are addressed statically.
template <int J, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (J < N) {
        if (!f(std::integral_constant<int, J>{})) return;
        static_for<J + 1, N>(f);
    }
}

// Run the DP of two row words (profile `prof`, LA symbols each) against the
// lane's word (bytes in bw) for lbmax_w columns, lbmax_w wave-uniform, and
// return G[LA][len] for both halves.
//
// Lane words are padded with a sentinel symbol whose profile row is -2048 in
// every position.  A column of that symbol leaves the whole DP column
// unchanged: its diagonal candidate G + (-2048) is <= 0 <= every G, so each
// cell takes max(G[i][j], G[i-1][j+1]), and since G is non-decreasing down a
// column this equals G[i][j].  So every lane simply runs the wave's longest
// word and ends with G[LA][its own length], with no per-lane branch inside
// the column sequence; the compiler then rotates the registers of col[]
// freely instead of moving values back every column.
template <int LA, int LBMAX, int QS = 16>
__device__ __forceinline__ h2 dp_lane(const uint32_t (&bw)[LBMAX / 4], int lbmax_w, const uint8_t *prof,
                                      uint32_t stride_b)
{
    constexpr int NQ = (LA + 3) / 4;
    h2 col[LA];
#pragma unroll
    for (int i = 0; i < LA; ++i) col[i] = h2{0, 0};

    const uint32_t pb = in_vgpr(lds_addr_of(prof));
    u32x4 wa[NQ], wb[NQ];
    load_row<NQ, QS>(wa, pb + sym_at(bw, 0) * stride_b);
    static_for<0, LBMAX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j >= lbmax_w) return false;
        u32x4(&cur)[NQ] = (j & 1) ? wb : wa;
        u32x4(&nxt)[NQ] = (j & 1) ? wa : wb;
        // prefetch the profile row of the next column (past the end of a word
        // the bytes are the sentinel, a valid row, so the read is in bounds)
        if constexpr (j + 1 < LBMAX) load_row<NQ, QS>(nxt, pb + sym_at(bw, j + 1) * stride_b);
        // column j+1 of G: cell i+1 = max3(G[i][j] + w, G[i+1][j], G[i][j+1])
        h2 t = as_h2(cur[0][0]);   // G[0][j] = 0, plus w of row 0
        h2 up = h2{0, 0};          // G[0][j+1] = 0
        if constexpr (j == 0) {
            // the first column: G[i][0] = 0, so the diagonal candidates are
            // the weights themselves and the left ones are 0
#pragma unroll
            for (int i = 0; i < LA; ++i) {
                const h2 v = max3(as_h2(cur[i >> 2][i & 3]), h2{0, 0}, up);
                col[i] = v;
                up = v;
            }
            return true;
        }
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            // the diagonal candidate of the next cell uses the old col[i]
            h2 tn = h2{0, 0};
            if (i + 1 < LA) tn = col[i] + as_h2(cur[(i + 1) >> 2][(i + 1) & 3]);
            const h2 v = max3(t, col[i], up);
            col[i] = v;
            up = v;
            t = tn;
        }
        return true;
    });
    return col[LA - 1];
}

// The DP of two row pairs at once: (u, u') from the profile half at prof and
// (v, v') from the half at prof + off_b, both against the lane's word.  Row c
// of the two-pair profile holds both halves, so one address per column serves
// both pairs' reads (the second through the instruction's offset field).
// Returns G[LA][len] of the first pair in ga, of the second in gb.
template <int LA, int LBMAX, uint32_t OFF_B>
__device__ __forceinline__ void dp_lane2(const uint32_t (&bw)[LBMAX / 4], int lbmax_w, const uint8_t *prof,
                                         uint32_t stride_b, h2 &ga, h2 &gb)
{
    constexpr int NQ = (LA + 3) / 4;
    h2 ca[LA], cb[LA];
#pragma unroll
    for (int i = 0; i < LA; ++i) ca[i] = cb[i] = h2{0, 0};

    const uint32_t pb = in_vgpr(lds_addr_of(prof));
    u32x4 wa[NQ], wb[NQ];
    static_for<0, LBMAX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j >= lbmax_w) return false;
        const uint32_t row = pb + sym_at(bw, j) * stride_b;
        load_row(wa, row);
        load_row(wb, row + OFF_B);
        if constexpr (j == 0) {
            h2 ua = h2{0, 0}, ub = h2{0, 0};
#pragma unroll
            for (int i = 0; i < LA; ++i) {
                ca[i] = ua = max3(as_h2(wa[i >> 2][i & 3]), h2{0, 0}, ua);
                cb[i] = ub = max3(as_h2(wb[i >> 2][i & 3]), h2{0, 0}, ub);
            }
            return true;
        }
        h2 ta = as_h2(wa[0][0]), tb = as_h2(wb[0][0]);
        h2 ua = h2{0, 0}, ub = h2{0, 0};
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            h2 tna = h2{0, 0}, tnb = h2{0, 0};
            if (i + 1 < LA) {
                tna = ca[i] + as_h2(wa[(i + 1) >> 2][(i + 1) & 3]);
                tnb = cb[i] + as_h2(wb[(i + 1) >> 2][(i + 1) & 3]);
            }
            ca[i] = ua = max3(ta, ca[i], ua);
            cb[i] = ub = max3(tb, cb[i], ub);
            ta = tna;
            tb = tnb;
        }
        return true;
    });
    ga = ca[LA - 1];
    gb = cb[LA - 1];
}

}  // namespace nw
