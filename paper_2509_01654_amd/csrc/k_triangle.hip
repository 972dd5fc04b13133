// k_triangle.hip -- launchers of the triangle kernels, and the naive kernel.
//
// Naive kernel (k_tri_naive): the paper's GPU scheme (Section 4.2): one thread
// per pair index, a 1-D grid, idx -> (row, column) through the closed form of
// the row index, and one DP per thread with its scratch in shared memory (one
// row of the score matrix instead of the whole matrix).
#include "k_tri_tiled.h"

namespace nw {

template <typename OutT>
__global__ __launch_bounds__(256) void k_tri_naive(DevVocab V, uint64_t idx_begin, uint64_t idx_end, OutT *out)
{
    __shared__ int16_t rows[256][kMaxLen + 1];
    int16_t *row = rows[threadIdx.x];   // this thread's scratch: one row of the score matrix
    const int64_t n = V.n;
    const int gap = V.gap;
    const double z = (double)n - 0.5;
    for (uint64_t idx = idx_begin + (uint64_t)blockIdx.x * 256u + threadIdx.x; idx < idx_end;
         idx += (uint64_t)gridDim.x * 256u) {
        // r = floor(z - sqrt(z^2 - 2 idx)), z = n - 1/2 (Section 4.2), then an
        // integer fix-up so rounding can never pick the wrong row
        int64_t r = (int64_t)floor(z - sqrt(z * z - 2.0 * (double)idx));
        if (r < 0) r = 0;
        if (r > n - 2) r = n - 2;
        while (r > 0 && row_start_idx(n, r) > idx) --r;
        while (r + 1 < n - 1 && row_start_idx(n, r + 1) <= idx) ++r;
        const int64_t c = r + 1 + (int64_t)(idx - row_start_idx(n, r));
        const int la = V.clen[r], lb = V.clen[c];
        const uint8_t *A = V.csym + r * V.WB;
        const uint8_t *B = V.csym + c * V.WB;
        for (int j = 0; j <= lb; ++j) row[j] = (int16_t)(gap * j);
        for (int i = 1; i <= la; ++i) {
            int diag = row[0];
            row[0] = (int16_t)(gap * i);
            const int a = A[i - 1];
            for (int j = 1; j <= lb; ++j) {
                const int bsym = B[j - 1];
                const int sim = V.has_submat ? (int)V.submat[a * V.alphabet + bsym] : (a == bsym ? V.match : V.mismatch);
                const int up = row[j];
                int v = diag + sim;
                v = max(v, up + gap);
                v = max(v, (int)row[j - 1] + gap);
                diag = up;
                row[j] = (int16_t)v;
            }
        }
        out[idx - idx_begin] = (OutT)row[lb];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define X(lo, hi) void nw_tri_fill_##lo(tri_kernel_t *tab);
NW_TRI_SPLITS
#undef X

static const tri_kernel_t *tiled_table()
{
    static tri_kernel_t tab[kMaxLen + 1];
    static bool init = [] {
#define X(lo, hi) nw_tri_fill_##lo(tab);
        NW_TRI_SPLITS
#undef X
        return true;
    }();
    (void)init;
    return tab;
}

hipError_t launch_triangle_tiled(const DevVocab &V, uint64_t idx_begin, uint64_t idx_end, int out_kind, void *d_out,
                                 hipStream_t stream)
{
    if (idx_begin >= idx_end || V.n < 2) return hipSuccess;
    const uint32_t nblk_pairs = (uint32_t)((uint64_t)V.nb * (V.nb + 1) / 2);
    const tri_kernel_t *tab = tiled_table();
    for (int LA = 0; LA <= V.lmax; ++LA) {
        const size_t lds = tri_lds_bytes(LA, V.alphabet, V.CB);
        const void *fn = reinterpret_cast<const void *>(tab[LA]);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        DevVocab Vc = V;
        uint64_t ib = idx_begin, ie = idx_end;
        void *po = d_out;
        int ok = out_kind;
        void *args[] = {&Vc, &ib, &ie, &po, &ok};
        hipError_t e = hipLaunchKernel(fn, dim3(nblk_pairs), dim3(kThreads), args, lds, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_triangle_naive(const DevVocab &V, uint64_t idx_begin, uint64_t idx_end, int out_kind, void *d_out,
                                 hipStream_t stream)
{
    if (idx_begin >= idx_end) return hipSuccess;
    const uint64_t count = idx_end - idx_begin;
    const uint64_t blocks = (count + 255) / 256;
    const uint32_t grid = (uint32_t)(blocks < (1u << 20) ? blocks : (1u << 20));
    if (out_kind == OUT_I8)
        hipLaunchKernelGGL(k_tri_naive<int8_t>, dim3(grid), dim3(256), 0, stream, V, idx_begin, idx_end,
                           (int8_t *)d_out);
    else
        hipLaunchKernelGGL(k_tri_naive<int16_t>, dim3(grid), dim3(256), 0, stream, V, idx_begin, idx_end,
                           (int16_t *)d_out);
    return hipGetLastError();
}

}  // namespace nw
