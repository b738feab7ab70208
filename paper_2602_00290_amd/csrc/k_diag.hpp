// Diagnostics kernels over the first core.
//
// k_unfold_gram: the FP64 Gram matrix A^T A of the (N_X) x (N_nu ldz) unfolding
// of Z (row x = the cell's N_nu consecutive rows of Z, contiguous), from which
// the host forms the internal delta-ranks of the combined core (the
// discussion of the internal structure of Z).  A launch covers the output
// rows [lo, hi): block (x, y) computes the 64 x 64 tile (lo / 64 + y, x) when
// x >= lo / 64 + y (upper triangle; the other blocks exit) and writes its rows
// inside [lo, hi) to out, rows counted from lo.  It runs over all cells in
// chunks of 32, staging both column ranges of the chunk in LDS (FP64), each
// thread accumulating a 4 x 4 register tile.  No partials: the sum over cells
// runs in one fixed order.
#pragma once

#include "tt_common.hpp"

namespace ttrt {

template <typename T>
__global__ __launch_bounds__(256) void k_unfold_gram(const T* __restrict__ Z, long long n_rows, int n, int lo, int hi,
                                                     double* __restrict__ out) {
    constexpr int TILE = 64, CH = 32;
    __shared__ double Ai[CH][TILE + 1], Aj[CH][TILE + 1];
    const int ti = lo / TILE + (int)blockIdx.y, tj = (int)blockIdx.x;
    if (tj < ti) return;   // lower triangle: uniform over the block
    const int i0 = TILE * ti, j0 = TILE * tj;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;   // 4 x 4 tile at (4 ty, 4 tx)
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (long long r0 = 0; r0 < n_rows; r0 += CH) {
        for (int idx = threadIdx.x; idx < CH * TILE; idx += 256) {
            const int rr = idx / TILE, cc = idx - rr * TILE;
            const long long row = r0 + rr;
            const bool ok = row < n_rows;
            Ai[rr][cc] = (ok && i0 + cc < n) ? (double)Z[row * n + i0 + cc] : 0.0;
            Aj[rr][cc] = (ok && j0 + cc < n) ? (double)Z[row * n + j0 + cc] : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < CH; ++rr) {
            double x[4], y[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) x[a] = Ai[rr][4 * ty + a];
#pragma unroll
            for (int b = 0; b < 4; ++b) y[b] = Aj[rr][4 * tx + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + 4 * ty + a, j = j0 + 4 * tx + b;
            if (i >= lo && i < hi && j < n) out[(size_t)(i - lo) * n + j] = acc[a][b];
        }
}

}  // namespace ttrt
