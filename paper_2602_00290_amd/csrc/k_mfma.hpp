// MFMA kernels for FP32-stored first cores on gfx950.
//
// Lane layouts (per wave of 64 lanes, checked against a host product):
//   v_mfma_f32_32x32x2f32:  A[i][k] from lane i + 32k, B[k][j] from lane j + 32k,
//                           D[i][j] in lane j + 32*((i/4)%2), register 4*(i/8) + i%4.
//   v_mfma_f64_16x16x4f64:  A[i][k] from lane i + 16k, B[k][j] from lane j + 16k,
//                           D[i][j] in lane j + 16*(i%4), register i/4.
#pragma once

#include "k_big.hpp"

namespace ttrt {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// out[i] = (float)in[i], i < n.
__global__ __launch_bounds__(256) void k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

// FP32 gather contraction on MFMA (same operation as k_gather_gemm<float, MODE>):
//   MODE_PROJECT: B[k,:] = d_k (sum_j Z[nbr_j(k),:] G_j + sum_q z_q(k) G_rank1[q])
//   MODE_OUTPUT:  Z_out = B V_r
//   MODE_ANGLE:   Y = Z W for the direction-space projection: Y's group-major
//                 row grp N_X + cell from Z's row cell G + grp, rows ldb + kYPad
//                 apart (Gop = W, N_r1 x ldb)
// A pass in direction space leaves B group-major: the gathered projection
// then stands aside, and the output forms the state's row cell G + grp from
// B's row grp N_X + cell (gathered reads, contiguous writes: 4.55 -> 4.26 ms
// on the 3D workload against the other way round).
// Block: 128 rows x BN columns, 4 waves of 32 rows each; K staged in chunks of
// 32 through LDS (row stride 33 floats: conflict-free column reads).
template <int MODE, int BN>
__global__ __launch_bounds__(256) void k_gemm_f32_mfma(Geom g, OpDesc op, const DevState* __restrict__ st,
                                                        const float* __restrict__ A, const float* __restrict__ Gop,
                                                        float* __restrict__ Out, RowData rd) {
    constexpr int BM = 128, KC = 32, NB = BN / 32;
    __shared__ float As[BM][KC + 1];
    __shared__ float Gs[KC][BN + 4];
    __shared__ long long nbr[1 + kMaxTerms][BM];
    __shared__ float rowd[BM];
    __shared__ float rowz[kMaxBC + 1][BM];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const long long row0 = (long long)blockIdx.x * BM;
    const int col0 = blockIdx.y * BN;
    if (MODE == MODE_PROJECT && st->stencil) return;
    if (MODE == MODE_ANGLE && !st->stencil) return;
    int lda, ldg, ldo, nblk, kper;
    if (MODE == MODE_PROJECT) {
        lda = st->ldz; kper = st->ldz; ldg = st->ldb; ldo = st->ldb; nblk = op.n_gather;
    } else if (MODE == MODE_ANGLE) {
        lda = st->ldz; kper = st->ldz; ldg = st->ldb; ldo = st->ldb + kYPadF; nblk = 1;
    } else {
        lda = st->ldb; kper = st->ldb; ldg = st->ldzn; ldo = st->ldzn; nblk = 1;
    }
    const int ncol = MODE == MODE_ANGLE ? st->ldb : ldo;   // columns formed
    if (col0 >= ncol) return;
    const int NXc = (int)(g.M / g.G);
    for (int idx = tid; idx < nblk * BM; idx += 256) {
        const int j = idx / BM, i = idx % BM;
        const long long k = row0 + i;
        long long src = -1;
        if (k < g.M) {
            if (MODE == MODE_ANGLE) {
                const int grp = (int)(k / NXc), cell = (int)(k - (long long)grp * NXc);
                src = (long long)cell * g.G + grp;
            } else if (MODE == MODE_OUTPUT && st->stencil) {
                // state row k = cell G + grp reads B's group-major row grp N_X + cell
                const int cell = (int)(k / g.G), grp = (int)(k - (long long)cell * g.G);
                src = (long long)grp * NXc + cell;
            } else {
                src = (MODE == MODE_OUTPUT || j == 0) ? k : neighbour_row(g, k, op.gaxis[j], op.gdir[j]);
            }
        }
        nbr[j][i] = src;
    }
    if (MODE == MODE_PROJECT && tid < BM) {
        const long long k = row0 + tid;
        if (k < g.M) {
            rowd[tid] = (float)row_scale(g, op, rd, k);
            for (int q = 0; q < op.n_r1; ++q) rowz[q][tid] = (float)rank1_value(g, op, rd, k, q);
        }
    }
    f32x16 acc[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
    __syncthreads();
    for (int j = 0; j < nblk; ++j) {
        for (int k0 = 0; k0 < kper; k0 += KC) {
            // A chunk: 128 rows x 32 floats as 4-float groups (kper is a multiple of 8)
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const int idx = tid + 256 * it;
                const int r = idx >> 3, c4 = (idx & 7) * 4;
                const long long src = nbr[j][r];
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (src >= 0 && k0 + c4 < kper) v = *reinterpret_cast<const float4*>(A + src * (long long)lda + k0 + c4);
                As[r][c4 + 0] = v.x;
                As[r][c4 + 1] = v.y;
                As[r][c4 + 2] = v.z;
                As[r][c4 + 3] = v.w;
            }
            // G chunk: 32 x BN
            for (int idx = tid; idx < KC * (BN / 4); idx += 256) {
                const int kk = idx / (BN / 4), c4 = (idx % (BN / 4)) * 4;
                const int grow = j * kper + k0 + kk;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (k0 + kk < kper) {
                    const float* gp = Gop + (long long)grow * ldg + col0 + c4;
                    if (col0 + c4 + 3 < ldg) {
                        v = make_float4(gp[0], gp[1], gp[2], gp[3]);
                    } else {
                        if (col0 + c4 + 0 < ldg) v.x = gp[0];
                        if (col0 + c4 + 1 < ldg) v.y = gp[1];
                        if (col0 + c4 + 2 < ldg) v.z = gp[2];
                    }
                }
                Gs[kk][c4 + 0] = v.x;
                Gs[kk][c4 + 1] = v.y;
                Gs[kk][c4 + 2] = v.z;
                Gs[kk][c4 + 3] = v.w;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < KC / 2; ++kk) {
                const float a = As[32 * w + (l & 31)][2 * kk + (l >> 5)];
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    const float b = Gs[2 * kk + (l >> 5)][32 * c + (l & 31)];
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
                }
            }
            __syncthreads();
        }
    }
    // epilogue: D[i][j] of wave w sits in lane j + 32*((i/4)%2), register 4*(i/8) + i%4
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int col = col0 + 32 * c + (l & 31);
        if (col >= ncol) continue;
        float g1[kMaxBC + 1];
        if (MODE == MODE_PROJECT) {
            const int base = op.n_gather * kper;
            for (int q = 0; q < op.n_r1; ++q) g1[q] = Gop[(long long)(base + q) * ldg + col];
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
            const int il = 32 * w + i;
            const long long k = row0 + il;
            if (k >= g.M) continue;
            float v = acc[c][r];
            if (MODE == MODE_PROJECT) {
                for (int q = 0; q < op.n_r1; ++q) v += rowz[q][il] * g1[q];
                v *= rowd[il];
            }
            Out[k * ldo + col] = v;
        }
    }
}

// FP64 Gram matrix of an FP32 first core on FP64 MFMA: G = B^T B over each
// block's rows (64 x 64, only the 10 upper 16 x 16 blocks are formed; the
// products of FP32 values are exact in FP64).  Each wave takes 4 rows per
// MFMA step; the 4 waves of a block add their partial blocks through LDS and
// the block writes its full symmetric partial to Gout[blockIdx.x].
__global__ __launch_bounds__(256) void k_gram_f64_mfma(const float* __restrict__ B, const DevState* __restrict__ st,
                                                       long long nrows, long long rows_per_block,
                                                       double* __restrict__ Gout) {
    __shared__ double Gs[64][65];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int ncols = st->k1, ldb = st->ldb;
    const long long begin = (long long)blockIdx.x * rows_per_block;
    long long end = begin + rows_per_block;
    if (end > nrows) end = nrows;
    f64x4 acc[10];
#pragma unroll
    for (int b = 0; b < 10; ++b) acc[b] = (f64x4){0.0, 0.0, 0.0, 0.0};
    const int col = l & 15, kr = l >> 4;
    float nxt[4];
    {
        const long long row = begin + 4 * w + kr;
#pragma unroll
        for (int gidx = 0; gidx < 4; ++gidx) {
            const int c = 16 * gidx + col;
            nxt[gidx] = (row < end && c < ncols) ? B[row * ldb + c] : 0.0f;
        }
    }
    for (long long k0 = begin + 4 * w; k0 < end; k0 += 16) {
        double v[4];
#pragma unroll
        for (int gidx = 0; gidx < 4; ++gidx) v[gidx] = (double)nxt[gidx];
        {   // prefetch the next group of 4 rows of this wave
            const long long row = k0 + 16 + kr;
#pragma unroll
            for (int gidx = 0; gidx < 4; ++gidx) {
                const int c = 16 * gidx + col;
                nxt[gidx] = (row < end && c < ncols) ? B[row * ldb + c] : 0.0f;
            }
        }
        int b = 0;
#pragma unroll
        for (int gi = 0; gi < 4; ++gi)
#pragma unroll
            for (int gj = gi; gj < 4; ++gj) {
                acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[gi], v[gj], acc[b], 0, 0, 0);
                ++b;
            }
    }
    for (int idx = tid; idx < 64 * 65; idx += 256) (&Gs[0][0])[idx] = 0.0;
    __syncthreads();
    for (int ww = 0; ww < 4; ++ww) {
        if (w == ww) {
            int b = 0;
#pragma unroll
            for (int gi = 0; gi < 4; ++gi)
#pragma unroll
                for (int gj = gi; gj < 4; ++gj) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * gi + (l >> 4) + 4 * r;   // D row (column of B)
                        const int jj = 16 * gj + (l & 15);
                        Gs[i][jj] += acc[b][r];
                    }
                    ++b;
                }
        }
        __syncthreads();
    }
    double* out = Gout + (size_t)blockIdx.x * 64 * 64;
    for (int idx = tid; idx < 64 * 64; idx += 256) {
        const int i = idx / 64, j = idx % 64;
        out[idx] = (i <= j) ? Gs[i][j] : Gs[j][i];
    }
}

}  // namespace ttrt
