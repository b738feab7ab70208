// Split-BF16 contractions on gfx950 MFMA (precision TT_PREC_BF16X).
//
// Each FP32 operand x is split as x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (both round-to-nearest; x - hi is exact in FP32), and a
// product is formed from three bf16 MFMA products hi*hi + hi*lo + lo*hi with
// FP32 accumulation; the dropped lo*lo term and the split residual are below
// 2^-16 of |x||y|.
//
// v_mfma_f32_16x16x32_bf16 lane layout (64 lanes):
//   A[i][k] from lane i + 16 (k / 8), element k % 8 (8 bf16 per lane);
//   B[k][j] from lane j + 16 (k / 8), element k % 8;
//   D[i][j] in lane j + 16 (i / 4), register i % 4.
#pragma once

#include "k_mfma.hpp"

namespace ttrt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4b __attribute__((ext_vector_type(4)));

constexpr int kBxKC = 32;   // K depth of one bf16 MFMA and of one staged chunk

// Operand split for k_gemm_bf16x: G (K x N, row-major, leading dimension
// ldg; K and N read from the state by `which`) into hi and lo bf16 arrays in
// the layout [chunk kc][column n < NP][32], zero beyond K and N.
//   which = 0: the gather operand (K = st->kall, N = ldg = st->ldb)
//   which = 1: the output operand V_r (K = st->ldb, N = ldg = st->ldzn)
__global__ __launch_bounds__(256) void k_split_bf16(const DevState* __restrict__ st, int which, const float* __restrict__ G,
                                                    int NP, int kc_cap, __bf16* __restrict__ hi, __bf16* __restrict__ lo) {
    const int K = which == 0 ? st->kall : st->ldb;
    const int ldg = which == 0 ? st->ldb : st->ldzn;
    const int n_kc = (K + kBxKC - 1) / kBxKC;
    const long long total = (long long)n_kc * NP * kBxKC;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int kk = (int)(idx % kBxKC);
        const long long t = idx / kBxKC;
        const int n = (int)(t % NP), kc = (int)(t / NP);
        const int k = kc * kBxKC + kk;
        const float x = (k < K && n < ldg) ? G[(size_t)k * ldg + n] : 0.0f;
        const __bf16 h = (__bf16)x;
        hi[idx] = h;
        lo[idx] = (__bf16)(x - (float)h);
    }
    (void)kc_cap;
}

// Split-BF16 gather contraction (same operation as k_gather_gemm<float, MODE>):
//   MODE_PROJECT: B[k,:] = d_k (sum_j Z[nbr_j(k),:] G_j + sum_q z_q(k) G_rank1[q])
//   MODE_OUTPUT:  Z_out = B V_r
// Block: 256 threads = 4 waves x 32 rows (two 16-row tiles) = 128 rows, by
// 16 NCT columns.  K runs in chunks of 32: the A chunk (gathered, scaled by
// d, rank-1 values in the last chunk) is staged in LDS as FP32 and split per
// lane; the operand chunk (pre-split) is copied to LDS column-major.
template <int MODE, int NCT>
__global__ __launch_bounds__(256) void k_gemm_bf16x(Geom g, OpDesc op, const DevState* __restrict__ st,
                                                     const float* __restrict__ A, const __bf16* __restrict__ Ghi,
                                                     const __bf16* __restrict__ Glo, float* __restrict__ Out,
                                                     RowData rd) {
    constexpr int BM = 128, NP = 16 * NCT, LDA = kBxKC + 4, LDG = kBxKC + 8;
    __shared__ __align__(16) float As[BM * LDA];
    __shared__ __align__(16) __bf16 Bh[NP * LDG];
    __shared__ __align__(16) __bf16 Bl[NP * LDG];
    __shared__ long long nbr[kMaxTerms + 1][BM];
    __shared__ float rowd[BM];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const long long row0 = (long long)blockIdx.x * BM;
    int lda, K, KG, ldo, nblk, kper;
    if (MODE == MODE_PROJECT) {
        lda = st->ldz; kper = st->ldz; nblk = op.n_gather; KG = nblk * kper; K = st->kall; ldo = st->ldb;
    } else {
        lda = st->ldb; kper = st->ldb; nblk = 1; KG = kper; K = kper; ldo = st->ldzn;
    }
    for (int idx = tid; idx < nblk * BM; idx += 256) {
        const int j = idx / BM, i = idx % BM;
        const long long k = row0 + i;
        long long src = -1;
        if (k < g.M) src = (MODE == MODE_OUTPUT || j == 0) ? k : neighbour_row(g, k, op.gaxis[j], op.gdir[j]);
        nbr[j][i] = src;
    }
    if (tid < BM) {
        const long long k = row0 + tid;
        rowd[tid] = (MODE == MODE_PROJECT && k < g.M) ? (float)row_scale(g, op, rd, k) : 1.0f;
    }
    f32x4b acc[2][NCT];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int c = 0; c < NCT; ++c) acc[rt][c] = (f32x4b){0.f, 0.f, 0.f, 0.f};
    const int n_kc = (K + kBxKC - 1) / kBxKC;
    const int q = l >> 4, m = l & 15;
    static_assert(NP * 4 <= 512, "at most two 16-byte operand slots per thread");
    constexpr bool G2 = NP * 4 > 256;   // second 16-byte operand slot per thread (hi and lo each)
    // registers holding the next chunk while the current one computes
    float4 ra[4];
    uint4 gh0 = make_uint4(0, 0, 0, 0), gl0 = gh0, gh1 = gh0, gl1 = gh0;
    auto fetch = [&](int kc) __attribute__((always_inline)) {
        const int k0 = kc * kBxKC;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int slot = tid + 256 * it;
            const int r = slot >> 3, c4 = (slot & 7) * 4;
            const int k = k0 + c4;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            const long long rowk = row0 + r;
            if (k < KG) {
                const int j = k / kper, cc = k - j * kper;
                const long long src = nbr[j][r];
                if (src >= 0) v = *reinterpret_cast<const float4*>(A + src * (long long)lda + cc);
            } else if (MODE == MODE_PROJECT && k < K && rowk < g.M) {
                float t[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int qq = k - KG + e;
                    if (qq < op.n_r1) t[e] = (float)rank1_value(g, op, rd, rowk, qq);
                }
                v = make_float4(t[0], t[1], t[2], t[3]);
            }
            ra[it] = v;
        }
        const uint4* sh = reinterpret_cast<const uint4*>(Ghi + (size_t)kc * NP * kBxKC);
        const uint4* sl = reinterpret_cast<const uint4*>(Glo + (size_t)kc * NP * kBxKC);
        if (tid < NP * 4) {
            gh0 = sh[tid];
            gl0 = sl[tid];
        }
        if constexpr (G2) {
            gh1 = sh[tid + 256];
            gl1 = sl[tid + 256];
        }
    };
    __syncthreads();
    if (n_kc > 0) fetch(0);
    for (int kc = 0; kc < n_kc; ++kc) {
        __syncthreads();   // the previous chunk's readers are done
        // A chunk (scaled by d) and operand chunk (hi, lo; column-major) into LDS
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int slot = tid + 256 * it;
            const int r = slot >> 3, c4 = (slot & 7) * 4;
            const float d = rowd[r];
            const float4 v = ra[it];
            *reinterpret_cast<float4*>(As + r * LDA + c4) = make_float4(v.x * d, v.y * d, v.z * d, v.w * d);
        }
        if (tid < NP * 4) {
            const int n = tid >> 2, part = tid & 3;
            *reinterpret_cast<uint4*>(Bh + n * LDG + part * 8) = gh0;
            *reinterpret_cast<uint4*>(Bl + n * LDG + part * 8) = gl0;
        }
        if constexpr (G2) {
            const int idx = tid + 256;
            const int n = idx >> 2, part = idx & 3;
            *reinterpret_cast<uint4*>(Bh + n * LDG + part * 8) = gh1;
            *reinterpret_cast<uint4*>(Bl + n * LDG + part * 8) = gl1;
        }
        __syncthreads();
        if (kc + 1 < n_kc) fetch(kc + 1);   // in flight while this chunk computes
        // A operand of both row tiles, split into hi / lo
        bf16x8 ah[2], al[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const float* ap = As + (32 * w + 16 * rt + m) * LDA + 8 * q;
            const float4 x0 = *reinterpret_cast<const float4*>(ap);
            const float4 x1 = *reinterpret_cast<const float4*>(ap + 4);
            const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 h = (__bf16)xs[e];
                ah[rt][e] = h;
                al[rt][e] = (__bf16)(xs[e] - (float)h);
            }
        }
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(Bh + (16 * c + m) * LDG + 8 * q);
            const bf16x8 bl = *reinterpret_cast<const bf16x8*>(Bl + (16 * c + m) * LDG + 8 * q);
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rt], bh, acc[rt][c], 0, 0, 0);
                acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rt], bl, acc[rt][c], 0, 0, 0);
                acc[rt][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rt], bh, acc[rt][c], 0, 0, 0);
            }
        }
    }
    // D[i][j] of row tile rt: row 32 w + 16 rt + 4 q + r, column 16 c + m
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long row = row0 + 32 * w + 16 * rt + 4 * q + r;
            if (row >= g.M) continue;
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const int col = 16 * c + m;
                if (col < ldo) Out[row * ldo + col] = acc[rt][c][r];
            }
        }
}

}  // namespace ttrt
