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

// Per-row tables of the projection (built once per problem, like the fused
// path's): d in aux[k].x, the rows of gather blocks 1.. in nbr[k * ns + j - 1],
// and the operator's rank-1 columns in R[k * rw + q] (q < rw).
struct BxRows {
    const float2* aux;
    const int* nbr;
    int ns;
    const float* R;
    int rw;
};

// Split-BF16 gather contraction (same operation as k_gather_gemm<float, MODE>):
//   MODE_PROJECT: B[k,:] = d_k (sum_j Z[nbr_j(k),:] G_j + sum_q z_q(k) G_rank1[q])
//   MODE_OUTPUT:  Z_out = B V_r
// Block: 256 threads = 4 waves x 32 rows (two 16-row tiles) = 128 rows, by
// 16 NCT columns.  K runs in chunks of 32: each lane loads its own A fragment
// (gathered rows, rank-1 values in the last chunk) into registers, scales it
// by d and splits it; the operand chunk (pre-split) is copied to LDS
// column-major.  The block's row data (d, neighbour rows, rank-1 values) is
// copied from the per-row tables into LDS at the start; with 32-bit row
// indices, registers and LDS allow three waves per SIMD (the kernel waits on
// its loads).
template <int MODE, int NCT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void k_gemm_bf16x(Geom g, OpDesc op, const DevState* __restrict__ st,
                  const float* __restrict__ A, const __bf16* __restrict__ Ghi,
                  const __bf16* __restrict__ Glo, float* __restrict__ Out,
                  BxRows rows) {
    constexpr int BM = 128, NP = 16 * NCT, LDG = kBxKC + 8;
    __shared__ __align__(16) __bf16 Bh[NP * LDG];
    __shared__ __align__(16) __bf16 Bl[NP * LDG];
    __shared__ int nbr[kMaxTerms + 1][BM];
    __shared__ float rowd[BM];
    __shared__ float rowz[kMaxBC + 4][BM];   // rank-1 values, zero past n_r1 (read four at a time)
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
        int src = -1;
        if (k < g.M) src = (MODE == MODE_OUTPUT || j == 0) ? (int)k : rows.nbr[k * rows.ns + j - 1];
        nbr[j][i] = src;
    }
    if (tid < BM) {
        const long long k = row0 + tid;
        const bool ok = MODE == MODE_PROJECT && k < g.M;
        rowd[tid] = (ok && op.scale_d) ? rows.aux[k].x : 1.0f;
        if (MODE == MODE_PROJECT)
            for (int qq = 0; qq < kMaxBC + 4; ++qq)
                rowz[qq][tid] = (ok && qq < op.n_r1) ? rows.R[k * rows.rw + qq] : 0.0f;
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
    const FastDiv dkp(kper);   // gather block of a K index (exact: K < 2^22)
    // registers holding the next chunk while the current one computes
    float4 ra[4];
    uint4 gh0 = make_uint4(0, 0, 0, 0), gl0 = gh0, gh1 = gh0, gl1 = gh0;
    auto fetch = [&](int kc) __attribute__((always_inline)) {
        const int k0 = kc * kBxKC;
        // this lane's A fragment (row m of each row tile, columns 8 q .. 8 q + 7
        // of the chunk) straight into registers: an 8-column segment never
        // crosses a gather block (ld is a multiple of 8)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int r = 32 * w + 16 * rt + m;
            const int k = k0 + 8 * q;
            float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
            if (k < KG) {
                const int j = dkp.q(k), cc = k - j * kper;
                const long long src = nbr[j][r];
                if (src >= 0) {
                    const float* ap = A + src * (long long)lda + cc;
                    v0 = *reinterpret_cast<const float4*>(ap);
                    v1 = *reinterpret_cast<const float4*>(ap + 4);
                }
            } else if (MODE == MODE_PROJECT && k < K) {
                const int qq = k - KG;
                v0 = make_float4(rowz[qq][r], rowz[qq + 1][r], rowz[qq + 2][r], rowz[qq + 3][r]);
                v1 = make_float4(rowz[qq + 4][r], rowz[qq + 5][r], rowz[qq + 6][r], rowz[qq + 7][r]);
            }
            ra[2 * rt] = v0;
            ra[2 * rt + 1] = v1;
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
        // operand chunk (hi, lo; column-major) into LDS
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
        // A operand of both row tiles, scaled by d and split into hi / lo
        bf16x8 ah[2], al[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            // the split is of the rounded FP32 products (no contraction of the
            // scaling into the residual x - hi)
#pragma clang fp contract(off)
            const float d = rowd[32 * w + 16 * rt + m];
            const float4 x0 = ra[2 * rt], x1 = ra[2 * rt + 1];
            const float xs[8] = {x0.x * d, x0.y * d, x0.z * d, x0.w * d, x1.x * d, x1.y * d, x1.z * d, x1.w * d};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 h = (__bf16)xs[e];
                ah[rt][e] = h;
                al[rt][e] = (__bf16)(xs[e] - (float)h);
            }
        }
        __syncthreads();
        if (kc + 1 < n_kc) fetch(kc + 1);   // in flight while this chunk computes
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
