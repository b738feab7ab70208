// FP64 Gram matrix of a stored FP32 or FP64 first core with 128 columns (k1
// up to 128) on FP64 MFMA, for the unfused Gram rounding of wide first cores.
#pragma once

#include "k_fused.hpp"

namespace ttrt {

// FP64 Gram matrix of a stored FP32 first core with 128 columns on FP64 MFMA
// (the unfused Gram path for wide cores, k1 up to 128).  A block walks its
// rows in chunks of 64: each chunk is loaded with coalesced 16-byte loads (the
// next chunk's loads are in flight while the current one computes) and staged
// in LDS.  Wave W of the 4 owns the upper 16 x 16 blocks of block rows W and
// 7 - W (9 blocks each, balanced).  Each wave runs its own instantiation of
// the loop with the block rows fixed at compile time, so only its 9
// accumulators are live (three waves per SIMD instead of two); its A operands
// are read from LDS at fixed columns and the B operands of the column groups
// it needs.  Each block writes its compact partial (36 blocks x 4 registers x
// 64 lanes) for k_sum_gram<8>.
// TB is the stored element type (float, or double for FP64 data: 32-row
// chunks, the same LDS bytes).
template <int W, typename TB>
__device__ __forceinline__ void gram_w8_wave(const TB* __restrict__ B, int ldb, long long begin, long long end,
                                             TB* Bs, double* __restrict__ outp) {
    constexpr int NCT = 8;
    constexpr int NC = 16 * NCT;              // columns
    constexpr int VE = 16 / sizeof(TB);       // elements per 16-byte load
    constexpr int CH = 16 * VE;               // rows per chunk: 64 (float), 32 (double)
    constexpr int LDC = NC + 4;               // LDS row stride (elements)
    constexpr int V4 = CH * NC / VE / 256;    // 16-byte loads per thread per chunk
    typedef TB vec_t __attribute__((ext_vector_type(VE)));
    constexpr int GA = W, GB = NCT - 1 - W;   // this wave's two block rows
    constexpr int NA = NCT - GA, NBB = NCT - GB;
    const int tid = threadIdx.x, l = tid & 63;
    f64x4 accA[NA], accB[NBB];
#pragma unroll
    for (int g = 0; g < NA; ++g) accA[g] = (f64x4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < NBB; ++g) accB[g] = (f64x4){0.0, 0.0, 0.0, 0.0};
    vec_t nx[V4];
    auto load = [&](long long r0) {
#pragma unroll
        for (int v = 0; v < V4; ++v) {
            const int slot = tid + 256 * v;
            const int r = slot / (NC / VE), c4 = (slot % (NC / VE)) * VE;
            const long long row = r0 + r;
            vec_t x = (vec_t)(TB)0;
            // columns from k1 up to ldb are zero in B; beyond ldb they are not read
            if (row < end && c4 < ldb) x = *reinterpret_cast<const vec_t*>(B + row * ldb + c4);
            nx[v] = x;
        }
    };
    const int col = l & 15, kr = l >> 4;
    if (begin < end) load(begin);
    for (long long r0 = begin; r0 < end; r0 += CH) {
        __syncthreads();   // the previous chunk's readers are done
#pragma unroll
        for (int v = 0; v < V4; ++v) {
            const int slot = tid + 256 * v;
            const int r = slot / (NC / VE), c4 = (slot % (NC / VE)) * VE;
            *reinterpret_cast<vec_t*>(Bs + r * LDC + c4) = nx[v];
        }
        __syncthreads();
        if (r0 + CH < end) load(r0 + CH);
#pragma unroll 2
        for (int k = 0; k < CH; k += 4) {
            const TB* rp = Bs + (k + kr) * LDC + col;
            const double a = (double)rp[16 * GA], b2 = (double)rp[16 * GB];
            double v[NCT];
#pragma unroll
            for (int g = GB < GA ? GB : GA; g < NCT; ++g) v[g] = (double)rp[16 * g];
#pragma unroll
            for (int g = 0; g < NA; ++g) accA[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, v[GA + g], accA[g], 0, 0, 0);
#pragma unroll
            for (int g = 0; g < NBB; ++g)
                accB[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(b2, v[GB + g], accB[g], 0, 0, 0);
        }
    }
    // block index of (ga, gb) in the upper enumeration: ga NCT - ga (ga - 1) / 2 + (gb - ga)
#pragma unroll
    for (int g = 0; g < NA; ++g) {
        const int bi = GA * NCT - GA * (GA - 1) / 2 + g;
#pragma unroll
        for (int r = 0; r < 4; ++r) outp[(bi * 4 + r) * 64 + l] = accA[g][r];
    }
#pragma unroll
    for (int g = 0; g < NBB; ++g) {
        const int bi = GB * NCT - GB * (GB - 1) / 2 + g;
#pragma unroll
        for (int r = 0; r < 4; ++r) outp[(bi * 4 + r) * 64 + l] = accB[g][r];
    }
}

__global__ __launch_bounds__(256) void k_gram_f64_mfma_w8(const float* __restrict__ B, const DevState* __restrict__ st,
                                                           long long nrows, long long rows_per_block,
                                                           double* __restrict__ Gpart) {
    constexpr int NB = gram_blocks(8);
    __shared__ float Bs[64 * (128 + 4)];
    const int ldb = st->ldb;
    const long long begin = (long long)blockIdx.x * rows_per_block;
    long long end = begin + rows_per_block;
    if (end > nrows) end = nrows;
    double* outp = Gpart + (size_t)blockIdx.x * NB * 256;
    // the wave index is uniform over a wave; every branch meets the same barriers
    switch (threadIdx.x >> 6) {
        case 0: gram_w8_wave<0, float>(B, ldb, begin, end, Bs, outp); break;
        case 1: gram_w8_wave<1, float>(B, ldb, begin, end, Bs, outp); break;
        case 2: gram_w8_wave<2, float>(B, ldb, begin, end, Bs, outp); break;
        default: gram_w8_wave<3, float>(B, ldb, begin, end, Bs, outp); break;
    }
}

// The same for a stored FP64 first core (FP64 data on the Gram route).
__global__ __launch_bounds__(256) void k_gram_f64_mfma_w8d(const double* __restrict__ B,
                                                            const DevState* __restrict__ st, long long nrows,
                                                            long long rows_per_block, double* __restrict__ Gpart) {
    constexpr int NB = gram_blocks(8);
    __shared__ double Bs[32 * (128 + 4)];
    const int ldb = st->ldb;
    const long long begin = (long long)blockIdx.x * rows_per_block;
    long long end = begin + rows_per_block;
    if (end > nrows) end = nrows;
    double* outp = Gpart + (size_t)blockIdx.x * NB * 256;
    switch (threadIdx.x >> 6) {
        case 0: gram_w8_wave<0, double>(B, ldb, begin, end, Bs, outp); break;
        case 1: gram_w8_wave<1, double>(B, ldb, begin, end, Bs, outp); break;
        case 2: gram_w8_wave<2, double>(B, ldb, begin, end, Bs, outp); break;
        default: gram_w8_wave<3, double>(B, ldb, begin, end, Bs, outp); break;
    }
}

}  // namespace ttrt
