// Fused gather contraction over the first core on gfx950 MFMA (FP32 state).
//
// One persistent kernel walks 32-row tiles of the merged (cell, group) rows:
//
//   B[k,:] = d_k ( sum_j Z[nbr_j(k),:] G_j + sum_q z_q(k) g_q )       (projection)
//
// with the K dimension laid out as [gather block 0 | block 1 | ... | rank-1
// columns] (n_gather * ldz + n_r1 rows of the operand).  The d_k row factor
// and the rank-1 column values are applied to the A operand as it is loaded,
// so the MFMA result is B itself.
//
//   GRAM = true:  B stays in registers and its FP64 Gram matrix B^T B is
//                 accumulated on FP64 MFMA (products of FP32 values are exact
//                 in FP64); B is never written.  Each block writes the upper
//                 16 x 16 blocks of its partial Gram matrix.
//   GRAM = false: the operand is G' = G V_r and the tile is stored: this is
//                 Z_out = B V_r evaluated from Z without B in memory.
//
// Lane layouts (v_mfma_f32_16x16x4f32 and v_mfma_f64_16x16x4f64, 64 lanes):
//   A[i][k] from lane i + 16 k,  B[k][j] from lane j + 16 k,
//   D[i][j] in lane j + 16 (i / 4), register i % 4.
// The K index of a lane's slot is permuted: in group t (16 K values) lane l
// supplies K = 16 t + 4 (l / 16) + e to the e-th MFMA of the group, so that
// one 16-byte load per lane feeds four MFMAs.  The f32 output tile then sits
// in exactly the FP64 A/B operand layout the Gram MFMA needs (rows of B are
// summed over, so any row-to-slot assignment that both operands share works).
#pragma once

#include "k_mfma.hpp"

namespace ttrt {

typedef float f32x4v __attribute__((ext_vector_type(4)));

constexpr int kFusedWaves = 8;
constexpr int kFusedThreads = 64 * kFusedWaves;

__host__ __device__ constexpr int gram_blocks(int nct) { return nct * (nct + 1) / 2; }

// Gather structure of one operator for the fused kernels.  Gather block
// j >= 1 of row k reads the row nbr[k * ns + j - 1] of the per-problem
// neighbour table (-1: none), built once at create (every operator with
// streaming terms has the same gather order).  The rank-1 columns of the
// operator are a dense block of rw columns per row, stored roff elements
// after the start of the current Z.  Every load of the fused kernels is
// unconditional: a slot with nothing to read points at a zero region (zoff),
// which keeps the loads branch-free so that they stay in flight across the
// pipeline.
struct FusedNbr {
    int n_gather;
    int ns;           // entries per row of the neighbour table (2 d_X)
    int rw;
    long long roff;
    long long zoff;   // offset of a zero region of at least 64 elements (loads with nothing to read go there)
    int scale_d;
};

constexpr int kOffSlots = 9;   // gather blocks 0..6, 7: rank-1 block, 8: always empty
constexpr int kFusedStages = 2;
constexpr int kTbStride = 36;   // row stride (floats) of the output kernel's per-wave transpose buffer   // A-operand groups in flight per wave (4 measured no faster)

// K groups the fused kernels run for T groups of data: a multiple of the
// stage count and at least two rounds of stages (padding groups have a zero
// operand).
__host__ __device__ inline int fused_groups(int T, int ns) {
    const int g = (T + ns - 1) / ns * ns;
    return g < 2 * ns ? 2 * ns : g;
}

// Bytes of dynamic LDS for k_fused_f32<NCT, GRAM> with `ngroups` K groups:
// operand and per-wave row-offset tables (the Gram reduction reuses the
// space).
__host__ __device__ inline size_t fused_lds_bytes(int nct, bool gram, int ngroups) {
    const size_t op = (size_t)fused_groups(ngroups, kFusedStages) * nct * 64 * 16;
    const size_t offs = (size_t)kFusedWaves * 2 * kOffSlots * 16 * sizeof(int);
    const size_t tb = gram ? 0 : (size_t)kFusedWaves * 32 * kTbStride * sizeof(float);
    const size_t main = op + offs + tb;
    const size_t red = gram ? (size_t)(kFusedWaves / 2) * gram_blocks(nct) * 256 * sizeof(double) : 0;
    return main > red ? main : red;
}

// Per-row constants of the fused kernels, computed once per problem (T is
// fixed): d_k = 1 / (1 + c dt (kappa_k + kappa_s,k)) in FP32 and the boundary mask of the
// row's cell (bit 2a: first cell along axis a, bit 2a + 1: last cell).
__global__ __launch_bounds__(256) void k_row_aux(Geom g, RowData rd, float2* __restrict__ aux) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= g.M) return;
    int mask = 0;
    for (int a = 0; a < g.dim; ++a) {
        const int idx = axis_index(g, k, a);
        const int n = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
        if (idx == 0) mask |= 1 << (2 * a);
        if (idx == n - 1) mask |= 1 << (2 * a + 1);
    }
    float2 v;
    v.x = (float)(1.0 / (1.0 + g.cdt * row_kappa_tot(g, rd, k)));
    v.y = __int_as_float(mask);
    aux[k] = v;
}

// Neighbour rows of the gather blocks j = 1 .. ns of operator `op` (shifted
// copies of Z: the upwind neighbour of each streaming term, wrapped on
// periodic axes, -1 outside the domain), ns per row.
__global__ __launch_bounds__(256) void k_nbr_table(Geom g, OpDesc op, int ns, int* __restrict__ tab) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= g.M) return;
    for (int j = 1; j <= ns; ++j) {
        long long r = -1;
        if (j < op.n_gather) r = neighbour_row(g, k, op.gaxis[j], op.gdir[j]);
        tab[k * ns + j - 1] = (int)r;
    }
}

// Rank-1 columns of operator `op` as a dense M x rw block (zero beyond
// n_r1); the fused kernels scale them by d_k with the rest of the row.
__global__ __launch_bounds__(256) void k_rank1_rows(Geom g, OpDesc op, RowData rd, int rw, float* __restrict__ R) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= g.M) return;
    for (int q = 0; q < rw; ++q) R[k * rw + q] = q < op.n_r1 ? (float)rank1_value(g, op, rd, k, q) : 0.0f;
}

template <int NCT, bool GRAM>
__global__ __launch_bounds__(kFusedThreads) void k_fused_f32(Geom g, FusedNbr fn, const DevState* __restrict__ st,
                                                              const float* __restrict__ Z,
                                                              const float* __restrict__ Gsw,
                                                              float* __restrict__ Out, const float2* __restrict__ aux,
                                                              const int* __restrict__ nbr, double* __restrict__ Gpart,
                                                              long long ntiles) {
    constexpr int NB = gram_blocks(NCT);
    extern __shared__ __align__(16) unsigned char fused_lds[];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int m = l & 15, q = l >> 4;
    const int ldz = st->ldz;
    const int KG = fn.n_gather * ldz;
    const int K = KG + fn.rw;
    const int T = (K + 15) >> 4;
    constexpr int NS = kFusedStages;
    const int T2 = fused_groups(T, NS);
    const int ldo = GRAM ? 0 : st->ldzn;
    const FastDiv dldo(GRAM ? 1 : ldo);
    const unsigned magic = ((1u << 20) + (unsigned)ldz - 1u) / (unsigned)ldz;   // k0 / ldz = (k0 magic) >> 20 for k0 < 2^14

    f32x4v* Gs = reinterpret_cast<f32x4v*>(fused_lds);
    int* offs_all = reinterpret_cast<int*>(fused_lds + (size_t)T2 * NCT * 64 * 16);
    int* offs = offs_all + w * (2 * kOffSlots * 16);                 // [rt][slot][m] of this wave
    float* tb = reinterpret_cast<float*>(offs_all + kFusedWaves * 2 * kOffSlots * 16) + w * 32 * kTbStride;

    {   // operand, already in lane order
        const f32x4v* src = reinterpret_cast<const f32x4v*>(Gsw);
        const int nvec = T * NCT * 64;
        for (int idx = tid; idx < T2 * NCT * 64; idx += kFusedThreads)
            Gs[idx] = idx < nvec ? src[idx] : (f32x4v){0.f, 0.f, 0.f, 0.f};
    }
    const int zoff = (int)fn.zoff;
    if (l < 32) offs[(l >> 4) * kOffSlots * 16 + 8 * 16 + (l & 15)] = zoff;   // slot 8 of both row tiles
    __syncthreads();

    // contiguous tile ranges per wave; consecutive ranges on one XCD (blocks
    // are dealt to the 8 XCDs round robin)
    const int nb = gridDim.x, b = blockIdx.x;
    const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const long long gw = (long long)lb * kFusedWaves + w;
    const long long nw = (long long)nb * kFusedWaves;
    const int t_begin = (int)(gw * ntiles / nw), t_end = (int)((gw + 1) * ntiles / nw);

    // Row data of a tile into this wave's offset table (slots 0..8 of both row
    // tiles), from the row's table entries loaded a tile ahead (RowPre).  Lane
    // (m, q) writes slots q and q + 4 of row m: slot 0 is the row itself,
    // slots 1..6 gather blocks, slot 7 the rank-1 block.  Returns d of the
    // lane's two A rows.  Branch-free: a slot with nothing to read points at
    // the zero region.
    struct RowPre {
        float2 a;
        int n1, n2;   // neighbour rows of slots q and q + 4 (when they are gather blocks)
    };
    const int last = (int)g.M - 1;
    const int ns = fn.ns;
    const int i1 = min(max(q - 1, 0), ns - 1), i2 = min(q + 3, ns - 1);
    auto pre_of = [&](int tile, int rt) -> RowPre {
        int row = 32 * tile + 16 * rt + m;
        row = row < last ? row : last;   // rows past the end are never used
        RowPre r;
        r.a = aux[row];
        r.n1 = nbr[(size_t)row * ns + i1];
        r.n2 = nbr[(size_t)row * ns + i2];
        return r;
    };
    auto tile_rows = [&](int tile, const RowPre& p0, const RowPre& p1, float& d0, float& d1) {
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int row = 32 * tile + 16 * rt + m;
            const bool valid = row < g.M;
            const RowPre& pr = rt == 0 ? p0 : p1;
            const float d = fn.scale_d ? pr.a.x : 1.0f;
            if (rt == 0) d0 = d; else d1 = d;
            int lo = (q < fn.n_gather && pr.n1 >= 0) ? pr.n1 * ldz : zoff;
            lo = q == 0 ? row * ldz : lo;
            int hi = (q + 4 < fn.n_gather && pr.n2 >= 0) ? pr.n2 * ldz : zoff;
            hi = q == 3 ? (fn.rw > 0 ? (int)(fn.roff + (long long)row * fn.rw) : zoff) : hi;
            offs[(rt * kOffSlots + q) * 16 + m] = valid ? lo : zoff;
            offs[(rt * kOffSlots + q + 4) * 16 + m] = valid ? hi : zoff;
        }
    };
    // Element offsets of the A operand of K group t (both row tiles) from the
    // offset table: gather block k0 / ldz, the rank-1 block (7) or nothing
    // (8), plus the column within the block.  Branch-free; the table entries
    // are LDS reads whose results are used one pipeline stage later.
    const char* zb = reinterpret_cast<const char*>(Z);
    auto addr_a = [&](int t, int& o0, int& o1, int& cc) {
        const int k0 = 16 * t + 4 * q;
        const int jj = (int)(__umul24((unsigned)k0, magic) >> 20);
        // selects written as masks (all ones / zero)
        const int gm = -(int)(k0 < KG), rm = -(int)(k0 < K);
        const int slot = (jj & gm) | ((8 + rm) & ~gm);
        cc = ((k0 - (int)__umul24((unsigned)jj, (unsigned)ldz)) & gm) | ((k0 - KG) & rm & ~gm);
        o0 = offs[slot * 16 + m];
        o1 = offs[(kOffSlots + slot) * 16 + m];
    };
    // one 16-byte load per row tile, not yet scaled by d (the scale is applied
    // when the group is consumed, so the load stays in flight); 32-bit byte
    // offsets from the uniform base (the workspace spans < 4 GiB)
    auto load_a = [&](int o0, int o1, int cc, f32x4v& a0, f32x4v& a1) {
        a0 = *reinterpret_cast<const f32x4v*>(zb + (unsigned)(o0 + cc) * 4u);
        a1 = *reinterpret_cast<const f32x4v*>(zb + (unsigned)(o1 + cc) * 4u);
    };

    f64x4 gacc[GRAM ? NB : 1];
#pragma unroll
    for (int i = 0; i < (GRAM ? NB : 1); ++i) gacc[i] = (f64x4){0.0, 0.0, 0.0, 0.0};

    // Software pipeline over the flat sequence of (tile, group) with NS
    // register stages in rotation (the K loop is unrolled by NS, so no stage
    // is ever copied: a copy would wait for its load).  Group t is scaled out
    // of its stage, the stage is refilled with group t + NS at once (address
    // from the previous step), the offsets of group t + NS + 1 are read, and
    // only then are group t's MFMAs issued; the B operand of group t + 1 is
    // read from LDS meanwhile.  Groups past T2 are the next tile's first
    // groups: its offset table is written once this tile's last offsets have
    // been read (after step T2 - NS - 2), so the pipeline runs across tile
    // boundaries.  Row-table entries are loaded a tile ahead.
    const f32x4v zero4 = (f32x4v){0.f, 0.f, 0.f, 0.f};
    float d0 = 0.f, d1 = 0.f, nd0 = 0.f, nd1 = 0.f;
    f32x4v sa[NS], sb[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) sa[u] = sb[u] = zero4;
    int po0 = zoff, po1 = zoff, pcc = 0;
    if (t_begin < t_end) {
        tile_rows(t_begin, pre_of(t_begin, 0), pre_of(t_begin, 1), d0, d1);
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            int o0, o1, cc;
            addr_a(u, o0, o1, cc);
            load_a(o0, o1, cc, sa[u], sb[u]);
        }
        addr_a(NS, po0, po1, pcc);
    }
    f32x4v acc[2][NCT];
    // (group t + 1 = T2 reads past the operand into the offset tables: unused
    // and in bounds)
    auto stage = [&](int t, f32x4v& s0, f32x4v& s1, f32x4v (&bc)[NCT], f32x4v (&bn)[NCT]) {
#pragma unroll
        for (int c = 0; c < NCT; ++c) bn[c] = Gs[((t + 1) * NCT + c) * 64 + l];
        const f32x4v a0 = s0 * d0, a1 = s1 * d1;
        // the stage registers are free once scaled: refill them before the
        // MFMAs (the empty asm keeps the scaling ahead of the refill, so the
        // refill can reuse the stage registers)
        asm volatile("" ::"v"(a0), "v"(a1));
        __builtin_amdgcn_sched_barrier(0);
        load_a(po0, po1, pcc, s0, s1);
        __builtin_amdgcn_sched_barrier(0);
        addr_a(t + NS + 1 < T2 ? t + NS + 1 : t + NS + 1 - T2, po0, po1, pcc);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[e], bc[c][e], acc[0][c], 0, 0, 0);
                acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[e], bc[c][e], acc[1][c], 0, 0, 0);
            }
    };
    for (int tile = t_begin; tile < t_end; ++tile) {
        const bool more = tile + 1 < t_end;
        const RowPre na0 = pre_of(tile + 1, 0), na1 = pre_of(tile + 1, 1);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int c = 0; c < NCT; ++c) acc[rt][c] = zero4;

        f32x4v bA[NCT], bB[NCT];
#pragma unroll
        for (int c = 0; c < NCT; ++c) bA[c] = Gs[c * 64 + l];
        for (int t = 0; t < T2; t += NS) {
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                if (u & 1)
                    stage(t + u, sa[u], sb[u], bB, bA);
                else
                    stage(t + u, sa[u], sb[u], bA, bB);
                // the offsets of group T2 - 1 were read in step T2 - NS - 2:
                // the table now takes the next tile's rows (past the last
                // tile the old rows stay; their loads are in bounds and unused)
                if (t + u == T2 - NS - 2 && more) tile_rows(tile + 1, na0, na1, nd0, nd1);
            }
        }
        const int R0 = 32 * tile;

        if constexpr (GRAM) {
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double v[NCT];
#pragma unroll
                    for (int c = 0; c < NCT; ++c) v[c] = (double)acc[rt][c][r];
                    int bi = 0;
#pragma unroll
                    for (int ga = 0; ga < NCT; ++ga)
#pragma unroll
                        for (int gb = ga; gb < NCT; ++gb) {
                            gacc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[ga], v[gb], gacc[bi], 0, 0, 0);
                            ++bi;
                        }
                }
        } else {
            // the tile's 32 rows x ldo columns are contiguous in Out: transpose
            // the accumulators (D[i][j] of row tile rt: row 16 rt + 4 q + r,
            // column 16 c + m) through this wave's LDS buffer, then 16-byte stores
#pragma unroll
            for (int c = 0; c < NCT; ++c)
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) tb[(16 * rt + 4 * q + r) * kTbStride + 16 * c + m] = acc[rt][c][r];
            asm volatile("" ::: "memory");
            const int nrow = (int)min((long long)32, g.M - (long long)R0);
            const int nvec = (nrow * ldo) >> 2;
            char* ob = reinterpret_cast<char*>(Out) + (size_t)R0 * ldo * 4;
            for (int e = l; e < nvec; e += 64) {
                const int f = 4 * e, row = dldo.q(f), col = f - row * ldo;
                const f32x4v v = *reinterpret_cast<const f32x4v*>(tb + row * kTbStride + col);
                *reinterpret_cast<f32x4v*>(ob + (unsigned)f * 4u) = v;
            }
            asm volatile("" ::: "memory");
        }
        d0 = nd0;
        d1 = nd1;
    }

    if constexpr (GRAM) {
        // fixed-order reduction of the 8 waves' partial Gram blocks through LDS
        double* red = reinterpret_cast<double*>(fused_lds);
        constexpr int PER = NB * 256;   // doubles per wave
        __syncthreads();
        for (int half = kFusedWaves / 2; half >= 1; half >>= 1) {
            if (w >= half && w < 2 * half) {
#pragma unroll
                for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                    for (int r = 0; r < 4; ++r) red[(size_t)(w - half) * PER + (bi * 4 + r) * 64 + l] = gacc[bi][r];
            }
            __syncthreads();
            if (w < half) {
#pragma unroll
                for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                    for (int r = 0; r < 4; ++r) gacc[bi][r] += red[(size_t)w * PER + (bi * 4 + r) * 64 + l];
            }
            __syncthreads();
        }
        if (w == 0) {
            double* outp = Gpart + (size_t)b * PER;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int r = 0; r < 4; ++r) outp[(bi * 4 + r) * 64 + l] = gacc[bi][r];
        }
    }
}

// Sum the per-block partial Gram blocks of k_fused_f32<NCT, true> in a fixed
// order and expand them into the full symmetric (16 NCT) x (16 NCT) matrix
// (row-major, leading dimension ldg).  Partial entry (bi, r, lane) is element
// (16 ga + 4 r + lane / 16, 16 gb + lane % 16) of upper block bi = (ga, gb).
template <int NCT>
__global__ __launch_bounds__(256) void k_sum_gram(const double* __restrict__ parts, int nparts,
                                                  double* __restrict__ out, int ldg) {
    constexpr int NB = gram_blocks(NCT);
    constexpr int n = NB * 256;
    __shared__ double sh[8][32];
    const int e = blockIdx.x * 32 + (threadIdx.x & 31);
    const int qg = threadIdx.x >> 5;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (e < n) {
        int p = qg;
        for (; p + 24 < nparts; p += 32) {
            s0 += parts[(size_t)p * n + e];
            s1 += parts[(size_t)(p + 8) * n + e];
            s2 += parts[(size_t)(p + 16) * n + e];
            s3 += parts[(size_t)(p + 24) * n + e];
        }
        for (; p < nparts; p += 8) s0 += parts[(size_t)p * n + e];
    }
    sh[qg][threadIdx.x & 31] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (qg == 0 && e < n) {
        double t = 0.0;
        for (int k = 0; k < 8; ++k) t += sh[k][threadIdx.x];
        const int bi = e >> 8, r = (e >> 6) & 3, ln = e & 63;
        int ga = 0, rem = bi;
        while (rem >= NCT - ga) { rem -= NCT - ga; ++ga; }
        const int gb = ga + rem;
        const int i = 16 * ga + 4 * r + (ln >> 4), j = 16 * gb + (ln & 15);
        out[(size_t)i * ldg + j] = t;
        if (ga != gb) out[(size_t)j * ldg + i] = t;
    }
}

}  // namespace ttrt
