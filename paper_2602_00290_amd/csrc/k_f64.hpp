// FP64 contractions of the first core on gfx950 FP64 MFMA (v_mfma_f64_16x16x4f64).
//
//   MODE_PROJECT: B[k,:] = d_k ( sum_j Z[nbr_j(k),:] G_j + sum_q z_q(k) G_rank1[q] )
//                 (B = Z_new L_Theta of the pending TT sum, without Z_new)
//   MODE_OUTPUT:  Z_out = B V_r
//
// Each block runs 8 waves over row blocks of 16 RT rows per wave (RT = 2
// 16-row tiles; RT = 1 where two would spill registers: 128 columns, or 64
// with the fused Gram's 40 accumulator doubles) and loops over consecutive row
// blocks (a contiguous range per block, consecutive ranges on one XCD).  K runs in chunks of 32:
// each lane loads its A fragment straight into registers, four consecutive K
// values per row tile and 16-K group (a 4-aligned run of K never crosses a
// gather block: every leading dimension is a multiple of 8), and the operand
// chunk is staged in LDS, column-major, in two buffers (one barrier per
// chunk); the next chunk's loads are in flight while the current one
// computes.  The row data of a row block (d, neighbour rows, rank-1 values)
// is derived from the row indices and the problem arrays into LDS at its
// start, so no per-row tables are read.
//
// v_mfma_f64_16x16x4f64 lane layout (64 lanes, l = m + 16 q):
//   A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k,
//   D[i][j] in lane j + 16 (i % 4), register i / 4.
// In 16-K group t lane (m, q) supplies K = 16 t + 4 q + e to the e-th MFMA
// (A row m; B column 16 c + m), so one pair of 16-byte loads feeds four MFMAs.
// Consecutive MFMAs go to different accumulators (RT NCT independent chains).
// The accumulator of a row tile holds row 4 r + q, column 16 c + m in
// register r of lane (m, q): for a fixed r that is an A/B operand of a K = 4
// step over the rows 4 r .. 4 r + 3, which is how the fused FP64 Gram B^T B
// is accumulated from the accumulators (GRAM = true).  Each block writes the
// upper 16 x 16 blocks of its partial Gram matrix for k_sum_gram<NCT>.
#pragma once

#include "k_fused.hpp"

namespace ttrt {

constexpr int kF64Waves = 8;
constexpr int kF64Threads = 64 * kF64Waves;
constexpr int kF64Rows = 32 * kF64Waves;   // rows per row block (two row tiles per wave)
constexpr int kF64KC = 32;                 // K per staged chunk
constexpr int kF64LdK = kF64KC + 2;        // LDS column stride (doubles) of the staged operand
constexpr int kF64Z = kMaxBC + 4;          // rank-1 value rows (read four at a time)

typedef double f64x2 __attribute__((ext_vector_type(2)));

// Gather blocks whose rows the row data holds: the identity and the shifted
// copies (upwind, Rusanov), or up to kMaxBlocks with the HLL flux's
// per-(term, shift) blocks.
__host__ __device__ constexpr int f64_nbr_rows(bool hll) { return hll ? kMaxBlocks : kMaxTerms + 1; }

// Dynamic LDS bytes of k_mm_f64<.., NCT, GRAM, RT, HLL>: two operand buffers
// and the row data of 128 RT rows (the Gram reduction at the end reuses the
// space).
__host__ __device__ inline size_t f64_lds_bytes(int nct, bool gram, int rt, bool hll = false) {
    const size_t nrow = (size_t)16 * rt * kF64Waves;
    const size_t op = (size_t)2 * 16 * nct * kF64LdK * sizeof(double);
    const size_t rows = nrow * (sizeof(double) + f64_nbr_rows(hll) * sizeof(int)) +
                        (size_t)kF64Z * nrow * sizeof(double) + (hll ? (size_t)kMaxBlocks * nrow * sizeof(double) : 0);
    const size_t main = op + rows;
    const size_t red = gram ? (size_t)(kF64Waves / 2) * gram_blocks(nct) * 256 * sizeof(double) : 0;
    return main > red ? main : red;
}

// x / d and x % d for 0 <= x < 2^31 and 1 <= d: the FP64 product with the
// reciprocal is within one of the quotient, which the remainder corrects.
__device__ __forceinline__ int divmod_d(int x, int d, double rcp, int& rem) {
    int q = (int)((double)x * rcp);
    int r = x - q * d;
    if (r < 0) { --q; r += d; }
    if (r >= d) { ++q; r -= d; }
    rem = r;
    return q;
}

template <int MODE, int NCT, bool GRAM, int RT, bool HLL = false>
__global__ __launch_bounds__(kF64Threads) void k_mm_f64(Geom g, OpDesc op, const DevState* __restrict__ st,
                                                         const double* __restrict__ A,
                                                         const double* __restrict__ Gop, double* __restrict__ Out,
                                                         RowData rd, double* __restrict__ Gpart) {
    constexpr int NP = 16 * NCT;
    constexpr int NB = gram_blocks(NCT);
    constexpr int ROWS = 16 * RT * kF64Waves;   // rows per row block
    extern __shared__ __align__(16) unsigned char f64_lds[];
    // the operator's per-block tables (dynamically indexed: kept out of SGPRs)
    __shared__ int s_gax[kMaxBlocks], s_gdir[kMaxBlocks], s_r1kind[kMaxBlocks], s_r1face[kMaxBlocks];
    __shared__ int s_gwk[kMaxBlocks], s_r1hll[kMaxBlocks];
    __shared__ double s_r1coef[kMaxBlocks];
    double* Bs0 = reinterpret_cast<double*>(f64_lds);                         // 2 x [NP][kF64LdK]
    double* rowd = Bs0 + (size_t)2 * NP * kF64LdK;                             // [rows]
    double* rowz = rowd + ROWS;                                            // [kF64Z][rows]
    double* rowc = rowz + (size_t)kF64Z * ROWS;                            // HLL: [blocks][rows] weights
    int* nbr = reinterpret_cast<int*>(rowc + (HLL ? (size_t)kMaxBlocks * ROWS : 0));   // [blocks][rows]

    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int m = l & 15, q = l >> 4;
    if (tid < kMaxBlocks) {
        s_gax[tid] = op.gaxis[tid];
        s_gdir[tid] = op.gdir[tid];
        s_r1kind[tid] = op.r1kind[tid];
        s_r1face[tid] = op.r1face[tid];
        s_r1coef[tid] = op.r1coef[tid];
        s_gwk[tid] = op.gwk[tid];
        s_r1hll[tid] = op.r1hll[tid];
    }
    int lda, K, KG, ldo, nblk, kper, ldg;
    if (MODE == MODE_PROJECT) {
        lda = st->ldz; kper = st->ldz; nblk = op.n_gather; KG = nblk * kper; K = st->kall; ldo = st->ldb;
        ldg = st->ldb;
    } else {
        lda = st->ldb; kper = st->ldb; nblk = 1; KG = kper; K = kper; ldo = st->ldzn; ldg = st->ldzn;
    }
    const int n_kc = (K + kF64KC - 1) / kF64KC;
    const FastDiv dkp(kper);
    const double rG = 1.0 / g.G, rnx = 1.0 / g.nx, rny = 1.0 / g.ny;

    // contiguous row-block ranges per block; consecutive ranges on one XCD
    // (blocks are dealt to the 8 XCDs round robin)
    const long long nrb = (g.M + ROWS - 1) / ROWS;
    const int nbk = gridDim.x, b = blockIdx.x;
    const int lb = (nbk % 8 == 0) ? (b % 8) * (nbk / 8) + b / 8 : b;
    const long long rb_begin = (long long)lb * nrb / nbk, rb_end = (long long)(lb + 1) * nrb / nbk;

    f64x4 gacc[GRAM ? NB : 1];
#pragma unroll
    for (int i = 0; i < (GRAM ? NB : 1); ++i) gacc[i] = (f64x4){0.0, 0.0, 0.0, 0.0};

    // operand chunk kc (K rows k0 .. k0 + 31, NP columns, zero beyond K and
    // ldg) into registers: slot s holds column n = s % NP of the K rows
    // 2 (s / NP) and 2 (s / NP) + 1, so that consecutive lanes read
    // consecutive columns (coalesced) and write 16 bytes along K into the
    // [n][k] layout, lanes n .. n + 15 starting 4 banks apart
    constexpr int OPP = kF64KC * NP / 2;                 // slots per chunk
    constexpr int OPN = (OPP + kF64Threads - 1) / kF64Threads;
    f64x2 opr[OPN];
    auto fetch_op = [&](int kc) __attribute__((always_inline)) {
        const double* gk = Gop + (size_t)kc * kF64KC * ldg;   // uniform chunk base, 32-bit offsets
        const int kr = K - kc * kF64KC;                       // K rows left from the chunk start
#pragma unroll
        for (int v = 0; v < OPN; ++v) {
            const int idx = tid + kF64Threads * v;
            const int n = idx % NP, kk = 2 * (idx / NP);
            f64x2 x = (f64x2){0.0, 0.0};
            if (idx < OPP && n < ldg) {
                const int o = kk * ldg + n;
                if (kk < kr) x[0] = gk[o];
                if (kk + 1 < kr) x[1] = gk[o + ldg];
            }
            opr[v] = x;
        }
    };
    auto store_op = [&](double* Bs) __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < OPN; ++v) {
            const int idx = tid + kF64Threads * v;
            if (idx < OPP)
                *reinterpret_cast<f64x2*>(Bs + (size_t)(idx % NP) * kF64LdK + 2 * (idx / NP)) = opr[v];
        }
    };
    // this lane's A fragments of one 16-K group (flat index t = 2 kc + gi):
    // RT row tiles, four consecutive K values each; loaded one group ahead
    f64x2 ra[RT][2];
    double rw[RT];   // HLL: the per-row weight of the fragment's gather block
    auto fetch_a = [&](int t) __attribute__((always_inline)) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int r = 16 * RT * w + 16 * rt + m;
            const int k = 16 * t + 4 * q;
            f64x2 v0 = (f64x2){0.0, 0.0}, v1 = v0;
            if constexpr (HLL) rw[rt] = 1.0;
            if (k < KG) {
                const int j = dkp.q(k), cc = k - j * kper;
                const int src = nbr[j * ROWS + r];
                if constexpr (HLL) rw[rt] = rowc[j * ROWS + r];
                if (src >= 0) {
                    const double* ap = A + (long long)src * lda + cc;
                    v0 = *reinterpret_cast<const f64x2*>(ap);
                    v1 = *reinterpret_cast<const f64x2*>(ap + 2);
                }
            } else if (MODE == MODE_PROJECT && k < K) {
                const int qq = k - KG;
                v0 = (f64x2){rowz[qq * ROWS + r], rowz[(qq + 1) * ROWS + r]};
                v1 = (f64x2){rowz[(qq + 2) * ROWS + r], rowz[(qq + 3) * ROWS + r]};
            }
            ra[rt][0] = v0;
            ra[rt][1] = v1;
        }
    };
    const int n_grp = (K + 15) >> 4;   // 16-K groups with data (the last chunk may hold one)

    for (long long rb = rb_begin; rb < rb_end; ++rb) {
        const long long row0 = rb * ROWS;
        __syncthreads();   // the previous row block's readers of the row data are done
        if (tid < ROWS) {
            // one row per thread: cell, group and cell coordinates once, then the
            // neighbour rows of the gather blocks, d and the rank-1 values
            const long long k = row0 + tid;
            const bool ok = k < g.M;
            int grp = 0, ix = 0, iy = 0, iz = 0;
            const int cell = ok ? divmod_d((int)k, g.G, rG, grp) : 0;
            iy = divmod_d(cell, g.nx, rnx, ix);
            iz = divmod_d(iy, g.ny, rny, iy);
            const int idx3[3] = {ix, iy, iz}, n3[3] = {g.nx, g.ny, g.nz};
            const int st3[3] = {g.G, g.G * g.nx, g.G * g.nx * g.ny};
            // HLL: the row's face factors along each axis (towards cell -/+ e_d)
            double eL[3] = {1.0, 1.0, 1.0}, eR[3] = {1.0, 1.0, 1.0};
            if constexpr (HLL) {
                if (ok)
                    for (int ax = 0; ax < g.dim; ++ax) {
                        eL[ax] = hll_face_eps(g, rd, k, ax, -1);
                        eR[ax] = hll_face_eps(g, rd, k, ax, 1);
                    }
            }
            for (int j = 0; j < nblk; ++j) {
                int src = ok ? (int)k : -1;
                if (MODE == MODE_PROJECT && j > 0 && ok) {
                    const int ax = s_gax[j], dir = s_gdir[j];
                    int jj = idx3[ax] + dir;
                    const bool out = jj < 0 || jj >= n3[ax];
                    if (out && !g.periodic[ax]) src = -1;
                    else {
                        jj = out ? (jj + n3[ax]) % n3[ax] : jj;
                        src = (int)k + (jj - idx3[ax]) * st3[ax];
                    }
                }
                nbr[j * ROWS + tid] = src;
                if constexpr (HLL) {
                    const int ax = s_gax[j];
                    rowc[j * ROWS + tid] = s_gwk[j] == 0 ? 1.0 : hll_weight(s_gwk[j], eL[ax], eR[ax], g.lam[ax]);
                }
            }
            if (MODE == MODE_PROJECT) {
                double kap = 0.0;
                if (ok) kap = rd.kfull ? rd.kfull[k] : rd.kappa0[cell] * rd.kscale[grp];
                const double ktot = (ok && rd.kscat) ? kap + rd.kscat[k] : kap;
                rowd[tid] = (ok && op.scale_d) ? 1.0 / (1.0 + g.cdt * ktot) : 1.0;
                for (int qq = 0; qq < kF64Z; ++qq) {
                    double v = 0.0;
                    if (ok && qq < op.n_r1) {
                        if (s_r1kind[qq] == 0) {
                            v = g.cdt * kap * rd.eps[k];
                            if (rd.kscat) v += g.cdt * rd.kscat[k] * rd.jn[k];
                        } else {
                            const int face = s_r1face[qq], ax = face >> 1;
                            const int edge = (face & 1) ? n3[ax] - 1 : 0;
                            double coef = s_r1coef[qq];
                            if (s_r1kind[qq] == 2) {   // HLL inflow column: the face's factor
                                const double e = (face & 1) ? eR[ax] : eL[ax];
                                coef *= s_r1hll[qq] == 1 ? 0.5 * (1.0 + e) : 0.5 * (1.0 - e);
                            }
                            if (idx3[ax] == edge) v = coef * rd.ghost[face * g.G + grp];
                        }
                    }
                    rowz[qq * ROWS + tid] = v;
                }
            }
        }
        f64x4 acc[RT][NCT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int c = 0; c < NCT; ++c) acc[rt][c] = (f64x4){0.0, 0.0, 0.0, 0.0};
        __syncthreads();
        if (n_kc > 0) {
            fetch_op(0);
            fetch_a(0);
            store_op(Bs0);
        }
        for (int kc = 0; kc < n_kc; ++kc) {
            __syncthreads();   // chunk kc is in buffer kc & 1; the other buffer's readers are done
            const double* Bs = Bs0 + (size_t)(kc & 1) * NP * kF64LdK;
            const bool more = kc + 1 < n_kc;
            if (more) fetch_op(kc + 1);   // in flight while this chunk computes
#pragma unroll
            for (int gi = 0; gi < 2; ++gi) {
                const int t = 2 * kc + gi;
                if (t >= n_grp) break;    // an all-zero padding group (uniform)
                f64x2 a[RT][2];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if constexpr (HLL) {
                        a[rt][0] = ra[rt][0] * rw[rt];
                        a[rt][1] = ra[rt][1] * rw[rt];
                    } else {
                        a[rt][0] = ra[rt][0];
                        a[rt][1] = ra[rt][1];
                    }
                }
                if (t + 1 < n_grp) fetch_a(t + 1);   // the next group, across the chunk boundary
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    double bv[NCT];
#pragma unroll
                    for (int c = 0; c < NCT; ++c) bv[c] = Bs[(size_t)(16 * c + m) * kF64LdK + 16 * gi + 4 * q + e];
#pragma unroll
                    for (int c = 0; c < NCT; ++c)
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
                            acc[rt][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][e >> 1][e & 1], bv[c],
                                                                              acc[rt][c], 0, 0, 0);
                }
            }
            if (more) store_op(Bs0 + (size_t)((kc + 1) & 1) * NP * kF64LdK);
        }
        // row factor d on the rows (row 4 r + q of the tile in register r) and store
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * RT * w + 16 * rt + 4 * r + q;
                const long long row = row0 + i;
                const double d = MODE == MODE_PROJECT ? rowd[i] : 1.0;
#pragma unroll
                for (int c = 0; c < NCT; ++c) {
                    acc[rt][c][r] *= d;
                    const int col = 16 * c + m;
                    if (row < g.M && col < ldo) Out[row * ldo + col] = acc[rt][c][r];
                }
            }
        if constexpr (GRAM) {
            // B^T B over this wave's rows (rows past M are zero)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int bi = 0;
#pragma unroll
                    for (int ga = 0; ga < NCT; ++ga)
#pragma unroll
                        for (int gb = ga; gb < NCT; ++gb) {
                            gacc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[rt][ga][r], acc[rt][gb][r], gacc[bi],
                                                                            0, 0, 0);
                            ++bi;
                        }
                }
        }
    }

    if constexpr (GRAM) {
        // fixed-order reduction of the 8 waves' partial Gram blocks through LDS
        double* red = reinterpret_cast<double*>(f64_lds);
        constexpr int PER = NB * 256;   // doubles per wave
        __syncthreads();
        for (int half = kF64Waves / 2; half >= 1; half >>= 1) {
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

}  // namespace ttrt
