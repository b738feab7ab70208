// Kernels over the large first core (M = N_X * N_nu rows).
#pragma once

#include "k_small.hpp"
#include "tt_common.hpp"

namespace ttrt {

// Problem arrays used to evaluate the rank-1 columns and the absorption factor
// of a merged row on the fly.
struct RowData {
    const double* kappa0;   // N_X
    const double* kscale;   // N_nu
    const double* eps;      // M  (eps_g(T_cell))
    const double* ghost;    // 6 x N_nu isotropic ghost intensities
    const double* kfull;    // M opacities per (cell, group) row, or null for kappa0 x kscale
    const double* kscat;    // M scattering opacities, or null (no scattering)
    const double* jn;       // M angle means J^{m+1} of the source update (with scattering)
};

__device__ inline double row_kappa(const Geom& g, const RowData& rd, long long k) {
    if (rd.kfull) return rd.kfull[k];
    const long long cell = k / g.G;
    const int grp = (int)(k - cell * g.G);
    return rd.kappa0[cell] * rd.kscale[grp];
}

// absorption plus scattering opacity of row k (the implicit source's denominator)
__device__ inline double row_kappa_tot(const Geom& g, const RowData& rd, long long k) {
    const double ka = row_kappa(g, rd, k);
    return rd.kscat ? ka + rd.kscat[k] : ka;
}

// HLL flux: interface factor eps = (1 - exp(-tau)) / tau (1 at tau = 0) of
// the face of row k towards its neighbour along axis d in direction s, with
// tau = beta dx_d (kappa_k + kappa_neighbour) / 2 (total opacities of the
// row's group; the row's own on a non-periodic boundary face).
__device__ inline double hll_eps_of(double tau) { return tau > 0.0 ? -expm1(-tau) / tau : 1.0; }

__device__ inline double hll_face_eps(const Geom& g, const RowData& rd, long long k, int d, int s) {
    const double k0 = row_kappa_tot(g, rd, k);
    const long long nb = neighbour_row(g, k, d, s);
    const double kn = nb >= 0 ? row_kappa_tot(g, rd, nb) : k0;
    return hll_eps_of(g.hbeta * g.dx[d] * 0.5 * (k0 + kn));
}

// Per-row weight of HLL weight kind w (1..6: centre, minus and plus
// coefficients of the n^+ term, then of the n^- term) from the row's face
// factors eL (towards cell - e_d) and eR along the block's axis with lam_d.
__device__ inline double hll_weight(int w, double eL, double eR, double lam) {
    switch (w) {
        case 1: return -0.5 * lam * (eL + eR);
        case 2: return 0.5 * lam * (1.0 + eL);
        case 3: return -0.5 * lam * (1.0 - eR);
        case 4: return 0.5 * lam * (eL + eR);
        case 5: return 0.5 * lam * (1.0 - eL);
        case 6: return -0.5 * lam * (1.0 + eR);
        default: return 1.0;
    }
}

// Value in row k of rank-1 column q of the operator (before the d scaling):
// the isotropic source c dt (kappa eps + kappa_s J^{m+1}), or an inflow column.
__device__ inline double rank1_value(const Geom& g, const OpDesc& op, const RowData& rd, long long k, int q) {
    if (op.r1kind[q] == 0) {
        const double v = g.cdt * row_kappa(g, rd, k) * rd.eps[k];
        return rd.kscat ? v + g.cdt * rd.kscat[k] * rd.jn[k] : v;
    }
    const int face = op.r1face[q];
    const int axis = face >> 1, high = face & 1;
    const int n = axis == 0 ? g.nx : (axis == 1 ? g.ny : g.nz);
    const int idx = axis_index(g, k, axis);
    if (idx != (high ? n - 1 : 0)) return 0.0;
    const long long cell = k / g.G;
    const int grp = (int)(k - cell * g.G);
    double coef = op.r1coef[q];
    if (op.r1kind[q] == 2) {   // HLL inflow: the face's factor, the inside cell's opacity
        const double e = hll_face_eps(g, rd, k, axis, high ? 1 : -1);
        coef *= op.r1hll[q] == 1 ? 0.5 * (1.0 + e) : 0.5 * (1.0 - e);
    }
    return coef * rd.ghost[face * g.G + grp];
}

__device__ inline double row_scale(const Geom& g, const OpDesc& op, const RowData& rd, long long k) {
    return op.scale_d ? 1.0 / (1.0 + g.cdt * row_kappa_tot(g, rd, k)) : 1.0;
}

// ---------------------------------------------------------------------------
// Gather contraction
// ---------------------------------------------------------------------------
//
// MODE_PROJECT:  B[k,:] = d_k * ( sum_j Z[nbr_j(k),:] G_j + sum_q z_q(k) G_rank1[q] )
//                with j over the gather blocks (Z itself and its shifted copies
//                O_{d-} Z, O_{d+} Z), i.e. B = Z_new L_Theta for the pending TT
//                sum without forming Z_new (Appendix A operator terms).
// MODE_OUTPUT:   Z_out = B V_r (plain contraction, K = ldb).
// 64 x 64 output tile per 256-thread block, K staged through LDS in chunks of 8.
// MODE_ANGLE: Y = Z W of the direction-space projection (k_mm_f64 only)
enum { MODE_PROJECT = 0, MODE_OUTPUT = 1, MODE_ANGLE = 2 };

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_gather_gemm(Geom g, OpDesc op, const DevState* __restrict__ st,
                                                      const T* __restrict__ A, const T* __restrict__ Gop,
                                                      T* __restrict__ Out, RowData rd) {
    constexpr int BM = 64, BN = 64, KC = 8;
    __shared__ T As[KC][BM + 4];
    __shared__ T Gs[KC][BN + 4];
    __shared__ long long nbr[kMaxBlocks][BM];
    const int tid = threadIdx.x;
    const long long row0 = (long long)blockIdx.x * BM;
    const int col0 = blockIdx.y * BN;
    int lda, ldg, ldo, nblk, kper;
    if (MODE == MODE_PROJECT) {
        lda = st->ldz; kper = st->ldz; ldg = st->ldb; ldo = st->ldb; nblk = op.n_gather;
    } else {
        lda = st->ldb; kper = st->ldb; ldg = st->ldzn; ldo = st->ldzn; nblk = 1;
    }
    if (col0 >= ldo) return;
    for (int idx = tid; idx < nblk * BM; idx += 256) {
        const int j = idx / BM, i = idx % BM;
        const long long k = row0 + i;
        long long src = -1;
        if (k < g.M) src = (MODE == MODE_OUTPUT || j == 0) ? k : neighbour_row(g, k, op.gaxis[j], op.gdir[j]);
        nbr[j][i] = src;
    }
    const int tx = tid & 15, ty = tid >> 4;
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (T)0;
    __syncthreads();
    for (int j = 0; j < nblk; ++j) {
        for (int k0 = 0; k0 < kper; k0 += KC) {
            {   // A tile: 64 rows x 8, two consecutive elements per thread
                const int r = tid >> 2, kk = (tid & 3) * 2;
                const long long src = nbr[j][r];
                T a0 = (T)0, a1 = (T)0;
                if (src >= 0) {
                    const T* p = A + src * (long long)lda + k0 + kk;
                    if (k0 + kk < kper) a0 = p[0];
                    if (k0 + kk + 1 < kper) a1 = p[1];
                }
                As[kk][r] = a0;
                As[kk + 1][r] = a1;
            }
            {   // G tile: 8 x 64
                const int kk = tid >> 5, c = (tid & 31) * 2;
                const int grow = j * kper + k0 + kk;
                T g0 = (T)0, g1 = (T)0;
                if (k0 + kk < kper) {
                    if (col0 + c < ldg) g0 = Gop[(long long)grow * ldg + col0 + c];
                    if (col0 + c + 1 < ldg) g1 = Gop[(long long)grow * ldg + col0 + c + 1];
                }
                Gs[kk][c] = g0;
                Gs[kk][c + 1] = g1;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                T a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) b[jj] = Gs[kk][tx * 4 + jj];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) acc[i][jj] += a[i] * b[jj];
            }
            __syncthreads();
        }
    }
    // epilogue
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const long long k = row0 + ty * 4 + i;
        if (k >= g.M) continue;
        double dk = 1.0;
        double zq[kMaxBlocks];
        if (MODE == MODE_PROJECT) {
            dk = row_scale(g, op, rd, k);
            for (int q = 0; q < op.n_r1; ++q) zq[q] = rank1_value(g, op, rd, k, q);
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int c = col0 + tx * 4 + jj;
            if (c >= ldo) continue;
            double v = (double)acc[i][jj];
            if (MODE == MODE_PROJECT) {
                const int base = op.n_gather * kper;
                for (int q = 0; q < op.n_r1; ++q) v += zq[q] * (double)Gop[(long long)(base + q) * ldg + c];
                v *= dk;
            }
            Out[k * ldo + c] = (T)v;
        }
    }
}

// ---------------------------------------------------------------------------
// Householder TSQR: R factor of a tall matrix
// ---------------------------------------------------------------------------
//
// Each block owns a contiguous range of rows and keeps an upper-triangular R
// (KP x KP, FP64, packed by rows) in LDS.  Rows arrive in chunks of NG*BR;
// the NG threads of column c (adjacent lanes of one wave) hold BR rows each
// of the chunk's column c in registers (thread rg holds chunk rows
// i*NG + rg).  For every column j the reflector that zeroes the chunk's
// column j against R[j][j] is formed (LAPACK dlarfg convention:
// beta = -sign(alpha) ||(alpha, x)||, tau = (beta - alpha) / beta,
// v = x / (alpha - beta)) and applied to the columns c > j of R and of the
// chunk.  A column's dot product v^T T[:, c] runs down its threads'
// registers and across their lanes (DPP moves, shuffles beyond 16 lanes), so
// only the reflector crosses waves: the threads of column j + 1 form it as
// soon as their own update by reflector j is done, and one block barrier per
// column step publishes it.  The block writes its final R (KP x KP, zeros
// below the diagonal) to Rout[blk].
// ncols = k1 from the state; lda is the state's ldb when lda_from_state.
// rows_per_R > 0 (tree levels): the input is a stack of KP x KP R factors of
// which only the first rows_per_R rows can be non-zero (k1 <= rows_per_R);
// row r of the level is row r % rows_per_R of factor r / rows_per_R.
// (the body of k_tsqr for the block with index blk; also called by the
// persistent small-solve kernel with one block over all rows)
template <typename TS, int KP, int NG, int BR>
__device__ __forceinline__ void tsqr_body(const TS* __restrict__ A, int lda_static, int lda_from_state, int rows_per_R,
                                          long long nrows, long long rows_per_block, const DevState* __restrict__ st,
                                          double* __restrict__ Rout, int blk) {
    static_assert(NG <= 64 && (64 % NG) == 0, "the row groups of a column share one wave");
    // R's upper triangle, packed by rows (KP (KP + 1) / 2 entries: two
    // 128-column blocks fit one CU's LDS)
    __shared__ double R[KP * (KP + 1) / 2];
    __shared__ double vbuf[2][NG * BR];   // reflector of the current column, chunk row order
    __shared__ double tbuf[2];            // its tau; 0 when the column has nothing to annihilate
    const int tid = threadIdx.x;
    const int c = tid / NG, rg = tid % NG;
    const int ncols = st->k1;
    const int lda = lda_from_state ? st->ldb : lda_static;
    // entry (j, c), c >= j
    auto ri = [](int j, int c) __attribute__((always_inline)) { return j * (2 * KP - j + 1) / 2 + (c - j); };
    for (int idx = tid; idx < KP * (KP + 1) / 2; idx += KP * NG) R[idx] = 0.0;
    __syncthreads();
    const long long begin = (long long)blk * rows_per_block;
    long long end = begin + rows_per_block;
    if (end > nrows) end = nrows;
    double T[BR];
    // sum over the NG lanes of one column: lane swaps within quads, then the
    // mirror images within 8 and 16 lanes (DPP moves, no LDS round trip),
    // then shuffles; every pairing adds the same two values, so every lane
    // ends with the same bits
    auto colsum = [&](double x) __attribute__((always_inline)) {
        x = group_sum(x, NG < 32 ? NG : 32);
        if constexpr (NG == 64) x += __shfl_xor(x, 32, 64);
        return x;
    };
    // sums of BR terms in four interleaved chains
    auto sum4 = [&](auto term) __attribute__((always_inline)) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < BR; ++i) a[i & 3] += term(i);
        return (a[0] + a[1]) + (a[2] + a[3]);
    };
    // run by the NG threads of column col once every earlier reflector has
    // been applied to their values
    auto form = [&](int col, int p) __attribute__((always_inline)) {
        const double xn2 = colsum(sum4([&](int i) { return T[i] * T[i]; }));
        double tau = 0.0;
        if (xn2 != xn2) {
            if (rg == 0) R[ri(col, col)] = xn2;   // NaN in the data: poison R so it reaches the SVD
        } else if (xn2 > 0.0) {
            const double alpha = R[ri(col, col)];
            const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            const double scal = 1.0 / (alpha - beta);
#pragma unroll
            for (int i = 0; i < BR; ++i) vbuf[p][i * NG + rg] = T[i] * scal;
            if (rg == 0) R[ri(col, col)] = beta;
        }
        if (rg == 0) tbuf[p] = tau;
    };
    for (long long k0 = begin; k0 < end; k0 += NG * BR) {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
            const long long row = k0 + i * NG + rg;
            const long long src = rows_per_R > 0 ? (row / rows_per_R) * KP + row % rows_per_R : row;
            T[i] = (row < end && c < ncols) ? (double)A[src * lda + c] : 0.0;
        }
        if (c == 0 && ncols > 0) form(0, 0);
        __syncthreads();
        for (int j = 0; j < ncols; ++j) {
            const int p = j & 1;
            const double tau = tbuf[p];
            if (tau != 0.0 && c > j && c < ncols) {
                const double d = sum4([&](int i) { return vbuf[p][i * NG + rg] * T[i]; });
                const double rjc = R[ri(j, c)];
                const double f = tau * (rjc + colsum(d));
#pragma unroll
                for (int i = 0; i < BR; ++i) T[i] -= f * vbuf[p][i * NG + rg];
                if (rg == 0) R[ri(j, c)] = rjc - f;
            }
            if (c == j + 1 && c < ncols) form(j + 1, p ^ 1);
            __syncthreads();
        }
    }
    double* out = Rout + (size_t)blk * KP * KP;
    for (int idx = tid; idx < KP * KP; idx += KP * NG) {
        const int i = idx / KP, j = idx % KP;
        out[idx] = (j >= i) ? R[ri(i, j)] : 0.0;
    }
}

template <typename TS, int KP, int NG, int BR>
__global__ __launch_bounds__(KP* NG) void k_tsqr(const TS* __restrict__ A, int lda_static, int lda_from_state,
                                                 int rows_per_R, long long nrows, long long rows_per_block,
                                                 const DevState* __restrict__ st, double* __restrict__ Rout) {
    tsqr_body<TS, KP, NG, BR>(A, lda_static, lda_from_state, rows_per_R, nrows, rows_per_block, st, Rout, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Gram accumulation (Gram rounding): G = B^T B in FP64
// ---------------------------------------------------------------------------
// Each block accumulates the Gram matrix of its rows: thread (i, j) of a
// 16 x 16 grid owns a 4 x 4 (KPxKP / 64 x 64) block.  Partial sums go to
// Gout[blockIdx.x] and are added up by k_sum_parts.
template <typename TS, int KP>
__global__ __launch_bounds__(256) void k_gram(const TS* __restrict__ B, const DevState* __restrict__ st, long long nrows,
                                              long long rows_per_block, double* __restrict__ Gout) {
    constexpr int KC = 16;
    constexpr int TPR = KP / 16;   // entries per thread per dimension
    __shared__ double Bs[KC][KP + 1];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int ncols = st->k1, ldb = st->ldb;
    double acc[TPR][TPR];
#pragma unroll
    for (int i = 0; i < TPR; ++i)
#pragma unroll
        for (int j = 0; j < TPR; ++j) acc[i][j] = 0.0;
    const long long begin = (long long)blockIdx.x * rows_per_block;
    long long end = begin + rows_per_block;
    if (end > nrows) end = nrows;
    for (long long k0 = begin; k0 < end; k0 += KC) {
        for (int idx = tid; idx < KC * KP; idx += 256) {
            const int r = idx / KP, c = idx % KP;
            const long long row = k0 + r;
            Bs[r][c] = (row < end && c < ncols) ? (double)B[row * ldb + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            double a[TPR], b[TPR];
#pragma unroll
            for (int i = 0; i < TPR; ++i) a[i] = Bs[r][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < TPR; ++j) b[j] = Bs[r][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < TPR; ++i)
#pragma unroll
                for (int j = 0; j < TPR; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
    double* out = Gout + (size_t)blockIdx.x * KP * KP;
#pragma unroll
    for (int i = 0; i < TPR; ++i)
#pragma unroll
        for (int j = 0; j < TPR; ++j) out[(ty + 16 * i) * KP + tx + 16 * j] = acc[i][j];
}

// out[e] = sum_p parts[p][e] for e < n.  Each block owns 32 consecutive
// entries; its 8 waves-groups of 32 threads take every 8th part (coalesced
// 256-byte rows), then the 8 partial sums are added in a fixed order, so the
// result is deterministic.
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ parts, int nparts, int n,
                                                   double* __restrict__ out) {
    __shared__ double sh[8][32];
    const int e = blockIdx.x * 32 + (threadIdx.x & 31);
    const int q = threadIdx.x >> 5;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (e < n) {
        int p = q;
        for (; p + 24 < nparts; p += 32) {
            s0 += parts[(size_t)p * n + e];
            s1 += parts[(size_t)(p + 8) * n + e];
            s2 += parts[(size_t)(p + 16) * n + e];
            s3 += parts[(size_t)(p + 24) * n + e];
        }
        for (; p < nparts; p += 8) s0 += parts[(size_t)p * n + e];
    }
    sh[q][threadIdx.x & 31] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (q == 0 && e < n) {
        double t = 0.0;
        for (int k = 0; k < 8; ++k) t += sh[k][threadIdx.x];
        out[e] = t;
    }
}

// ---------------------------------------------------------------------------
// Inspection: explicit first core of the pending TT sum, rows [k0, k0 + nr)
// ---------------------------------------------------------------------------
template <typename TS>
__global__ void k_materialize(Geom g, OpDesc op, const DevState* __restrict__ st, const TS* __restrict__ Z,
                              RowData rd, long long k0, long long nr, double* __restrict__ out) {
    const int r1 = st->r1, ldz = st->ldz;
    const int R1 = op.n_rblk * r1 + op.n_r1;
    const long long total = nr * R1;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long kk = idx / R1;
        const int col = (int)(idx % R1);
        const long long k = k0 + kk;
        double v;
        if (col < op.n_rblk * r1 && op.hll) {
            // HLL: the r-block's gather blocks, each with its per-row weight
            const int t = col / r1, a = col % r1;
            v = 0.0;
            for (int j = 0; j < op.n_gather; ++j) {
                if (op.gterm[j] != t) continue;
                const int ax = op.gaxis[j];
                const long long s = op.gdir[j] == 0 ? k : neighbour_row(g, k, ax, op.gdir[j]);
                if (s < 0) continue;
                const double w = op.gwk[j] == 0 ? 1.0
                                                : hll_weight(op.gwk[j], hll_face_eps(g, rd, k, ax, -1),
                                                             hll_face_eps(g, rd, k, ax, 1), g.lam[ax]);
                v += w * (double)Z[s * ldz + a];
            }
        } else if (col < op.n_rblk * r1) {
            const int t = col / r1, a = col % r1;
            v = op.rcoef0[t] * (double)Z[k * ldz + a];
            if (op.rshift2[t] >= 0) {
                const int j = op.rshift2[t];
                const long long s = neighbour_row(g, k, op.gaxis[j], op.gdir[j]);
                if (s >= 0) v += op.rcoef2[t] * (double)Z[s * ldz + a];
            }
            if (op.rshift[t] >= 0) {
                const int j = op.rshift[t];
                const long long s = neighbour_row(g, k, op.gaxis[j], op.gdir[j]);
                if (s >= 0) v += op.rcoef[t] * (double)Z[s * ldz + a];
            }
        } else {
            v = rank1_value(g, op, rd, k, col - op.n_rblk * r1);
        }
        out[idx] = v * row_scale(g, op, rd, k);
    }
}

// Explicit Theta_new (R1 x N_theta x R2, block diagonal) and Phi_new (R2 x N_phi).
__global__ void k_sum_small_cores(Geom g, OpDesc op, const DevState* __restrict__ st, const double* __restrict__ Th,
                                  const double* __restrict__ Ph, const double* __restrict__ gtab,
                                  const double* __restrict__ htab, double* __restrict__ ThN, double* __restrict__ PhN) {
    const int r1 = st->r1, r2 = st->r2, nt = g.nt, npn = g.np;
    const int nrb = op.n_rblk, nr1 = op.n_r1;
    const int R1 = nrb * r1 + nr1, R2 = nrb * r2 + nr1;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < R1 * nt * R2; idx += gridDim.x * blockDim.x) {
        const int col = idx % R2, rl = idx / R2;
        const int row = rl / nt, l = rl % nt;
        double v = 0.0;
        if (row < nrb * r1) {
            const int t = row / r1, a = row % r1;
            if (col >= t * r2 && col < (t + 1) * r2)
                v = Th[((size_t)a * nt + l) * r2 + (col - t * r2)] * gtab[op.rfac[t] * nt + l];
        } else {
            const int q = row - nrb * r1;
            if (col == nrb * r2 + q) v = gtab[op.r1fac[q] * nt + l];
        }
        ThN[idx] = v;
    }
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < R2 * npn; idx += gridDim.x * blockDim.x) {
        const int col = idx / npn, p = idx % npn;
        double v;
        if (col < nrb * r2) {
            const int t = col / r2, b = col % r2;
            v = Ph[(size_t)b * npn + p] * htab[op.rfac[t] * npn + p];
        } else {
            v = htab[op.r1fac[col - nrb * r2] * npn + p];
        }
        PhN[idx] = v;
    }
}

// Column sums of Z (r1 entries), for diagnostics: one pass over Z.  Block b
// of 1024 threads sums rows b*16 + rl (rl = thread / 64) with stride 16 *
// gridDim.x, four rows in flight per lane; lane c of a wave holds column
// c0 + c (64-column tiles), so a wave reads contiguous row segments.  The 16
// row lanes are added in a fixed order and the block writes parts[b * 128 + a]
// (the host adds the blocks).
template <typename TS>
__global__ __launch_bounds__(1024) void k_colsum(const DevState* __restrict__ st, const TS* __restrict__ Z, long long M,
                                                 double* __restrict__ parts) {
    const int r1 = st->r1, ldz = st->ldz;
    __shared__ double sh[16][64];
    const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
    const long long stride = (long long)gridDim.x * 16;
    for (int c0 = 0; c0 < r1; c0 += 64) {
        const int a = c0 + c;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (a < r1) {
            long long k = (long long)blockIdx.x * 16 + rl;
            for (; k + 3 * stride < M; k += 4 * stride) {
                s0 += (double)Z[k * ldz + a];
                s1 += (double)Z[(k + stride) * ldz + a];
                s2 += (double)Z[(k + 2 * stride) * ldz + a];
                s3 += (double)Z[(k + 3 * stride) * ldz + a];
            }
            for (; k < M; k += stride) s0 += (double)Z[k * ldz + a];
        }
        sh[rl][c] = (s0 + s1) + (s2 + s3);
        __syncthreads();
        if (rl == 0 && a < r1) {
            double t = 0.0;
            for (int i = 0; i < 16; ++i) t += sh[i][c];
            parts[(size_t)blockIdx.x * 128 + a] = t;
        }
        __syncthreads();
    }
}

}  // namespace ttrt
