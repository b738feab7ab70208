// Single-workgroup FP64 kernels on the small cores (Theta, Phi and the R factor
// of the first core).  All matrices here are at most a few hundred rows and
// columns; they live in global scratch (L2 resident) and are processed by one
// workgroup with block-level reductions.
#pragma once

#include "tt_common.hpp"

namespace ttrt {

constexpr int kSmallThreads = 1024;

// Operator description shared by the prep, projection and materialise kernels.
struct OpDesc {
    int n_rblk;                 // rank-r blocks of the TT sum (identity + streaming terms)
    int rfac[kMaxBlocks];       // angular factor row of each r-block
    int rshift[kMaxBlocks];     // gather block holding the shifted copy (-1: none)
    double rcoef0[kMaxBlocks];  // coefficient on the unshifted Z
    double rcoef[kMaxBlocks];   // coefficient on the shifted copy
    int n_gather;               // gather blocks: 0 = Z itself, then shifted copies of Z
    int gaxis[kMaxBlocks];
    int gdir[kMaxBlocks];
    int n_r1;                   // rank-1 blocks (boundary columns, emission)
    int r1fac[kMaxBlocks];
    int r1kind[kMaxBlocks];     // 0: emission c dt kappa eps, 1: inflow column
    int r1face[kMaxBlocks];
    int scale_d;                // rows scaled by d = 1/(1 + c dt kappa)
};

// ---------------------------------------------------------------------------
// block-level helpers
// ---------------------------------------------------------------------------

__device__ inline double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Householder QR of the m x n column-major matrix A (A[i + j*lda]) by the
// whole block.  k = min(m, n) reflectors; on return the upper triangle holds
// R (k x n) and the strict lower part of the first k columns holds the
// reflector tails (unit leading entry implied).  tau receives k scalars.
// Each column of the trailing matrix is handled by a group of `gs` threads.
__device__ void block_householder_qr(double* A, int lda, int m, int n, double* tau, double* red) {
    const int k = m < n ? m : n;
    const int nt = blockDim.x;
    for (int j = 0; j < k; ++j) {
        double part = 0.0;
        for (int i = j + 1 + threadIdx.x; i < m; i += nt) part += A[i + (size_t)j * lda] * A[i + (size_t)j * lda];
        const double xn2 = block_sum(part, red);
        const double alpha = A[j + (size_t)j * lda];
        double t = 0.0, beta = alpha, scal = 0.0;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            t = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        __syncthreads();
        if (xn2 > 0.0) {
            for (int i = j + 1 + threadIdx.x; i < m; i += nt) A[i + (size_t)j * lda] *= scal;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            A[j + (size_t)j * lda] = beta;
            tau[j] = t;
        }
        if (t != 0.0) {
            // trailing columns c = j+1..n-1; groups of gs threads per column
            const int ncol = n - j - 1;
            int gs = 1;
            while (gs < 32 && gs * 2 * ncol <= nt) gs *= 2;
            const int g = threadIdx.x / gs, gl = threadIdx.x % gs, ngroups = nt / gs;
            for (int cc = g; cc < ncol + ((ngroups - ncol % ngroups) % ngroups); cc += ngroups) {
                const int c = j + 1 + cc;
                double w = 0.0;
                if (cc < ncol) {
                    if (gl == 0) w = A[j + (size_t)c * lda];
                    for (int i = j + 1 + gl; i < m; i += gs) w += A[i + (size_t)j * lda] * A[i + (size_t)c * lda];
                }
                for (int off = gs >> 1; off >= 1; off >>= 1) w += __shfl_xor(w, off, 64);
                if (cc < ncol) {
                    const double f = t * w;
                    if (gl == 0) A[j + (size_t)c * lda] -= f;
                    for (int i = j + 1 + gl; i < m; i += gs) A[i + (size_t)c * lda] -= f * A[i + (size_t)j * lda];
                }
            }
        }
        __syncthreads();
    }
}

// Explicit Q (m x k, column-major, Q[i + c*ldq]) from the reflectors left in A.
__device__ void block_form_q(const double* A, int lda, int m, int k, const double* tau, double* Q, int ldq) {
    const int nt = blockDim.x;
    for (int idx = threadIdx.x; idx < m * k; idx += nt) {
        const int i = idx % m, c = idx / m;
        Q[i + (size_t)c * ldq] = (i == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = k - 1; j >= 0; --j) {
        const double t = tau[j];
        if (t != 0.0) {
            const int ncol = k - j;
            int gs = 1;
            while (gs < 32 && gs * 2 * ncol <= nt) gs *= 2;
            const int g = threadIdx.x / gs, gl = threadIdx.x % gs, ngroups = nt / gs;
            for (int cc = g; cc < ncol + ((ngroups - ncol % ngroups) % ngroups); cc += ngroups) {
                const int c = j + cc;
                double w = 0.0;
                if (cc < ncol) {
                    if (gl == 0) w = Q[j + (size_t)c * ldq];
                    for (int i = j + 1 + gl; i < m; i += gs) w += A[i + (size_t)j * lda] * Q[i + (size_t)c * ldq];
                }
                for (int off = gs >> 1; off >= 1; off >>= 1) w += __shfl_xor(w, off, 64);
                if (cc < ncol) {
                    const double f = t * w;
                    if (gl == 0) Q[j + (size_t)c * ldq] -= f;
                    for (int i = j + 1 + gl; i < m; i += gs) Q[i + (size_t)c * ldq] -= f * A[i + (size_t)j * lda];
                }
            }
        }
        __syncthreads();
    }
}

// One-sided (Hestenes) Jacobi on the n columns of the m x n column-major
// matrix A: rotates column pairs until all are orthogonal, so that A V = U S.
// When V is non-null the rotations are accumulated into the n x n matrix V
// (column-major, V[i + j*n], initialised to I here).  Pairs are scheduled by
// the round-robin tournament so each round touches disjoint columns.
__device__ void block_jacobi(double* A, int lda, int m, int n, double* V, int* flag, double* red) {
    const int nt = blockDim.x;
    if (V) {
        for (int idx = threadIdx.x; idx < n * n; idx += nt) V[idx] = (idx % n == idx / n) ? 1.0 : 0.0;
    }
    if (n < 2) {
        __syncthreads();
        return;
    }
    const int np = (n + 1) & ~1;          // players (a dummy when n is odd)
    const int npairs = np / 2;
    int gs = 64;                          // threads per pair (power of two, <= 64)
    while (gs > 1 && gs * npairs > nt) gs >>= 1;
    const int pair = threadIdx.x / gs, gl = threadIdx.x % gs;
    const double eps = 1e-15;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            for (int pp = pair; pp < npairs; pp += nt / gs) {
                // positions pp and np-1-pp; position 0 is fixed
                int pa = pp, pb = np - 1 - pp;
                int a = pa == 0 ? 0 : ((pa - 1 + round) % (np - 1)) + 1;
                int b = pb == 0 ? 0 : ((pb - 1 + round) % (np - 1)) + 1;
                if (a > b) { int t = a; a = b; b = t; }
                const bool real = b < n;
                double al = 0.0, be = 0.0, ga = 0.0;
                if (real) {
                    for (int i = gl; i < m; i += gs) {
                        const double x = A[i + (size_t)a * lda], y = A[i + (size_t)b * lda];
                        al += x * x; be += y * y; ga += x * y;
                    }
                }
                for (int off = gs >> 1; off >= 1; off >>= 1) {
                    al += __shfl_xor(al, off, 64);
                    be += __shfl_xor(be, off, 64);
                    ga += __shfl_xor(ga, off, 64);
                }
                if (real && ga != 0.0 && fabs(ga) > eps * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                    for (int i = gl; i < m; i += gs) {
                        const double x = A[i + (size_t)a * lda], y = A[i + (size_t)b * lda];
                        A[i + (size_t)a * lda] = c * x - s * y;
                        A[i + (size_t)b * lda] = s * x + c * y;
                    }
                    if (V) {
                        for (int i = gl; i < n; i += gs) {
                            const double x = V[i + (size_t)a * n], y = V[i + (size_t)b * n];
                            V[i + (size_t)a * n] = c * x - s * y;
                            V[i + (size_t)b * n] = s * x + c * y;
                        }
                    }
                    if (gl == 0) *flag = 1;
                }
            }
            __syncthreads();
        }
        const int f = *flag;
        __syncthreads();
        if (!f) break;
    }
}

// Column norms of A (m x n) into s[0..n), then a descending order in perm
// (ties by index).
__device__ void block_colnorms_sorted(const double* A, int lda, int m, int n, double* s, int* perm) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < m; ++i) acc += A[i + (size_t)j * lda] * A[i + (size_t)j * lda];
        s[j] = sqrt(acc);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double v = s[j];
        int rank = 0;
        for (int i = 0; i < n; ++i) {
            const double u = s[i];
            if (u > v || (u == v && i < j)) ++rank;
        }
        perm[rank] = j;
    }
    __syncthreads();
}

// Smallest r >= 1 with sqrt(sum_{i>=r} s_sorted[i]^2) <= delta, capped.
__device__ inline int delta_rank(const double* s, const int* perm, int n, double delta, int cap) {
    double tail = 0.0;
    int r = n;
    for (int i = n - 1; i >= 1; --i) {
        const double v = s[perm[i]];
        tail += v * v;
        if (sqrt(tail) <= delta) r = i; else break;
    }
    if (r > cap) r = cap;
    if (r < 1) r = 1;
    return r;
}

// ---------------------------------------------------------------------------
// prep: right-to-left orthogonalisation of the small cores of the TT sum
// ---------------------------------------------------------------------------
//
// The pending TT sum has Phi_new (R2 x N_phi, stacked), Theta_new (R1 x N_theta
// x R2, block diagonal) and the virtual first core Z_new.  This kernel
//  1. forms Phi_new^T and its QR:   Phi_new = L_Phi Q_Phi,
//  2. forms Theta' = Theta_new x_3 L_Phi and the QR of its row unfolding:
//     Theta'_(1) = L_Theta Q_Theta,
//  3. folds L_Theta with the streaming coefficients into the operand G of the
//     gather contraction B = d .* (sum_j (O_j Z) G_j + rank-1 terms), so that
//     B = Z_new L_Theta (the projected first core).
// Writes Q_Theta, Q_Phi, L_Theta and G; R1, R2, k1, k2 and ldb go to the state.
struct SmallScratch {
    double* A1;    // N_phi x R2cap
    double* Q1;    // N_phi x k2cap
    double* A2;    // (N_theta k2cap) x R1cap
    double* Q2;    // (N_theta k2cap) x k1cap
    double* tau;   // max(R1cap, R2cap)
    double* J;     // Jacobi matrix, k1cap x k1cap
    double* Th2;   // r1cap x N_theta k2cap
    double* C2;    // r1cap N_theta x k2cap
    double* V2;    // k2cap x k2cap
    double* sv;    // k1cap + k2cap singular values
    int* perm;     // k1cap + k2cap
    int* flag;
};

template <typename TC>
__global__ __launch_bounds__(kSmallThreads) void k_prep(Geom g, OpDesc op, DevState* st, const double* __restrict__ Th,
                                                        const double* __restrict__ Ph, const double* __restrict__ gtab,
                                                        const double* __restrict__ htab, SmallScratch sc,
                                                        double* __restrict__ LTh, int ldl, double* __restrict__ QTh,
                                                        double* __restrict__ QPh, TC* __restrict__ Gop, int ldgcap) {
    __shared__ double red[16];
    const int nt = g.nt, npn = g.np;
    const int r1 = st->r1, r2 = st->r2, ldz = st->ldz;
    const int nrb = op.n_rblk, nr1 = op.n_r1;
    const int R1 = nrb * r1 + nr1, R2 = nrb * r2 + nr1;
    const int k2 = R2 < npn ? R2 : npn;
    const int m2 = nt * k2;
    const int k1 = R1 < m2 ? R1 : m2;
    const int ldb = ld_for_rank(k1);

    // 1. A1 = Phi_new^T (N_phi x R2, column-major)
    for (int idx = threadIdx.x; idx < npn * R2; idx += blockDim.x) {
        const int p = idx % npn, col = idx / npn;
        double v;
        if (col < nrb * r2) {
            const int t = col / r2, b = col % r2;
            v = Ph[(size_t)b * npn + p] * htab[op.rfac[t] * npn + p];
        } else {
            v = htab[op.r1fac[col - nrb * r2] * npn + p];
        }
        sc.A1[p + (size_t)col * npn] = v;
    }
    __syncthreads();
    block_householder_qr(sc.A1, npn, npn, R2, sc.tau, red);
    block_form_q(sc.A1, npn, npn, k2, sc.tau, sc.Q1, npn);
    // Q_Phi = Q1^T (k2 x N_phi)
    for (int idx = threadIdx.x; idx < k2 * npn; idx += blockDim.x) {
        const int c = idx / npn, p = idx % npn;
        QPh[(size_t)c * npn + p] = sc.Q1[p + (size_t)c * npn];
    }
    // 2. A2 = Theta'^T ((N_theta k2) x R1, column-major); L_Phi[col][c] = R_Phi[c][col]
    for (int idx = threadIdx.x; idx < m2 * R1; idx += blockDim.x) {
        const int rowA = idx % m2, row = idx / m2;
        const int l = rowA / k2, c = rowA % k2;
        double v = 0.0;
        if (row < nrb * r1) {
            const int t = row / r1, a = row % r1;
            const double* th = Th + ((size_t)a * nt + l) * r2;
            for (int b = 0; b < r2; ++b) {
                const int col = t * r2 + b;
                const double lphi = (c <= col) ? sc.A1[c + (size_t)col * npn] : 0.0;
                v += th[b] * lphi;
            }
            v *= gtab[op.rfac[t] * nt + l];
        } else {
            const int q = row - nrb * r1;
            const int col = nrb * r2 + q;
            const double lphi = (c <= col) ? sc.A1[c + (size_t)col * npn] : 0.0;
            v = gtab[op.r1fac[q] * nt + l] * lphi;
        }
        sc.A2[rowA + (size_t)row * m2] = v;
    }
    __syncthreads();
    block_householder_qr(sc.A2, m2, m2, R1, sc.tau, red);
    block_form_q(sc.A2, m2, m2, k1, sc.tau, sc.Q2, m2);
    // Q_Theta = Q2^T (k1 x N_theta k2), L_Theta = R^T (R1 x k1)
    for (int idx = threadIdx.x; idx < k1 * m2; idx += blockDim.x) {
        const int i = idx / m2, rowA = idx % m2;
        QTh[(size_t)i * m2 + rowA] = sc.Q2[rowA + (size_t)i * m2];
    }
    for (int idx = threadIdx.x; idx < R1 * k1; idx += blockDim.x) {
        const int row = idx / k1, i = idx % k1;
        LTh[(size_t)row * ldl + i] = (i <= row) ? sc.A2[i + (size_t)row * m2] : 0.0;
    }
    __syncthreads();
    // 3. gather operand G: rows (gather block j, a < ldz), then rank-1 rows; ldb columns
    const int grows = op.n_gather * ldz + nr1;
    for (int idx = threadIdx.x; idx < grows * ldb; idx += blockDim.x) {
        const int row = idx / ldb, col = idx % ldb;
        double v = 0.0;
        if (col < k1) {
            if (row < op.n_gather * ldz) {
                const int j = row / ldz, a = row % ldz;
                if (a < r1) {
                    for (int t = 0; t < nrb; ++t) {
                        const double l = LTh[(size_t)(t * r1 + a) * ldl + col];
                        if (j == 0) v += op.rcoef0[t] * l;
                        if (op.rshift[t] == j) v += op.rcoef[t] * l;
                    }
                }
            } else {
                const int q = row - op.n_gather * ldz;
                v = LTh[(size_t)(nrb * r1 + q) * ldl + col];
            }
        }
        Gop[(size_t)row * ldb + col] = (TC)v;
    }
    if (threadIdx.x == 0) {
        st->R1 = R1; st->R2 = R2; st->k1 = k1; st->k2 = k2; st->ldb = ldb;
        if (R1 > st->max_R1) st->max_R1 = R1;
        if (R2 > st->max_R2) st->max_R2 = R2;
    }
}

// ---------------------------------------------------------------------------
// SVD chain: truncated SVDs of both bonds from the R factor of B = Z_new L_Theta
// ---------------------------------------------------------------------------
//
// Input: R_B (k1 x k1, upper triangular, row-major with leading dim ldr) with
// B = Q_B R_B.  The bond-1 SVD of the right-orthogonalised TT is the SVD of B:
// one-sided Jacobi on R_B^T gives R_B^T W = U S, whose normalised columns are
// the right singular vectors V of R_B (and of B).  The rest follows the
// left-to-right sweep of TT-SVD rounding with the norm kept in Z:
//   Z_out = B V_r, Theta'' = V_r^T Q_Theta, SVD of diag(S_r) Theta''
//   ((r1 N_theta) x k2) -> V2, S2; Theta_out = Theta'' x_3 V2_r,
//   Phi_out = V2_r^T Q_Phi.
// gram != 0: the input is the Gram matrix G = B^T B (k1 x k1, symmetric)
// instead; a two-sided Jacobi eigensolver gives V and S = sqrt(eig).
template <typename TC>
__global__ __launch_bounds__(kSmallThreads) void k_svd_chain(Geom g, DevState* st, const double* __restrict__ RB, int ldr,
                                                             int gram, const double* __restrict__ QTh,
                                                             const double* __restrict__ QPh, double tol, int cap1,
                                                             int cap2, SmallScratch sc, double* __restrict__ ThOut,
                                                             double* __restrict__ PhOut, TC* __restrict__ Vout,
                                                             double* __restrict__ sv_out) {
    __shared__ double red[16];
    __shared__ int sh_r[2];
    const int nt = g.nt, npn = g.np;
    const int k1 = st->k1, k2 = st->k2;
    const int m2 = nt * k2;
    double* J = sc.J;
    // J = R_B^T, column-major k1 x k1: column j holds row j of R_B
    for (int idx = threadIdx.x; idx < k1 * k1; idx += blockDim.x) {
        const int i = idx % k1, j = idx / k1;
        J[i + (size_t)j * k1] = RB[(size_t)j * ldr + i];
    }
    __syncthreads();
    double* s1 = sc.sv;
    int* p1 = sc.perm;
    if (!gram) {
        block_jacobi(J, k1, k1, k1, nullptr, sc.flag, red);
        block_colnorms_sorted(J, k1, k1, k1, s1, p1);
    } else {
        // G symmetric: cyclic two-sided Jacobi G <- W^T G W, W accumulated in A2
        double* W = sc.A2;
        for (int idx = threadIdx.x; idx < k1 * k1; idx += blockDim.x) W[idx] = (idx % k1 == idx / k1) ? 1.0 : 0.0;
        __syncthreads();
        const int np_ = (k1 + 1) & ~1, npairs = np_ / 2;
        for (int sweep = 0; sweep < 60 && k1 > 1; ++sweep) {
            if (threadIdx.x == 0) *sc.flag = 0;
            __syncthreads();
            for (int round = 0; round < np_ - 1; ++round) {
                // one thread per pair decides its rotation; rotations of disjoint pairs commute
                __shared__ double cs[2 * 128];
                __shared__ int pa_[128], pb_[128];
                for (int pp = threadIdx.x; pp < npairs; pp += blockDim.x) {
                    int pa = pp, pb = np_ - 1 - pp;
                    int a = pa == 0 ? 0 : ((pa - 1 + round) % (np_ - 1)) + 1;
                    int b = pb == 0 ? 0 : ((pb - 1 + round) % (np_ - 1)) + 1;
                    if (a > b) { int t = a; a = b; b = t; }
                    double c = 1.0, s = 0.0;
                    if (b < k1) {
                        const double app = J[a + (size_t)a * k1], aqq = J[b + (size_t)b * k1], apq = J[a + (size_t)b * k1];
                        if (apq != 0.0 && fabs(apq) > 1e-15 * sqrt(fabs(app * aqq))) {
                            const double zeta = (aqq - app) / (2.0 * apq);
                            const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                            c = 1.0 / sqrt(1.0 + t * t);
                            s = c * t;
                            *sc.flag = 1;
                        }
                    }
                    cs[2 * pp] = c; cs[2 * pp + 1] = s; pa_[pp] = a; pb_[pp] = b;
                }
                __syncthreads();
                // columns: J <- J R, W <- W R
                for (int idx = threadIdx.x; idx < npairs * k1; idx += blockDim.x) {
                    const int pp = idx / k1, i = idx % k1;
                    const int a = pa_[pp], b = pb_[pp];
                    if (b >= k1) continue;
                    const double c = cs[2 * pp], s = cs[2 * pp + 1];
                    const double x = J[i + (size_t)a * k1], y = J[i + (size_t)b * k1];
                    J[i + (size_t)a * k1] = c * x - s * y;
                    J[i + (size_t)b * k1] = s * x + c * y;
                    const double u = W[i + (size_t)a * k1], w = W[i + (size_t)b * k1];
                    W[i + (size_t)a * k1] = c * u - s * w;
                    W[i + (size_t)b * k1] = s * u + c * w;
                }
                __syncthreads();
                // rows: J <- R^T J
                for (int idx = threadIdx.x; idx < npairs * k1; idx += blockDim.x) {
                    const int pp = idx / k1, i = idx % k1;
                    const int a = pa_[pp], b = pb_[pp];
                    if (b >= k1) continue;
                    const double c = cs[2 * pp], s = cs[2 * pp + 1];
                    const double x = J[a + (size_t)i * k1], y = J[b + (size_t)i * k1];
                    J[a + (size_t)i * k1] = c * x - s * y;
                    J[b + (size_t)i * k1] = s * x + c * y;
                }
                __syncthreads();
            }
            const int f = *sc.flag;
            __syncthreads();
            if (!f) break;
        }
        for (int j = threadIdx.x; j < k1; j += blockDim.x) s1[j] = sqrt(fmax(J[j + (size_t)j * k1], 0.0));
        __syncthreads();
        for (int j = threadIdx.x; j < k1; j += blockDim.x) {
            const double v = s1[j];
            int rank = 0;
            for (int i = 0; i < k1; ++i) {
                const double u = s1[i];
                if (u > v || (u == v && i < j)) ++rank;
            }
            p1[rank] = j;
        }
        __syncthreads();
        // right singular vectors are the eigenvectors: copy W into J scaled by s so the
        // normalisation below is shared with the QR path
        for (int idx = threadIdx.x; idx < k1 * k1; idx += blockDim.x) {
            const int j = idx / k1;
            J[idx] = W[idx] * s1[j];
        }
        __syncthreads();
    }
    // norm, threshold, bond-1 rank
    double part = 0.0;
    for (int j = threadIdx.x; j < k1; j += blockDim.x) part += s1[j] * s1[j];
    const double norm2 = block_sum(part, red);
    const double norm = sqrt(norm2);
    const double delta = tol * norm / sqrt(2.0);
    if (threadIdx.x == 0) sh_r[0] = delta_rank(s1, p1, k1, delta, cap1);
    __syncthreads();
    const int r1n = sh_r[0];
    const int ldzn = ld_for_rank(r1n);
    const int ldb = st->ldb;
    // V_r (k1 x r1n): normalised columns of J in descending order
    for (int idx = threadIdx.x; idx < ldb * ldzn; idx += blockDim.x) {
        const int i = idx / ldzn, a = idx % ldzn;
        double v = 0.0;
        if (i < k1 && a < r1n) {
            const int j = p1[a];
            const double s = s1[j];
            v = (s > 0.0) ? J[i + (size_t)j * k1] / s : (i == j ? 1.0 : 0.0);
        }
        Vout[(size_t)i * ldzn + a] = (TC)v;
    }
    // Theta'' = V_r^T Q_Theta (r1n x N_theta k2), and C2 = diag(S_r) Theta''
    // reshaped ((r1n N_theta) x k2) column-major
    for (int idx = threadIdx.x; idx < r1n * m2; idx += blockDim.x) {
        const int a = idx / m2, col = idx % m2;
        const int j = p1[a];
        const double s = s1[j];
        double acc = 0.0;
        for (int i = 0; i < k1; ++i) {
            const double v = (s > 0.0) ? J[i + (size_t)j * k1] / s : (i == j ? 1.0 : 0.0);
            acc += v * QTh[(size_t)i * m2 + col];
        }
        sc.Th2[(size_t)a * m2 + col] = acc;
        const int l = col / k2, c = col % k2;
        sc.C2[(a * nt + l) + (size_t)c * (r1n * nt)] = s * acc;
    }
    __syncthreads();
    const int mC = r1n * nt;
    block_jacobi(sc.C2, mC, mC, k2, sc.V2, sc.flag, red);
    double* s2 = sc.sv + k1;
    int* p2 = sc.perm + k1;
    block_colnorms_sorted(sc.C2, mC, mC, k2, s2, p2);
    if (threadIdx.x == 0) {
        sh_r[1] = delta_rank(s2, p2, k2, delta, cap2 < k2 ? cap2 : k2);
    }
    __syncthreads();
    const int r2n = sh_r[1];
    // Theta_out[a][l][q] = sum_c Theta''[a][l][c] V2[c][p2[q]];  Phi_out[q][p] = sum_c V2[c][p2[q]] Q_Phi[c][p]
    for (int idx = threadIdx.x; idx < r1n * nt * r2n; idx += blockDim.x) {
        const int q = idx % r2n, al = idx / r2n;
        const int a = al / nt, l = al % nt;
        const int jq = p2[q];
        double acc = 0.0;
        for (int c = 0; c < k2; ++c) acc += sc.Th2[(size_t)a * m2 + l * k2 + c] * sc.V2[c + (size_t)jq * k2];
        ThOut[idx] = acc;
    }
    for (int idx = threadIdx.x; idx < r2n * npn; idx += blockDim.x) {
        const int q = idx / npn, p = idx % npn;
        const int jq = p2[q];
        double acc = 0.0;
        for (int c = 0; c < k2; ++c) acc += sc.V2[c + (size_t)jq * k2] * QPh[(size_t)c * npn + p];
        PhOut[idx] = acc;
    }
    // discarded tail and statistics
    double d1 = 0.0;
    for (int a = r1n + threadIdx.x; a < k1; a += blockDim.x) d1 += s1[p1[a]] * s1[p1[a]];
    for (int q = r2n + threadIdx.x; q < k2; q += blockDim.x) d1 += s2[p2[q]] * s2[p2[q]];
    const double disc2 = block_sum(d1, red);
    for (int j = threadIdx.x; j < k1; j += blockDim.x) sv_out[j] = s1[p1[j]];
    if (threadIdx.x == 0) {
        st->r1n = r1n;
        st->r2n = r2n;
        st->ldzn = ldzn;
        st->norm = norm;
        st->disc2 = disc2;
        if (!(norm2 < 1e300) || norm2 != norm2) st->nan_flag = 1;
        st->rounds += 1;
        const double M = (double)g.M, R1 = (double)st->R1, kk = (double)k1;
        st->fl[0] += 2.0 * M * R1 * kk;
        st->fl[1] += gram ? 2.0 * M * kk * kk : 2.0 * M * kk * kk - 2.0 / 3.0 * kk * kk * kk;
        st->fl[2] += 2.0 * M * kk * (double)r1n;
    }
}

// Make the truncated cores current.
__global__ void k_commit(DevState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->r1 = st->r1n;
        st->r2 = st->r2n;
        st->ldz = st->ldzn;
    }
}

}  // namespace ttrt
