// Single-workgroup FP64 kernels on the small cores (Theta, Phi and the R factor
// or Gram matrix of the projected first core).  Working matrices live in LDS
// when they fit (dynamic shared memory), otherwise in global scratch.
#pragma once

#include "tt_common.hpp"

namespace ttrt {

constexpr int kSmallThreads = 1024;
// Sweep stop of the Gram-path eigensolver (largest rotation tangent of the
// last sweep): the next sweep would rotate by ~1e-10, far below the FP32 data.
constexpr double kGramSweepTol = 1e-5;
constexpr int kSmallLdsBytes = 150 * 1024;

// Operator description shared by the prep, projection and materialise kernels.
struct OpDesc {
    int n_rblk;                 // rank-r blocks of the TT sum (identity + streaming terms)
    int rfac[kMaxBlocks];       // angular factor row of each r-block
    int rshift[kMaxBlocks];     // gather block holding the shifted copy (-1: none)
    double rcoef0[kMaxBlocks];  // coefficient on the unshifted Z
    double rcoef[kMaxBlocks];   // coefficient on the shifted copy
    int rshift2[kMaxBlocks];    // second shifted copy (the other neighbour; -1: none)
    double rcoef2[kMaxBlocks];
    int n_gather;               // gather blocks: 0 = Z itself, then shifted copies of Z
    int gaxis[kMaxBlocks];
    int gdir[kMaxBlocks];
    int n_r1;                   // rank-1 blocks (boundary columns, emission)
    int r1fac[kMaxBlocks];
    int r1kind[kMaxBlocks];     // 0: emission c dt kappa eps (+ scattering), 1: inflow column
    int r1face[kMaxBlocks];
    double r1coef[kMaxBlocks];  // inflow column: value r1coef * ghost on the face's cell layer
    int scale_d;                // rows scaled by d = 1/(1 + c dt kappa)
    // HLL flux: every gather block belongs to one r-block (gterm) with unit
    // coefficient and carries a per-row weight of kind gwk (0: 1; 1..6: the
    // centre / minus / plus coefficient of the n^+ (1..3) or n^- (4..6) term,
    // built from the row's interface factors); inflow columns of kind 2 take
    // (1 + eps) / 2 (r1hll 1) or (1 - eps) / 2 (r1hll 2) of the face's factor
    int hll;
    int gterm[kMaxBlocks];
    int gwk[kMaxBlocks];
    int r1hll[kMaxBlocks];
};

// Global fallbacks and persistent small buffers of the rounding.
struct SmallScratch {
    double* A1;    // N_phi x R2cap
    double* Q1;    // N_phi x N_phi + R2cap x k2cap
    double* A2;    // max((N_theta k2cap) x R1cap, k1cap x (k1cap | 1))
    double* Q2;    // (N_theta k2cap) x k1cap
    double* tau;   // max(R1cap, R2cap)
    double* J;     // k1cap x (k1cap | 1)
    double* Th2;   // r1cap x N_theta k2cap
    double* C2;    // r1cap N_theta x k2cap
    double* V2;    // k2cap x k2cap
    double* sv;    // 3 k1cap + k2cap
    int* perm;     // k1cap + k2cap
    int* flag;
    double* W;     // k1cap x (k1cap | 1) rotations of the first-bond Jacobi
    double* Wkeep; // k1cap x k1cap right singular vectors of the previous round
};

// Bump allocator over the dynamic LDS block, falling back to global memory.
struct LdsCarver {
    double* base;
    size_t used, cap;   // in doubles
    __device__ double* take(size_t n, double* fallback) {
        n = (n + 1) & ~(size_t)1;
        if (used + n <= cap) {
            double* p = base + used;
            used += n;
            return p;
        }
        return fallback;
    }
};

// ---------------------------------------------------------------------------
// block-level helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ double block_sum(double v, double* red) {
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
// whole block.  k = min(m, n) reflectors (LAPACK dlarfg convention); on return
// the upper triangle holds R (k x n) and the strict lower part of the first k
// columns holds the reflector tails (unit leading entry implied).
__device__ __forceinline__ void block_householder_qr(double* A, int lda, int m, int n, double* tau, double* red) {
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
__device__ __forceinline__ void block_form_q(const double* A, int lda, int m, int k, const double* tau, double* Q, int ldq) {
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

// Lane exchange within groups of 2..16 consecutive lanes by DPP (VALU
// latency instead of an LDS crossbar round trip).  CTRL: 0xB1 quad xor 1,
// 0x4E quad xor 2, 0x141 mirror within 8 lanes, 0x140 mirror within 16 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_swap(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over aligned groups of gs in {1, 2, 4, 8, 16, 32} consecutive lanes;
// every lane of a group receives the group total.
__device__ __forceinline__ double group_sum(double v, int gs) {
    if (gs >= 2) v += dpp_swap<0xB1>(v);
    if (gs >= 4) v += dpp_swap<0x4E>(v);
    if (gs >= 8) v += dpp_swap<0x141>(v);
    if (gs >= 16) v += dpp_swap<0x140>(v);
    if (gs >= 32) v += __shfl_xor(v, 16, 64);
    return v;
}

// 1/x and 1/sqrt(x) from the hardware estimates refined by two Newton steps
// (x finite and positive where used).
__device__ __forceinline__ double rcp_refined(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double rsq_refined(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// Jacobi rotation annihilating the off-diagonal g of [[a, g], [g, b]]:
// zeta = (b - a) / 2g, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) (the smaller
// root of t^2 + 2 zeta t - 1 = 0), c = 1/sqrt(1 + t^2), s = c t.  Applied as
// x' = c x - s y, y' = s x + c y on the column pair.
__device__ __forceinline__ void jacobi_rotation(double a, double b, double g, double* c, double* s, double* t) {
    const double zeta = (b - a) * rcp_refined(2.0 * g);
    double tt;
    if (fabs(zeta) > 1e150) {
        tt = 0.5 * rcp_refined(zeta);
    } else {
        const double q = fma(zeta, zeta, 1.0);
        const double root = q * rsq_refined(q);
        tt = copysign(rcp_refined(fabs(zeta) + root), zeta);
    }
    const double cc = rsq_refined(fma(tt, tt, 1.0));
    *c = cc;
    *s = cc * tt;
    *t = tt;
}

// Pair (a, b) of round `round` in the round-robin tournament over np players
// (player 0 fixed, the others rotating); a < b.  For 0 <= pp < np and
// 0 <= round < np - 1 the rotated index is below 2 (np - 1), so one
// conditional subtraction takes it mod np - 1 (an integer division by the
// run-time np costs tens of instructions on the round's critical path).
__device__ __forceinline__ void tournament_pair(int pp, int round, int np, int* a, int* b) {
    const int pa = pp, pb = np - 1 - pp, m = np - 1;
    int x = pa - 1 + round, y = pb - 1 + round;
    x = pa == 0 ? 0 : (x >= m ? x - m : x) + 1;
    y = pb == 0 ? 0 : (y >= m ? y - m : y) + 1;
    if (x > y) { const int t = x; x = y; y = t; }
    *a = x;
    *b = y;
}

// One-sided (Hestenes) Jacobi on the n columns of the m x n column-major A,
// accumulating the rotations into W (n x n column-major, caller-initialised):
// A W converges to U S with orthogonal columns, W to the right singular
// vectors.  Column norms are tracked through the rotations
// (alpha' = alpha - t gamma, beta' = beta + t gamma) and refreshed every sweep,
// so each pair needs one reduction.  A rotation is applied when
// |gamma| > 1e-15 sqrt(alpha beta) and gamma is above an absolute floor set by
// the matrix norm.  Convergence is quadratic, so the sweeps end after one
// whose largest rotation tangent is below 1e-8 (the next would move the
// columns by ~1e-16); at most 40 sweeps.  Returns the number of sweeps.
__device__ __forceinline__ int block_jacobi_1s(double* A, int lda, int m, int n, double* W, int ldw, double* nrm, int* flag,
                                                double* red) {
    if (n < 2) {
        __syncthreads();
        return 0;
    }
    const int nt = blockDim.x;
    const int np = (n + 1) & ~1, npairs = np / 2;
    int gs = 1;
    while (gs < 16 && gs * 8 < m) gs *= 2;      // ~8 rows per thread
    while (gs > 1 && gs * npairs > nt) gs >>= 1;
    const int pair = threadIdx.x / gs, gl = threadIdx.x % gs;
    const int ngroups = nt / gs;
    for (int sweep = 0; sweep < 40; ++sweep) {
        double part = 0.0;
        for (int j = threadIdx.x; j < n; j += nt) {
            double acc = 0.0;
            for (int i = 0; i < m; ++i) acc += A[i + (size_t)j * lda] * A[i + (size_t)j * lda];
            nrm[j] = acc;
            part += acc;
        }
        const double tot = block_sum(part, red);   // contains barriers
        const double floor_abs = 1e-30 * tot;
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            for (int pp0 = 0; pp0 < npairs; pp0 += ngroups) {
                const int pp = pp0 + pair;
                int a = 0, b = 0;
                bool real = false;
                if (pp < npairs) {
                    tournament_pair(pp, round, np, &a, &b);
                    real = b < n;
                }
                double ga = 0.0;
                if (real)
                    for (int i = gl; i < m; i += gs) ga += A[i + (size_t)a * lda] * A[i + (size_t)b * lda];
                ga = group_sum(ga, gs);
                if (real) {
                    const double al = nrm[a], be = nrm[b];
                    if (fabs(ga) > 1e-15 * sqrt(al * be) && fabs(ga) > floor_abs) {
                        double c, s, t;
                        jacobi_rotation(al, be, ga, &c, &s, &t);
                        for (int i = gl; i < m; i += gs) {
                            const double x = A[i + (size_t)a * lda], y = A[i + (size_t)b * lda];
                            A[i + (size_t)a * lda] = c * x - s * y;
                            A[i + (size_t)b * lda] = s * x + c * y;
                        }
                        for (int i = gl; i < n; i += gs) {
                            const double x = W[i + (size_t)a * ldw], y = W[i + (size_t)b * ldw];
                            W[i + (size_t)a * ldw] = c * x - s * y;
                            W[i + (size_t)b * ldw] = s * x + c * y;
                        }
                        if (gl == 0) {
                            nrm[a] = al - t * ga;
                            nrm[b] = be + t * ga;
                            if (fabs(t) > 1e-8) *flag = 1;
                        }
                    }
                }
            }
            __syncthreads();
        }
        const int f = *flag;
        __syncthreads();
        if (!f) return sweep + 1;
    }
    return 40;
}

// One-sided Jacobi with a compile-time layout: m = RPT * GS rows (rows beyond
// the data must be zero), n <= nt / GS * 2 columns, W n x n (rows beyond n
// unused).  Each pair of columns is owned by GS consecutive lanes holding RPT
// rows each, so a round issues all its LDS loads at once, forms
// alpha = |a|^2, beta = |b|^2, gamma = a.b by DPP group sums, and updates the
// two columns of A and of W from registers.  Same rotation rule and stopping
// rule as block_jacobi_1s.
template <int RPT, int GS, int WPT>
__device__ __forceinline__ int block_jacobi_1s_fixed(double* A, int lda, int n, double* W, int ldw, int* flag, double* red) {
    if (n < 2) {
        __syncthreads();
        return 0;
    }
    const int np = (n + 1) & ~1, npairs = np / 2;
    const int pair = threadIdx.x / GS, gl = threadIdx.x % GS;
    const bool active = pair < npairs;
    // absolute floor: pairs whose inner product is below 1e-30 ||A||_F^2 are noise
    double part = 0.0;
    for (int idx = threadIdx.x; idx < RPT * GS * n; idx += blockDim.x) {
        const double v = A[(idx % (RPT * GS)) + (size_t)(idx / (RPT * GS)) * lda];
        part += v * v;
    }
    const double floor_abs = 1e-30 * block_sum(part, red);
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            if (active) {
                int a, b;
                tournament_pair(pair, round, np, &a, &b);
                if (b < n) {
                    double x[RPT], y[RPT], u[WPT], v[WPT];
                    double* pa = A + (size_t)a * lda + gl;
                    double* pb = A + (size_t)b * lda + gl;
#pragma unroll
                    for (int k = 0; k < RPT; ++k) { x[k] = pa[k * GS]; y[k] = pb[k * GS]; }
                    double* wa = W + (size_t)a * ldw + gl;
                    double* wb = W + (size_t)b * ldw + gl;
#pragma unroll
                    for (int k = 0; k < WPT; ++k) {
                        const bool in = gl + k * GS < n;
                        u[k] = in ? wa[k * GS] : 0.0;
                        v[k] = in ? wb[k * GS] : 0.0;
                    }
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        al = fma(x[k], x[k], al);
                        be = fma(y[k], y[k], be);
                        ga = fma(x[k], y[k], ga);
                    }
                    al = group_sum(al, GS);
                    be = group_sum(be, GS);
                    ga = group_sum(ga, GS);
                    // |ga| > 1e-15 sqrt(al be), squared (no FP64 square root on
                    // the round's critical path)
                    if (ga * ga > 1e-30 * (al * be) && fabs(ga) > floor_abs) {
                        double c, s, t;
                        jacobi_rotation(al, be, ga, &c, &s, &t);
#pragma unroll
                        for (int k = 0; k < RPT; ++k) {
                            pa[k * GS] = c * x[k] - s * y[k];
                            pb[k * GS] = s * x[k] + c * y[k];
                        }
#pragma unroll
                        for (int k = 0; k < WPT; ++k) {
                            if (gl + k * GS < n) {
                                wa[k * GS] = c * u[k] - s * v[k];
                                wb[k * GS] = s * u[k] + c * v[k];
                            }
                        }
                        if (gl == 0 && fabs(t) > 1e-8) *flag = 1;
                    }
                }
            }
            __syncthreads();
        }
        const int f = *flag;
        __syncthreads();
        if (!f) return sweep + 1;
    }
    return 40;
}

// Two-sided cyclic Jacobi on the symmetric n x n column-major S, accumulating
// the rotations into W: W^T S W converges to diag(eigenvalues); sweeps end as
// in block_jacobi_1s.  S is a Gram
// matrix known to ~u tr(S) absolute, so off-diagonals below 1e-15 tr(S) are
// noise and are not rotated (rotations inside the negligible block would
// neither converge nor change its trace, i.e. the truncated tail norm).
// Two-sided Jacobi on a symmetric matrix (the Gram path).  Sweeps stop after
// one whose largest rotation tangent is at most tconv: the method converges
// quadratically, so the next sweep would rotate by about tconv^2.
__device__ __forceinline__ int block_jacobi_sym(double* S, int n, int ld, double* W, double* cs, int* pa_, int* pb_, int* flag,
                                                double tconv) {
    if (n < 2) {
        __syncthreads();
        return 0;
    }
    const int nt = blockDim.x;
    const int np = (n + 1) & ~1, npairs = np / 2;
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += fabs(S[i + (size_t)i * ld]);
    const double floor_abs = 1e-15 * tr;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            for (int pp = threadIdx.x; pp < npairs; pp += nt) {
                int a, b;
                tournament_pair(pp, round, np, &a, &b);
                double c = 1.0, s = 0.0;
                if (b < n) {
                    const double app = S[a + (size_t)a * ld], aqq = S[b + (size_t)b * ld], apq = S[a + (size_t)b * ld];
                    if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
                        double t;
                        jacobi_rotation(app, aqq, apq, &c, &s, &t);
                        if (fabs(t) > tconv) *flag = 1;
                    }
                }
                cs[2 * pp] = c;
                cs[2 * pp + 1] = s;
                pa_[pp] = a;
                pb_[pp] = b;
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < npairs * n; idx += nt) {   // columns: S <- S R, W <- W R
                const int pp = idx / n, i = idx % n;
                const int a = pa_[pp], b = pb_[pp];
                const double c = cs[2 * pp], s = cs[2 * pp + 1];
                if (b >= n || s == 0.0) continue;
                const double x = S[i + (size_t)a * ld], y = S[i + (size_t)b * ld];
                S[i + (size_t)a * ld] = c * x - s * y;
                S[i + (size_t)b * ld] = s * x + c * y;
                const double u = W[i + (size_t)a * ld], w = W[i + (size_t)b * ld];
                W[i + (size_t)a * ld] = c * u - s * w;
                W[i + (size_t)b * ld] = s * u + c * w;
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < npairs * n; idx += nt) {   // rows: S <- R^T S
                const int pp = idx / n, i = idx % n;
                const int a = pa_[pp], b = pb_[pp];
                const double c = cs[2 * pp], s = cs[2 * pp + 1];
                if (b >= n || s == 0.0) continue;
                const double x = S[a + (size_t)i * ld], y = S[b + (size_t)i * ld];
                S[a + (size_t)i * ld] = c * x - s * y;
                S[b + (size_t)i * ld] = s * x + c * y;
            }
            __syncthreads();
        }
        const int f = *flag;
        __syncthreads();
        if (!f) return sweep + 1;
    }
    return 40;
}

// Two-sided Jacobi on a 64 x 64 symmetric S (zero-padded beyond n) with 1024
// threads and one update phase per round: thread (p, q) maps the 2 x 2 block
// of S on the rows of pair p and the columns of pair q to R_p^T B R_q, and
// W <- W R is updated per (row, pair).  Same rotation and stopping rules as
// block_jacobi_sym.
__device__ __forceinline__ int block_jacobi_sym64(double* S, int ld, double* W, double* cs, int* pa_, int* pb_,
                                                  int* flag, double tconv) {
    const int np = 64, npairs = 32;
    double tr = 0.0;
    for (int i = 0; i < 64; ++i) tr += fabs(S[i + (size_t)i * ld]);
    const double floor_abs = 1e-15 * tr;
    const int p = threadIdx.x >> 5, q = threadIdx.x & 31;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            if (threadIdx.x < npairs) {
                int a, b;
                tournament_pair(threadIdx.x, round, np, &a, &b);
                double c = 1.0, sn = 0.0;
                const double app = S[a + (size_t)a * ld], aqq = S[b + (size_t)b * ld], apq = S[a + (size_t)b * ld];
                // |apq| > 1e-15 sqrt(|app aqq|), squared
                if (apq * apq > 1e-30 * fabs(app * aqq) && fabs(apq) > floor_abs) {
                    double t;
                    jacobi_rotation(app, aqq, apq, &c, &sn, &t);
                    if (fabs(t) > tconv) *flag = 1;
                    // a rotation by less than 1e-10 changes nothing the rounding can see
                    if (fabs(t) <= 1e-10) {
                        c = 1.0;
                        sn = 0.0;
                    }
                }
                cs[2 * threadIdx.x] = c;
                cs[2 * threadIdx.x + 1] = sn;
                pa_[threadIdx.x] = a;
                pb_[threadIdx.x] = b;
            }
            __syncthreads();
            const double sp = cs[2 * p + 1], sq = cs[2 * q + 1];
            if (sp != 0.0 || sq != 0.0) {   // both rotations identity: block unchanged
                const int ap = pa_[p], bp = pb_[p], aq = pa_[q], bq = pb_[q];
                const double cp = cs[2 * p], cq = cs[2 * q];
                double* s00 = S + ap + (size_t)aq * ld;
                double* s01 = S + ap + (size_t)bq * ld;
                double* s10 = S + bp + (size_t)aq * ld;
                double* s11 = S + bp + (size_t)bq * ld;
                const double b00 = *s00, b01 = *s01, b10 = *s10, b11 = *s11;
                const double c00 = cq * b00 - sq * b01, c01 = sq * b00 + cq * b01;
                const double c10 = cq * b10 - sq * b11, c11 = sq * b10 + cq * b11;
                const int i0 = threadIdx.x >> 5, i1 = i0 + 32;     // W rows handled by this thread
                double* w0a = W + i0 + (size_t)aq * ld;
                double* w0b = W + i0 + (size_t)bq * ld;
                double* w1a = W + i1 + (size_t)aq * ld;
                double* w1b = W + i1 + (size_t)bq * ld;
                const double u0 = *w0a, v0 = *w0b, u1 = *w1a, v1 = *w1b;
                // every thread reads and writes only its own 2 x 2 block of S and its
                // own W entries (rows p, p + 32 of columns aq, bq): no barrier here
                *s00 = cp * c00 - sp * c10;
                *s01 = cp * c01 - sp * c11;
                *s10 = sp * c00 + cp * c10;
                *s11 = sp * c01 + cp * c11;
                *w0a = cq * u0 - sq * v0;
                *w0b = sq * u0 + cq * v0;
                *w1a = cq * u1 - sq * v1;
                *w1b = sq * u1 + cq * v1;
            }
            __syncthreads();
        }
        const int f = *flag;
        __syncthreads();
        if (!f) return sweep + 1;
    }
    return 40;
}

// Two-sided Jacobi for n <= 128 with S (n x n, column-major, leading dimension
// ld) in LDS and W in global memory (leading dimension ldw): each round
// updates every 2 x 2 block (rows a_p, b_p; columns a_q, b_q) of S in one
// phase, R_p^T B R_q, and the rows of W per column pair (W <- W R); rounds
// leave the blocks of two identity rotations untouched.  Same rotation,
// skipping and stopping rules as block_jacobi_sym64, except that rotations
// with |t| <= tskip (default 1e-10) are skipped.  __syncthreads orders
// the global W accesses of consecutive rounds within the workgroup.
__device__ __forceinline__ int block_jacobi_sym_wide(double* S, int n, int ld, double* W, int ldw, double* cs, int* pa_,
                                                     int* pb_, int* flag, double tconv, double tskip = 1e-10) {
    if (n < 2) {
        __syncthreads();
        return 0;
    }
    const int nt = blockDim.x;
    const int np = (n + 1) & ~1, npairs = np / 2;
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += fabs(S[i + (size_t)i * ld]);
    const double floor_abs = 1e-15 * tr;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            for (int pp = threadIdx.x; pp < npairs; pp += nt) {
                int a, b;
                tournament_pair(pp, round, np, &a, &b);
                double c = 1.0, sn = 0.0;
                if (b < n) {
                    const double app = S[a + (size_t)a * ld], aqq = S[b + (size_t)b * ld], apq = S[a + (size_t)b * ld];
                    if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
                        double t;
                        jacobi_rotation(app, aqq, apq, &c, &sn, &t);
                        if (fabs(t) > tconv) *flag = 1;
                        if (fabs(t) <= tskip) {
                            c = 1.0;
                            sn = 0.0;
                        }
                    }
                }
                cs[2 * pp] = c;
                cs[2 * pp + 1] = sn;
                pa_[pp] = a;
                pb_[pp] = b;
            }
            __syncthreads();
            // S <- R^T S R by 2 x 2 blocks (dummy pairs, b >= n, carry identity rotations)
            for (int idx = threadIdx.x; idx < npairs * npairs; idx += nt) {
                const int p = idx / npairs, q = idx % npairs;
                const double sp = cs[2 * p + 1], sq = cs[2 * q + 1];
                if (sp == 0.0 && sq == 0.0) continue;
                const int ap = pa_[p], bp = pb_[p], aq = pa_[q], bq = pb_[q];
                const double cp = cs[2 * p], cq = cs[2 * q];
                // a dummy pair (odd n) has b = n: its row / column does not exist
                const bool vp = bp < n, vq = bq < n;
                const double b00 = S[ap + (size_t)aq * ld];
                const double b01 = vq ? S[ap + (size_t)bq * ld] : 0.0;
                const double b10 = vp ? S[bp + (size_t)aq * ld] : 0.0;
                const double b11 = (vp && vq) ? S[bp + (size_t)bq * ld] : 0.0;
                const double c00 = cq * b00 - sq * b01, c01 = sq * b00 + cq * b01;
                const double c10 = cq * b10 - sq * b11, c11 = sq * b10 + cq * b11;
                S[ap + (size_t)aq * ld] = cp * c00 - sp * c10;
                if (vq) S[ap + (size_t)bq * ld] = cp * c01 - sp * c11;
                if (vp) S[bp + (size_t)aq * ld] = sp * c00 + cp * c10;
                if (vp && vq) S[bp + (size_t)bq * ld] = sp * c01 + cp * c11;
            }
            // W <- W R: row i of columns a_q, b_q
            for (int idx = threadIdx.x; idx < npairs * n; idx += nt) {
                const int q = idx / n, i = idx % n;
                const double sq = cs[2 * q + 1];
                if (sq == 0.0) continue;
                const double cq = cs[2 * q];
                double* wa = W + i + (size_t)pa_[q] * ldw;
                double* wb = W + i + (size_t)pb_[q] * ldw;
                const double u = *wa, v = *wb;
                *wa = cq * u - sq * v;
                *wb = sq * u + cq * v;
            }
            __syncthreads();
        }
        const int f = *flag;
        __syncthreads();
        if (!f) return sweep + 1;
    }
    return 40;
}

// C = A B for 64 x 64 operands in LDS, elements addressed as A(i, k) =
// A[i * ai + k * ak], B(k, j) = B[k * bk + j * bj], C(i, j) = C[i + j * ldc];
// threads 0..255 each form a 4 x 4 tile (8 LDS reads per 16 FMAs).  The caller
// synchronises before and after.
__device__ __forceinline__ void block_mm64(const double* A, int ai, int ak, const double* B, int bk, int bj, double* C,
                                           int ldc) {
    if (threadIdx.x >= 256) return;
    const int i0 = 4 * (threadIdx.x & 15), j0 = 4 * (threadIdx.x >> 4);
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
#pragma unroll 4
    for (int k = 0; k < 64; ++k) {
        double a[4], bv[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) a[x] = A[(i0 + x) * ai + k * ak];
#pragma unroll
        for (int y = 0; y < 4; ++y) bv[y] = B[k * bk + (j0 + y) * bj];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * bv[y];
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) C[(i0 + x) + (size_t)(j0 + y) * ldc] = acc[x][y];
}

// C = A B with A (m x K) and B (K x n) in LDS or global memory: A(i, k) =
// A[i * ai + k * ak], B(k, j) = B[k * bk + j * bj], C(i, j) = C[i * ci + j * cj].
// Each thread forms 4 x 4 tiles of C (8 loads per 16 FMAs); indices beyond m
// and n are clamped on load and not stored.  The caller synchronises before
// and after.
__device__ __forceinline__ void block_mm_tiled(int m, int n, int K, const double* A, int ai, int ak, const double* B,
                                               int bk, int bj, double* C, int ci, int cj) {
    const int mt = (m + 3) >> 2, nt = (n + 3) >> 2;
    for (int t = threadIdx.x; t < mt * nt; t += blockDim.x) {
        const int i0 = 4 * (t % mt), j0 = 4 * (t / mt);
        int ia[4], jb[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            ia[x] = (i0 + x < m ? i0 + x : m - 1) * ai;
            jb[x] = (j0 + x < n ? j0 + x : n - 1) * bj;
        }
        double acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
#pragma unroll 4
        for (int k = 0; k < K; ++k) {
            double a[4], bv[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) a[x] = A[ia[x] + k * ak];
#pragma unroll
            for (int y = 0; y < 4; ++y) bv[y] = B[k * bk + jb[y]];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * bv[y];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
                if (i0 + x < m && j0 + y < n) C[(size_t)(i0 + x) * ci + (size_t)(j0 + y) * cj] = acc[x][y];
    }
}

// Descending order of s[0..n) into perm (ties by index).  A NaN sorts as
// -inf, so the comparison stays a total order and perm a permutation of
// 0..n-1 whatever the values (a NaN state is then reported, not indexed).
__device__ __forceinline__ void block_sort_desc(const double* s, int n, int* perm) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double v = s[j] == s[j] ? s[j] : -INFINITY;
        int rank = 0;
        for (int i = 0; i < n; ++i) {
            const double u = s[i] == s[i] ? s[i] : -INFINITY;
            if (u > v || (u == v && i < j)) ++rank;
        }
        perm[rank] = j;
    }
    __syncthreads();
}

// Smallest r >= 1 with sqrt(sum_{i>=r} s_sorted[i]^2) <= delta, capped.
__device__ __forceinline__ int delta_rank(const double* s, const int* perm, int n, double delta, int cap) {
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

// Exact x / d and x % d for 0 <= x < 2^22 (the runtime divisors of the
// small-core kernels are uniform and small; a plain integer division costs
// tens of VALU instructions).  x times the FP32 reciprocal of d is within
// (x / d) 2^-22 < 1 of x / d, so its truncation is off by at most one, which
// the remainder test corrects.
struct FastDiv {
    float rcp;
    int d;
    __device__ explicit FastDiv(int dd) : rcp(__builtin_amdgcn_rcpf((float)dd)), d(dd) {}
    __device__ int q(int x) const {
        const int q0 = (int)((float)x * rcp);
        const int r = x - __mul24(q0, d);
        return q0 + (r >= d ? 1 : 0) - (r < 0 ? 1 : 0);
    }
    __device__ int r(int x) const { return x - __mul24(q(x), d); }
};

}  // namespace ttrt

#include "k_eig.hpp"

namespace ttrt {

// ---------------------------------------------------------------------------
// prep: right-to-left orthogonalisation of the small cores of the TT sum
// ---------------------------------------------------------------------------
//
// The pending TT sum has Phi_new (R2 x N_phi, stacked), Theta_new (R1 x N_theta
// x R2, block diagonal) and the virtual first core Z_new.  This kernel
//  1. factors Phi_new = L_Phi Q_Phi with orthonormal rows Q_Phi: by Householder
//     QR of Phi_new^T when R2 < N_phi; when R2 >= N_phi any orthogonal Q_Phi
//     works and Q_Phi = I, L_Phi = Phi_new (no arithmetic);
//  2. forms Theta' = Theta_new x_3 L_Phi and factors its row unfolding
//     Theta'_(1) = L_Theta Q_Theta the same way (QR of its transpose when
//     R1 < N_theta k2, else Q_Theta = I and L_Theta = Theta'_(1));
//  3. folds L_Theta with the streaming coefficients into the operand G of the
//     gather contraction B = d .* (sum_j (O_j Z) G_j + rank-1 terms), so that
//     B = Z_new L_Theta (the projected first core; X_(1) = B Q_Theta (I x Q_Phi)).
// The state gets R1, R2, k1, k2, ldb, and whether both Q's are identities
// (the projected basis is then the canonical angular basis, so the previous
// round's singular vectors are a valid warm start).
// (the body of k_prep, also called by the persistent small-solve kernel;
// lds is the block's dynamic LDS of lds_doubles doubles)
template <typename TC>
__device__ __forceinline__ void prep_body(const Geom& g, const OpDesc& op, DevState* st, const double* __restrict__ Th,
                                          const double* __restrict__ Ph, const double* __restrict__ gtab,
                                          const double* __restrict__ htab, const SmallScratch& sc,
                                          double* __restrict__ LTh, int ldl, double* __restrict__ QTh,
                                          double* __restrict__ QPh, TC* __restrict__ Gop, TC* __restrict__ Gsw,
                                          int nct, double* lds, size_t lds_doubles,
                                          double* __restrict__ Wst = nullptr, double* __restrict__ Cst = nullptr) {
    __shared__ double red[16];
    LdsCarver cv{lds, 0, lds_doubles};
    const int nt = g.nt, npn = g.np;
    const int r1 = st->r1, r2 = st->r2, ldz = st->ldz;
    const int nrb = op.n_rblk, nr1 = op.n_r1;
    const int R1 = nrb * r1 + nr1, R2 = nrb * r2 + nr1;
    const bool phi_id = R2 >= npn;
    const int k2 = phi_id ? npn : R2;
    const int m2 = nt * k2;
    const bool th_id = R1 >= m2;
    const int k1 = th_id ? m2 : R1;
    const int ldb = ld_for_rank(k1);
    const FastDiv dnp(npn), dr1(r1), dr2(r2), dk2(k2), dm2(m2), dk1(k1), dldz(ldz), dldb(ldb);

    // the operator's block tables in LDS: they are indexed per lane below, and
    // a per-lane index into the kernel arguments is a vector memory load
    __shared__ int s_rfac[kMaxBlocks], s_rshift[kMaxBlocks], s_rshift2[kMaxBlocks], s_r1fac[kMaxBlocks];
    __shared__ double s_rcoef0[kMaxBlocks], s_rcoef[kMaxBlocks], s_rcoef2[kMaxBlocks];
    __shared__ int s_gterm[kMaxBlocks];
    if (threadIdx.x == 0) {
        for (int i = 0; i < kMaxBlocks; ++i) {
            s_rfac[i] = op.rfac[i];
            s_rshift[i] = op.rshift[i];
            s_r1fac[i] = op.r1fac[i];
            s_rcoef0[i] = op.rcoef0[i];
            s_rcoef[i] = op.rcoef[i];
            s_rshift2[i] = op.rshift2[i];
            s_rcoef2[i] = op.rcoef2[i];
            s_gterm[i] = op.gterm[i];
        }
    }
    // the angular core and the per-node factor tables in LDS where they fit
    // (every entry below is read many times)
    const double* thv = Th;
    const double* gtv = gtab;
    const double* htv = htab;
    {
        const int nth = r1 * nt * r2, ngt = (1 + g.n_terms) * nt, nht = (1 + g.n_terms) * npn;
        double* a = cv.take((size_t)nth, nullptr);
        double* b = cv.take((size_t)ngt, nullptr);
        double* c = cv.take((size_t)nht, nullptr);
        for (int i = threadIdx.x; a && i < nth; i += blockDim.x) a[i] = Th[i];
        for (int i = threadIdx.x; b && i < ngt; i += blockDim.x) b[i] = gtab[i];
        for (int i = threadIdx.x; c && i < nht; i += blockDim.x) c[i] = htab[i];
        if (a) thv = a;
        if (b) gtv = b;
        if (c) htv = c;
        __syncthreads();
    }

    // 1. L_Phi (R2 x k2, row-major) and Q_Phi (k2 x N_phi)
    double* Lphi = cv.take((size_t)R2 * k2, sc.Q1 + (size_t)npn * npn);
    if (phi_id) {
        for (int idx = threadIdx.x; idx < R2 * npn; idx += blockDim.x) {
            const int col = dnp.q(idx), p = idx - col * npn;
            double v;
            if (col < nrb * r2) {
                const int t = dr2.q(col), b = col - t * r2;
                v = Ph[(size_t)b * npn + p] * htv[s_rfac[t] * npn + p];
            } else {
                v = htv[s_r1fac[col - nrb * r2] * npn + p];
            }
            Lphi[idx] = v;
        }
        for (int idx = threadIdx.x; idx < npn * npn; idx += blockDim.x) QPh[idx] = (dnp.q(idx) == dnp.r(idx)) ? 1.0 : 0.0;
    } else {
        double* A1 = cv.take((size_t)npn * R2, sc.A1);
        double* Q1 = cv.take((size_t)npn * k2, sc.Q1);
        for (int idx = threadIdx.x; idx < npn * R2; idx += blockDim.x) {
            const int col = dnp.q(idx), p = idx - col * npn;
            double v;
            if (col < nrb * r2) {
                const int t = dr2.q(col), b = col - t * r2;
                v = Ph[(size_t)b * npn + p] * htv[s_rfac[t] * npn + p];
            } else {
                v = htv[s_r1fac[col - nrb * r2] * npn + p];
            }
            A1[p + (size_t)col * npn] = v;
        }
        __syncthreads();
        block_householder_qr(A1, npn, npn, R2, sc.tau, red);
        block_form_q(A1, npn, npn, k2, sc.tau, Q1, npn);
        for (int idx = threadIdx.x; idx < k2 * npn; idx += blockDim.x) {
            const int c = dnp.q(idx), p = idx - c * npn;
            QPh[(size_t)c * npn + p] = Q1[p + (size_t)c * npn];
        }
        for (int idx = threadIdx.x; idx < R2 * k2; idx += blockDim.x) {
            const int col = dk2.q(idx), c = idx - col * k2;
            Lphi[idx] = (c <= col) ? A1[c + (size_t)col * npn] : 0.0;
        }
    }
    __syncthreads();
    // 2. Theta' (R1 x N_theta x k2): value of element (row, l, c)
    auto theta_p = [&](int row, int l, int c) -> double {
        double v = 0.0;
        if (row < nrb * r1) {
            const int t = dr1.q(row), a = row - t * r1;
            const double* th = thv + ((size_t)a * nt + l) * r2;
            const double* lp = Lphi + (size_t)(t * r2) * k2 + c;
            for (int b = 0; b < r2; ++b) v += th[b] * lp[(size_t)b * k2];
            v *= gtv[s_rfac[t] * nt + l];
        } else {
            const int q = row - nrb * r1;
            v = gtv[s_r1fac[q] * nt + l] * Lphi[(size_t)(nrb * r2 + q) * k2 + c];
        }
        return v;
    };
    // L_Theta (R1 x k1) is only read here: LDS where it fits
    double* LT = LTh;
    int ldL = ldl;
    if (th_id) {
        if (double* a = cv.take((size_t)R1 * k1, nullptr)) {
            LT = a;
            ldL = k1;
        }
        for (int idx = threadIdx.x; idx < R1 * m2; idx += blockDim.x) {
            const int row = dm2.q(idx), i = idx - row * m2;
            const int l = dk2.q(i);
            LT[(size_t)row * ldL + i] = theta_p(row, l, i - l * k2);
        }
        for (int idx = threadIdx.x; idx < m2 * m2; idx += blockDim.x) QTh[idx] = (dm2.q(idx) == dm2.r(idx)) ? 1.0 : 0.0;
    } else {
        double* A2 = cv.take((size_t)m2 * R1, sc.A2);
        double* Q2 = cv.take((size_t)m2 * k1, sc.Q2);
        for (int idx = threadIdx.x; idx < m2 * R1; idx += blockDim.x) {
            const int row = dm2.q(idx), rowA = idx - row * m2;
            const int l = dk2.q(rowA);
            A2[rowA + (size_t)row * m2] = theta_p(row, l, rowA - l * k2);
        }
        __syncthreads();
        block_householder_qr(A2, m2, m2, R1, sc.tau, red);
        block_form_q(A2, m2, m2, k1, sc.tau, Q2, m2);
        for (int idx = threadIdx.x; idx < k1 * m2; idx += blockDim.x) {
            const int i = dm2.q(idx), rowA = idx - i * m2;
            QTh[(size_t)i * m2 + rowA] = Q2[rowA + (size_t)i * m2];
        }
        if (double* a = cv.take((size_t)R1 * k1, nullptr)) {
            LT = a;
            ldL = k1;
        }
        for (int idx = threadIdx.x; idx < R1 * k1; idx += blockDim.x) {
            const int row = dk1.q(idx), i = idx - row * k1;
            LT[(size_t)row * ldL + i] = (i <= row) ? A2[i + (size_t)row * m2] : 0.0;
        }
    }
    __syncthreads();
    // 3. gather operand G: rows (gather block j, a < ldz), then rank-1 rows; ldb columns
    const int grows = op.n_gather * ldz + nr1;
    auto gval = [&](int row, int col) -> double {
        double v = 0.0;
        if (col < k1) {
            if (row < op.n_gather * ldz) {
                const int j = dldz.q(row), a = row - j * ldz;
                if (a < r1) {
                    if (op.hll) {
                        // HLL: block j is its r-block's shifted copy with a per-row weight
                        v = LT[(size_t)(s_gterm[j] * r1 + a) * ldL + col];
                    } else {
                        for (int t = 0; t < nrb; ++t) {
                            const double l = LT[(size_t)(t * r1 + a) * ldL + col];
                            if (j == 0) v += s_rcoef0[t] * l;
                            if (s_rshift[t] == j) v += s_rcoef[t] * l;
                            if (s_rshift2[t] == j) v += s_rcoef2[t] * l;
                        }
                    }
                }
            } else {
                const int q = row - op.n_gather * ldz;
                v = LT[(size_t)(nrb * r1 + q) * ldL + col];
            }
        }
        return v;
    };
    for (int idx = threadIdx.x; idx < grows * ldb; idx += blockDim.x) {
        const int row = dldb.q(idx), col = idx - row * ldb;
        Gop[(size_t)row * ldb + col] = (TC)gval(row, col);
    }
    if (Gsw) {
        // the same operand in the lane order of the fused MFMA contraction:
        // slot ((t * nct + c) * 64 + lane) * 4 + e holds G[16 t + 4 (lane / 16) + e][16 c + lane % 16]
        const int ng = (grows + 15) / 16;
        const FastDiv dnct(nct);
        for (int idx = threadIdx.x; idx < ng * nct * 256; idx += blockDim.x) {
            const int e = idx & 3, ln = (idx >> 2) & 63, tc = idx >> 8;
            const int t = dnct.q(tc), c = tc - t * nct;
            const int row = 16 * t + 4 * (ln >> 4) + e, col = 16 * c + (ln & 15);
            Gsw[idx] = (row < grows && col < ldb) ? (TC)gval(row, col) : (TC)0;
        }
    }
    // 4. direction-space form of the projection (both factors square, so the
    //    columns of L_Theta are the directions (theta, phi)): block t of the
    //    sum's angular core is W = Theta x_3 Phi scaled by g_t(theta) h_t(phi).
    //    W (ldz x ldb, zero past r1 and k1), then per gather block j the
    //    direction factor C_j = sum_t coef(t, j) g_t h_t, then the rank-1
    //    blocks' direction rows R_q = g h (rows n_gather + q).
    const bool stencil = Wst && Cst && th_id && phi_id && !op.hll;
    if (stencil) {
        for (int idx = threadIdx.x; idx < ldz * ldb; idx += blockDim.x) {
            const int a = dldb.q(idx), i = idx - a * ldb;
            double v = 0.0;
            if (a < r1 && i < k1) {
                const int l = dnp.q(i), p = i - l * npn;
                const double* th = thv + ((size_t)a * nt + l) * r2;
                for (int b = 0; b < r2; ++b) v += th[b] * Ph[(size_t)b * npn + p];
            }
            Wst[idx] = v;
        }
        for (int idx = threadIdx.x; idx < (op.n_gather + nr1) * ldb; idx += blockDim.x) {
            const int j = dldb.q(idx), i = idx - j * ldb;
            double v = 0.0;
            if (i < k1) {
                const int l = dnp.q(i), p = i - l * npn;
                if (j < op.n_gather) {
                    for (int t = 0; t < nrb; ++t) {
                        const double gh = gtv[s_rfac[t] * nt + l] * htv[s_rfac[t] * npn + p];
                        if (j == 0) v += s_rcoef0[t] * gh;
                        if (s_rshift[t] == j) v += s_rcoef[t] * gh;
                        if (s_rshift2[t] == j) v += s_rcoef2[t] * gh;
                    }
                } else {
                    const int q = j - op.n_gather;
                    v = gtv[s_r1fac[q] * nt + l] * htv[s_r1fac[q] * npn + p];
                }
            }
            Cst[idx] = v;
        }
    }
    if (threadIdx.x == 0) {
        st->stencil = stencil ? op.n_gather + nr1 : 0;
        st->kall = grows;
        st->R1 = R1; st->R2 = R2; st->k1 = k1; st->k2 = k2; st->ldb = ldb; st->k1b = k1;
        if (R1 > st->max_R1) st->max_R1 = R1;
        if (R2 > st->max_R2) st->max_R2 = R2;
        st->canon_prev = st->canon;
        st->canon = (phi_id && th_id) ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// SVD chain: truncated SVDs of both bonds from the R factor (or Gram matrix)
// of B = Z_new L_Theta
// ---------------------------------------------------------------------------
//
// QR input: R_B (k1 x k1, upper triangular, row-major, leading dim ldr) with
// B = Q_B R_B; one-sided Jacobi on the columns of R_B W gives W = right
// singular vectors of R_B (= those of B) and the column norms give S.
// Gram input (gram != 0): G = B^T B; two-sided Jacobi W^T G W -> diag(S^2).
// When this round and the previous one both project onto the canonical
// angular basis, W starts from the previous round's singular vectors.
// The rest is the left-to-right sweep of TT-SVD rounding with the norm kept
// in Z:  Z_out = B V_r;  Theta'' = V_r^T Q_Theta;  SVD of diag(S_r) Theta''
// ((r1 N_theta) x k2) -> V2, S2;  Theta_out = Theta'' x_3 V2_r;
// Phi_out = V2_r^T Q_Phi.  Truncation: delta = tol ||X||_F / sqrt(2) per bond.
// (the body of k_svd_chain, also called by the persistent small-solve
// kernel; lds is the block's dynamic LDS of lds_doubles doubles, at least the
// fixed layout's when FAST)
template <typename TC, bool FAST>
__device__ __forceinline__ void svd_chain_body(const Geom& g, DevState* st, const double* __restrict__ RB, int ldr,
                                               int gram, const double* __restrict__ QTh,
                                               const double* __restrict__ QPh, double tol, int cap1, int cap2,
                                               const SmallScratch& sc, double* __restrict__ ThOut,
                                               double* __restrict__ PhOut, TC* __restrict__ Vout,
                                               double* __restrict__ sv_out, const TC* __restrict__ Gop,
                                               TC* __restrict__ Gfold, int nct_o, double* lds, size_t lds_doubles) {
    // Gop, Gfold, nct_o: non-null Gfold marks a fused pass (its operand G V_r is
    // formed afterwards by k_fold); they only change the flop accounting here
    (void)Gop;
    (void)nct_o;
    __shared__ double red[16];
    __shared__ int sh_r[2];
    __shared__ int sh_flag;
    __shared__ double cs[2 * 128];
    __shared__ int pa_[128], pb_[128];
    LdsCarver cv{lds, 0, lds_doubles};
    const int nt = g.nt, npn = g.np;
    const int k1 = st->k1, k2 = st->k2;
    const int m2 = nt * k2;
    // FAST (k1 <= 64, r1 N_theta <= 256, k2 <= 16): working matrices at fixed
    // LDS offsets, 64 x 64 with leading dimension 65 (columns on different
    // banks), zero / identity padded beyond k1.  Otherwise LDS where it fits
    // and global scratch beyond.
    const int kp = FAST ? 64 : k1;                       // padded order
    const int ld = FAST ? 65 : (k1 | 1);   // odd leading dimension: columns on different LDS banks
    const size_t reg0 = FAST ? (size_t)(64 * 65 > 257 * 16 ? 64 * 65 : 257 * 16) : 0;
    double* J = FAST ? lds : cv.take((size_t)k1 * ld, sc.J);
    // The Gram route's first bond by tridiagonalisation (k_eig.hpp) when its
    // scratch fits in LDS beside J; the Jacobi eigensolver otherwise, and as
    // the fallback when its eigenvectors fail their checks.
    double* trd_mem = nullptr;
    // (at k1 <= 64 the warm-started Jacobi on LDS is as fast: the fixed layout)
    if (gram && k1 >= 2 && !FAST && J != sc.J) trd_mem = cv.take(kTrdScratch, nullptr);
    double* W = FAST ? lds + reg0 : cv.take((size_t)k1 * ld, sc.W);
    double* T = FAST ? W + (size_t)kp * ld : cv.take((size_t)k1 * ld, sc.A2);
    double* nrm = FAST ? T + (size_t)kp * ld : cv.take((size_t)k1, sc.sv + 2 * k1);
    double* s1 = FAST ? nrm + kp : cv.take((size_t)k1, sc.sv);
    int* p1 = sc.perm;
    bool trd = trd_mem != nullptr;
    const bool warm = !trd && st->canon && st->canon_prev && st->k1_prev == k1;
    long long tph[8];
    int sw1 = 0, sw2 = 0;
    const FastDiv dkp(kp), dk1(k1), dk2(k2), dm2(m2), dnt(nt), dnp(npn);
    tph[0] = wall_clock64();
    // stage the input (R_B or G, row-major in global) column-major into T; W0
    auto stage = [&](bool wrm) {
        for (int idx = threadIdx.x; idx < kp * kp; idx += blockDim.x) {
            const int i = dkp.q(idx), j = idx - i * kp;      // coalesced along rows of the input
            T[i + (size_t)j * ld] = (i < k1 && j < k1) ? RB[(size_t)i * ldr + j] : 0.0;
            W[j + (size_t)i * ld] = (i < k1 && j < k1) ? (wrm ? sc.Wkeep[j + (size_t)i * k1] : (i == j ? 1.0 : 0.0))
                                                       : (i == j ? 1.0 : 0.0);
        }
        __syncthreads();
    };
    // Gram route by Jacobi: J = W^T G W (warm) or G, two-sided Jacobi, s1 = sqrt(diag)
    auto jacobi_gram = [&](bool wrm) {
        if (wrm && FAST) {
            // J = W^T G W on 64 x 64 tiles in LDS (zero / identity padded beyond k1)
            block_mm64(T, 1, ld, W, 1, ld, J, ld);       // J = G W
            __syncthreads();
            block_mm64(W, ld, 1, J, 1, ld, T, ld);       // T = W^T J
            __syncthreads();
        } else if (wrm) {
            // J = W^T G W: J <- G W, then T <- W^T J
            block_mm_tiled(k1, k1, k1, T, 1, ld, W, 1, ld, J, 1, ld);
            __syncthreads();
            block_mm_tiled(k1, k1, k1, W, ld, 1, J, 1, ld, T, 1, ld);
            __syncthreads();
        }
        for (int idx = threadIdx.x; idx < kp * kp; idx += blockDim.x) {
            const int j = dkp.q(idx), i = idx - j * kp;
            J[i + (size_t)j * ld] = T[i + (size_t)j * ld];
        }
        __syncthreads();
        tph[1] = wall_clock64();
        if (FAST)
            sw1 = block_jacobi_sym64(J, ld, W, cs, pa_, pb_, &sh_flag, kGramSweepTol);
        else
            sw1 = block_jacobi_sym_wide(J, k1, ld, W, ld, cs, pa_, pb_, &sh_flag, kGramSweepTol);
        tph[2] = wall_clock64();
        for (int j = threadIdx.x; j < k1; j += blockDim.x) s1[j] = sqrt(fmax(J[j + (size_t)j * ld], 0.0));
    };
    stage(warm);
    TrdScratch ws;
    if (trd) ws.carve(trd_mem);
    const int K = k1 < cap1 ? k1 : cap1;   // eigenvalues the truncation can keep
    if (!gram) {
        // J = R_B W (R_B upper triangular)
        for (int idx = threadIdx.x; idx < kp * kp; idx += blockDim.x) {
            const int j = dkp.q(idx), i = idx - j * kp;
            double acc = 0.0;
            if (warm) {
                for (int k = i; k < k1; ++k) acc += T[i + (size_t)k * ld] * W[k + (size_t)j * ld];
            } else {
                acc = T[i + (size_t)j * ld];
            }
            J[i + (size_t)j * ld] = acc;
        }
        __syncthreads();
        tph[1] = wall_clock64();
        // J = R_B W has non-zero rows only below k1 (R_B is k1 x k1 upper
        // triangular): for k1 <= 16 (32) the rotations run over 16 (32) rows
        if (FAST && k1 <= 16)
            sw1 = block_jacobi_1s_fixed<1, 16, 1>(J, ld, k1, W, ld, &sh_flag, red);
        else if (FAST && k1 <= 32)
            sw1 = block_jacobi_1s_fixed<2, 16, 2>(J, ld, k1, W, ld, &sh_flag, red);
        else if (FAST)
            sw1 = block_jacobi_1s_fixed<4, 16, 4>(J, ld, k1, W, ld, &sh_flag, red);
        else
            sw1 = block_jacobi_1s(J, ld, k1, k1, W, ld, nrm, &sh_flag, red);
        tph[2] = wall_clock64();
        for (int j = threadIdx.x; j < k1; j += blockDim.x) {
            double acc = 0.0;
            for (int i = 0; i < kp; ++i) acc += J[i + (size_t)j * ld] * J[i + (size_t)j * ld];
            s1[j] = sqrt(acc);
        }
    } else if (trd) {
        // J = G; T = Q^T G Q; the K largest eigenvalues, the rest of the trace
        // in entry K (so the tail sums of the truncation are trace-based); p1 = I
        for (int idx = threadIdx.x; idx < kp * kp; idx += blockDim.x) {
            const int j = dkp.q(idx), i = idx - j * kp;
            J[i + (size_t)j * ld] = T[i + (size_t)j * ld];
        }
        __syncthreads();
        tph[1] = wall_clock64();
        block_tridiag(J, k1, ld, ws, red);
        const double tr = block_trd_eigvals(k1, K, ws);
        const double gsc = ws.zr[4];   // the scale of the tridiagonalised matrix
        double part = 0.0;
        for (int j = threadIdx.x; j < K; j += blockDim.x) part += ws.lam[j];
        const double top = block_sum(part, red);
        for (int j = threadIdx.x; j < k1; j += blockDim.x) {
            s1[j] = j < K ? sqrt(fmax(ws.lam[j] * gsc, 0.0)) : (j == K ? sqrt(fmax((tr - top) * gsc, 0.0)) : 0.0);
            p1[j] = j;
        }
        tph[2] = wall_clock64();
    } else {
        jacobi_gram(warm);
    }
    __syncthreads();
    double norm2 = 0.0, norm = 0.0, delta = 0.0;
    int r1n = 1;
    auto truncate = [&](bool sort) {
        if (sort) block_sort_desc(s1, k1, p1);
        double part = 0.0;
        for (int j = threadIdx.x; j < k1; j += blockDim.x) part += s1[j] * s1[j];
        norm2 = block_sum(part, red);
        norm = sqrt(norm2);
        delta = tol * norm / sqrt(2.0);
        if (threadIdx.x == 0) sh_r[0] = delta_rank(s1, p1, k1, delta, cap1);
        __syncthreads();
        r1n = sh_r[0];
    };
    truncate(!trd);
    int trd_status = 0;        // 0 not tried, 1 done, 2 / 3 / 4 vectors refused (residual / orthogonality / > 64)
    double trd_emax = 0.0;
    if (trd) {
        // the r1n kept eigenvectors into columns 0 .. r1n - 1 of W
        const double tn = ws.zr[1];
        int fail;
        {
            // the reflectors to global memory, then the vectors of T in J's place
            for (int idx = threadIdx.x; idx < k1 * ld; idx += blockDim.x) {
                const int k = idx / ld, i = idx - k * ld;
                if (k < k1 - 2 && i >= k + 2 && i < k1) sc.J[idx] = J[idx];
            }
            __syncthreads();
            const bool cfit = (size_t)ld * r1n + (size_t)r1n * r1n <= (size_t)k1 * ld;
            double* C = cfit ? J + (size_t)ld * r1n : sc.A2;
            // more than 64 kept vectors (four per wave): the Jacobi below
            fail = r1n <= 64 ? block_trd_vectors<2, 4>(k1, r1n, ws, tn, sc.J, ld, J, ld, C, r1n, W, ld, red, trd_emax)
                             : 3;
        }
        trd_status = 1 + fail;
        if (fail) {
            // Jacobi from the cold start, then the truncation again
            trd = false;
            stage(false);
            jacobi_gram(false);
            __syncthreads();
            truncate(true);
        }
    }
    const int ldzn = ld_for_rank(r1n);
    const int ldb = st->ldb;
    // sorted V -> Wkeep (next warm start); V_r -> Vout in the contraction precision
    for (int idx = threadIdx.x; idx < k1 * k1; idx += blockDim.x) {
        const int a = dk1.q(idx), i = idx - a * k1;
        sc.Wkeep[idx] = W[i + (size_t)p1[a] * ld];
    }
    const FastDiv dldzn(ldzn);
    for (int idx = threadIdx.x; idx < ldb * ldzn; idx += blockDim.x) {
        const int i = dldzn.q(idx), a = idx - i * ldzn;
        double v = 0.0;
        if (i < k1 && a < r1n) v = W[i + (size_t)p1[a] * ld];
        Vout[(size_t)i * ldzn + a] = (TC)v;
    }
    // Theta'' = V_r^T Q_Theta (r1n x m2) and C2 = diag(S_r) Theta'' as ((r1n N_theta) x k2)
    const int mC = r1n * nt;
    const int mpad = FAST ? (mC <= 128 ? 128 : 256) : mC;   // fixed-layout row count (zero rows beyond mC)
    const int ldc = FAST ? mpad + 1 : mC;                    // padded column stride of C2
    // the first-bond matrix J is no longer needed: C2 takes its place where it fits
    double* C2 = FAST ? lds : ((size_t)ldc * k2 <= (size_t)k1 * ld ? J : cv.take((size_t)ldc * k2, sc.C2));
    if (FAST)
        for (int idx = threadIdx.x; idx < ldc * k2; idx += blockDim.x) C2[idx] = 0.0;
    double* V2 = FAST ? s1 + k1 : cv.take((size_t)k2 * k2, sc.V2);
    double* nrm2 = FAST ? V2 + (size_t)k2 * k2 : cv.take((size_t)k2, sc.sv + k1);
    // Theta'' = V_r^T Q_Theta from the sorted V (Wkeep, complete after the barrier)
    __syncthreads();
    block_mm_tiled(r1n, m2, k1, sc.Wkeep, k1, 1, QTh, m2, 1, sc.Th2, m2, 1);
    for (int idx = threadIdx.x; idx < k2 * k2; idx += blockDim.x) V2[idx] = (dk2.r(idx) == dk2.q(idx)) ? 1.0 : 0.0;
    __syncthreads();
    for (int idx = threadIdx.x; idx < r1n * m2; idx += blockDim.x) {
        const int a = dm2.q(idx), col = idx - a * m2;
        const int l = dk2.q(col), c = col - l * k2;
        C2[(a * nt + l) + (size_t)c * ldc] = s1[p1[a]] * sc.Th2[idx];
    }
    __syncthreads();
    tph[3] = wall_clock64();
    double* s2 = sc.sv + k1;
    int* p2 = sc.perm + k1;
    if (!FAST && gram) {
        // Gram route, as for the first bond: H = C2^T C2 in FP64 and its
        // eigenvectors (V2) and eigenvalues (S2^2) by two-sided Jacobi
        const int ldh = k2 | 1;
        double* H = cv.take((size_t)k2 * ldh, sc.A2);
        for (int idx = threadIdx.x; idx < k2 * k2; idx += blockDim.x) {
            const int e = dk2.q(idx), c = idx - e * k2;
            if (c > e) continue;
            const double* x = C2 + (size_t)c * ldc;
            const double* y = C2 + (size_t)e * ldc;
            double acc = 0.0;
            for (int i = 0; i < mC; ++i) acc += x[i] * y[i];
            H[c + (size_t)e * ldh] = acc;
            H[e + (size_t)c * ldh] = acc;
        }
        __syncthreads();
        if (k2 <= 16) {
            // one wave, no block barriers (V2 holds the identity)
            if (threadIdx.x < 64) sw2 = wave_jacobi_sym16(H, k2, ldh, V2, k2, cs, pa_, pb_, kGramSweepTol);
            __syncthreads();
        } else {
            sw2 = block_jacobi_sym_wide(H, k2, ldh, V2, k2, cs, pa_, pb_, &sh_flag, kGramSweepTol);
        }
        tph[4] = wall_clock64();
        for (int j = threadIdx.x; j < k2; j += blockDim.x) s2[j] = sqrt(fmax(H[j + (size_t)j * ldh], 0.0));
    } else {
        if (FAST && mpad == 128)
            sw2 = block_jacobi_1s_fixed<8, 16, 1>(C2, ldc, k2, V2, k2, &sh_flag, red);
        else if (FAST)
            sw2 = block_jacobi_1s_fixed<16, 16, 1>(C2, ldc, k2, V2, k2, &sh_flag, red);
        else
            sw2 = block_jacobi_1s(C2, ldc, mC, k2, V2, k2, nrm2, &sh_flag, red);
        tph[4] = wall_clock64();
        for (int j = threadIdx.x; j < k2; j += blockDim.x) {
            double acc = 0.0;
            for (int i = 0; i < mC; ++i) acc += C2[i + (size_t)j * ldc] * C2[i + (size_t)j * ldc];
            s2[j] = sqrt(acc);
        }
    }
    __syncthreads();
    block_sort_desc(s2, k2, p2);
    if (threadIdx.x == 0) sh_r[1] = delta_rank(s2, p2, k2, delta, cap2 < k2 ? cap2 : k2);
    __syncthreads();
    const int r2n = sh_r[1];
    const FastDiv dr2n(r2n);
    for (int idx = threadIdx.x; idx < r1n * nt * r2n; idx += blockDim.x) {
        const int al = dr2n.q(idx), q = idx - al * r2n;
        const int a = dnt.q(al), l = al - a * nt;
        const int jq = p2[q];
        double acc = 0.0;
        for (int c = 0; c < k2; ++c) acc += sc.Th2[(size_t)a * m2 + l * k2 + c] * V2[c + (size_t)jq * k2];
        ThOut[idx] = acc;
    }
    for (int idx = threadIdx.x; idx < r2n * npn; idx += blockDim.x) {
        const int q = dnp.q(idx), p = idx - q * npn;
        const int jq = p2[q];
        double acc = 0.0;
        for (int c = 0; c < k2; ++c) acc += V2[c + (size_t)jq * k2] * QPh[(size_t)c * npn + p];
        PhOut[idx] = acc;
    }
    double d1 = 0.0;
    for (int a = r1n + threadIdx.x; a < k1; a += blockDim.x) d1 += s1[p1[a]] * s1[p1[a]];
    for (int q = r2n + threadIdx.x; q < k2; q += blockDim.x) d1 += s2[p2[q]] * s2[p2[q]];
    const double disc2 = block_sum(d1, red);
    for (int j = threadIdx.x; j < k1; j += blockDim.x) sv_out[j] = s1[p1[j]];
    tph[5] = wall_clock64();
    if (threadIdx.x == 0) {
        for (int i = 0; i < 6; ++i) st->tph[i] = tph[i];
        st->tph[6] = trd_status;
        st->tph[7] = __double_as_longlong(trd_emax);
        st->sweeps[0] = sw1;
        st->sweeps[1] = sw2;
        st->r1n = r1n;
        st->r2n = r2n;
        st->ldzn = ldzn;
        st->norm = norm;
        st->disc2 = disc2;
        st->k1_prev = k1;
        if (!(norm2 < 1e300) || norm2 != norm2) st->nan_flag = 1;
        st->rounds += 1;
        if (st->stencil) st->stencil_rounds += 1;
        // B's width (a randomized pass runs the chain on its compressed core)
        const double M = (double)g.M, R1 = (double)st->R1, kk = (double)st->k1b;
        if (Gfold) {
            // fused path: projection (FP32, fl[0]) and symmetric Gram (FP64,
            // fl[1]) run in one kernel; the output contraction re-reads Z
            // with K = R1
            st->fl[0] += 2.0 * M * R1 * kk;
            st->fl[1] += M * kk * (kk + 1.0);
            st->fl[2] += 2.0 * M * R1 * (double)r1n;
        } else {
            if (st->stencil) {
                // direction-space projection: Y = Z W (K = ldz), then one
                // multiply-add per gather and rank-1 block
                st->fl_dir[0] += 2.0 * M * kk * (double)st->ldz;
                st->fl_dir[1] += 2.0 * M * kk * (double)st->stencil;
            } else {
                st->fl[0] += 2.0 * M * R1 * kk;
            }
            st->fl[1] += gram ? M * kk * (kk + 1.0) : 2.0 * M * kk * kk - 2.0 / 3.0 * kk * kk * kk;
            st->fl[2] += 2.0 * M * kk * (double)r1n;
        }
    }
}

// Operand of the fused output contraction, G' = G V_r (FP64 sums of the FP32
// gather operand with the FP64 right singular vectors kept by the SVD chain),
// in the lane order of the fused MFMA kernel: slot ((t * nct + c) * 64 + lane)
// * 4 + e holds G'[16 t + 4 (lane / 16) + e][16 c + lane % 16].
template <typename TC>
__global__ __launch_bounds__(kSmallThreads) void k_prep(Geom g, OpDesc op, DevState* st, const double* __restrict__ Th,
                                                        const double* __restrict__ Ph, const double* __restrict__ gtab,
                                                        const double* __restrict__ htab, SmallScratch sc,
                                                        double* __restrict__ LTh, int ldl, double* __restrict__ QTh,
                                                        double* __restrict__ QPh, TC* __restrict__ Gop,
                                                        TC* __restrict__ Gsw, int nct, double* __restrict__ Wst,
                                                        double* __restrict__ Cst) {
    extern __shared__ double lds[];
    prep_body<TC>(g, op, st, Th, Ph, gtab, htab, sc, LTh, ldl, QTh, QPh, Gop, Gsw, nct, lds,
                  (size_t)kSmallLdsBytes / sizeof(double), Wst, Cst);
}

template <typename TC, bool FAST>
__global__ __launch_bounds__(kSmallThreads) void k_svd_chain(Geom g, DevState* st, const double* __restrict__ RB, int ldr,
                                                             int gram, const double* __restrict__ QTh,
                                                             const double* __restrict__ QPh, double tol, int cap1,
                                                             int cap2, SmallScratch sc, double* __restrict__ ThOut,
                                                             double* __restrict__ PhOut, TC* __restrict__ Vout,
                                                             double* __restrict__ sv_out, const TC* __restrict__ Gop,
                                                             TC* __restrict__ Gfold, int nct_o) {
    extern __shared__ double lds[];
    svd_chain_body<TC, FAST>(g, st, RB, ldr, gram, QTh, QPh, tol, cap1, cap2, sc, ThOut, PhOut, Vout, sv_out, Gop,
                             Gfold, nct_o, lds, (size_t)kSmallLdsBytes / sizeof(double));
}

template <typename TC>
__global__ __launch_bounds__(256) void k_fold(const DevState* __restrict__ st, const TC* __restrict__ Gop,
                                              const double* __restrict__ Wkeep, TC* __restrict__ Gfold, int nct) {
    const int kall = st->kall, k1 = st->k1, ldb = st->ldb, r1n = st->r1n;
    const int ng = (kall + 15) / 16;
    const int total = ng * nct * 256;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int e = idx & 3, ln = (idx >> 2) & 63, tc = idx >> 8;
        const int c = tc % nct, t = tc / nct;
        const int row = 16 * t + 4 * (ln >> 4) + e, a = 16 * c + (ln & 15);
        double v = 0.0;
        if (row < kall && a < r1n) {
            const TC* gr = Gop + (size_t)row * ldb;
            const double* wc = Wkeep + (size_t)a * k1;
            for (int i = 0; i < k1; ++i) v += (double)gr[i] * wc[i];
        }
        Gfold[idx] = (TC)v;
    }
}

// Make the truncated cores current.
__global__ void k_commit(DevState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->r1_in = st->r1;
        st->r1 = st->r1n;
        st->r2 = st->r2n;
        st->ldz = st->ldzn;
    }
}

}  // namespace ttrt
