// Randomized rounding (the solver's third rounding method, Section 3.1
// footnote): before the delta-truncated SVD rounding, the TT sum is compressed
// to sketch ranks l = (incoming solution ranks) + p by the
// randomize-then-orthogonalize scheme of the cited randomized rounding work.
//
// The sum is never formed here: after k_prep it is B x (Q_Theta, Q_Phi) with
// B = Z_new L (M x k1, projected by the big kernels) and Q_Theta, Q_Phi right-
// orthonormal.  Contracting the sum from the right with a random TT (cores
// G2: l1 x N_theta x l2, G3: l2 x N_phi) gives Omega = (Q_Theta, Q_Phi) x
// (G2, G3) (k1 x l1), and the first-core sketch is Y1 = B Omega.  Everything
// the scheme needs from Y1 follows from the FP64 Gram G = B^T B:
//   Y1^T Y1 = Omega^T G Omega = V Lambda V^T,   Q1 = B Omega V Lambda^-1/2,
//   Q1^T B = Lambda^-1/2 V^T Omega^T G,
// so the compression costs no pass over the first core.  The middle core is
// then projected exactly as in the scheme (sketch with G3, orthonormal basis,
// projection), the compressed TT (Q1, Q2, Phi') is right-orthogonalised again,
// and the SVD chain truncates it: its first core is B P (P = k1 x k~1) with
// Gram P^T G P.  After the chain, k_rand_fold forms the output operand P V_r.
//
// Sketch directions whose singular value is at most kRandKeep times the
// largest are dropped (a sketch wider than the tensor's rank has a null
// part); through the Gram, singular values are resolved to ~1e-8 of the
// largest, below that threshold.
#pragma once

#include "k_small.hpp"

namespace ttrt {

constexpr double kRandKeep = 1e-7;

// Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds over a
// 128-bit counter; each multiplies counter words 0 and 2 by the round
// multipliers and mixes both product halves with words 1 and 3 and the key,
// which is bumped by the Weyl increments between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, unsigned k0, unsigned k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
        c = make_uint4((unsigned)(p1 >> 32) ^ c.y ^ k0, (unsigned)p1, (unsigned)(p0 >> 32) ^ c.w ^ k1, (unsigned)p0);
    }
    return c;
}

// Entry e of sketch core `core` (0: G2, 1: G3) in rounding pass `round`: the
// counter (e, core, round, 0) under the key (seed mod 2^32, seed div 2^32);
// words 0 and 1 give x = w0 2^21 + (w1 >> 11) < 2^53 and the entry
// x 2^-52 - 1, uniform on [-1, 1) and exact in FP64.
__device__ __forceinline__ double sketch_entry(unsigned long long seed, int core, int round, int e) {
    const uint4 w = philox4x32_10(make_uint4((unsigned)e, (unsigned)core, (unsigned)round, 0u), (unsigned)seed,
                                  (unsigned)(seed >> 32));
    const unsigned long long x = ((unsigned long long)w.x << 21) | (unsigned long long)(w.y >> 11);
    return (double)x * 0x1p-52 - 1.0;
}

// Buffers of the randomized rounding (FP64, global).
struct RandBufs {
    double* G;      // kp x kp (row-major): Gram of the compressed first core, the chain's input
    double* QTh;    // k1cap x N_theta x k2cap: right-orthonormal middle core of the compressed TT
    double* QPh;    // k2cap x N_phi: its last core
    double* P;      // k1cap x k1cap: compressed first core = B P (row-major, k1 x k~1)
    double* Veff;   // k1cap x k1cap: output operand P V_r, column a at a * k1
    double* w;      // working area
};

// Doubles of RandBufs::w for the given caps (each piece rounded to even).
__host__ __device__ inline size_t rand_work_doubles(int k1cap, int nt, int np, int k2cap) {
    const size_t a = (size_t)k1cap * (k1cap + 2), b = (size_t)k1cap * nt * k2cap + 2;
    const size_t c = (size_t)k2cap * (np > k2cap ? np : k2cap) + 2;
    return 12 * a + 8 * b + 6 * c + 4 * (size_t)(k1cap + np + 2) + 64;
}

// Compression of the TT sum to the sketch ranks (one workgroup).  Inputs: the
// Gram G (k1 x k1, leading dimension ldg) of B and the right-orthonormal cores
// Q_Theta, Q_Phi left by k_prep; the incoming ranks st->r1, st->r2 and the
// pass number st->rounds key the sketch.  Outputs: RandBufs G, QTh, QPh, P,
// and st->k1, st->k2 set to the compressed TT's ranks for the SVD chain
// (st->k1b keeps the columns of B).  Warm starts are switched off (the sketch
// basis changes every pass).
__global__ __launch_bounds__(kSmallThreads) void k_rand_sketch(Geom g, DevState* st, const double* __restrict__ G,
                                                              int ldg, const double* __restrict__ QTh,
                                                              const double* __restrict__ QPh, int p_over,
                                                              unsigned long long seed, RandBufs rb, int kp_out) {
    extern __shared__ double lds[];
    __shared__ double red[16];
    __shared__ double cs[2 * 128];
    __shared__ int pa_[128], pb_[128];
    __shared__ int perm[128];
    __shared__ double sval[128];
    __shared__ int sh_flag;
    __shared__ int sh_n;
    LdsCarver cv{lds, 0, (size_t)kSmallLdsBytes / sizeof(double)};
    const int tid = threadIdx.x, nth = blockDim.x;
    const int nt = g.nt, npn = g.np;
    const int k1 = st->k1, k2 = st->k2, m2 = nt * k2;
    const int l1 = min(st->r1 + p_over, k1), l2 = min(st->r2 + p_over, k2);
    const int rnd = st->rounds;
    double* wk = rb.w;
    auto take = [&](size_t n) {
        double* q = wk;
        wk += (n + 1) & ~(size_t)1;
        return q;
    };
    // LDS where it fits (iterated arrays first), else the global work area
    auto place = [&](size_t n) { return cv.take(n, take(n)); };
    // random cores: R2[(a nt + l) l2 + b], R3[b np + p]
    double* R3 = take((size_t)l2 * npn);
    double* R2 = take((size_t)l1 * nt * l2);
    for (int e = tid; e < l2 * npn; e += nth) R3[e] = sketch_entry(seed, 1, rnd, e);
    for (int e = tid; e < l1 * nt * l2; e += nth) R2[e] = sketch_entry(seed, 0, rnd, e);
    __syncthreads();
    // W3 = Q_Phi G3^T (k2 x l2)
    double* W3 = take((size_t)k2 * l2);
    for (int idx = tid; idx < k2 * l2; idx += nth) {
        const int c = idx / l2, b = idx - c * l2;
        double acc = 0.0;
        for (int p = 0; p < npn; ++p) acc += QPh[(size_t)c * npn + p] * R3[(size_t)b * npn + p];
        W3[idx] = acc;
    }
    __syncthreads();
    // U[a][l k2 + c] = sum_b G2[a, l, b] W3[c, b]  (l1 x m2)
    double* U = take((size_t)l1 * m2);
    for (int idx = tid; idx < l1 * m2; idx += nth) {
        const int a = idx / m2, j = idx - a * m2;
        const int l = j / k2, c = j - l * k2;
        double acc = 0.0;
        for (int b = 0; b < l2; ++b) acc += R2[((size_t)a * nt + l) * l2 + b] * W3[(size_t)c * l2 + b];
        U[idx] = acc;
    }
    __syncthreads();
    // Omega = Q_Theta U^T (k1 x l1), GO = G Omega, S = Omega^T G Omega (l1 x l1)
    double* Om = take((size_t)k1 * l1);
    block_mm_tiled(k1, l1, m2, QTh, m2, 1, U, 1, m2, Om, l1, 1);
    __syncthreads();
    double* GO = take((size_t)k1 * l1);
    block_mm_tiled(k1, l1, k1, G, ldg, 1, Om, l1, 1, GO, l1, 1);
    __syncthreads();
    const int ldS = l1 | 1;
    double* S = place((size_t)l1 * ldS);
    double* V1 = place((size_t)l1 * ldS);
    block_mm_tiled(l1, l1, k1, Om, 1, l1, GO, l1, 1, S, 1, ldS);
    for (int idx = tid; idx < l1 * l1; idx += nth) {
        const int j = idx / l1, i = idx - j * l1;
        V1[i + (size_t)j * ldS] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < l1 * l1; idx += nth) {
        const int j = idx / l1, i = idx - j * l1;
        if (i < j) {
            const double v = 0.5 * (S[i + (size_t)j * ldS] + S[j + (size_t)i * ldS]);
            S[i + (size_t)j * ldS] = v;
            S[j + (size_t)i * ldS] = v;
        }
    }
    __syncthreads();
    // no rotation is skipped: P1 divides eigenvector j by sigma_j, so a
    // coupling c left between directions 1 and j would leave Q1_j a component
    // c sigma_1 / sigma_j along the dominant direction (Q1 no longer orthonormal)
    block_jacobi_sym_wide(S, l1, ldS, V1, ldS, cs, pa_, pb_, &sh_flag, 1e-8, 0.0);
    for (int j = tid; j < l1; j += nth) sval[j] = fmax(S[j + (size_t)j * ldS], 0.0);
    __syncthreads();
    block_sort_desc(sval, l1, perm);
    if (tid == 0) {
        int n = 1;
        while (n < l1 && sval[perm[n]] > kRandKeep * kRandKeep * sval[perm[0]]) ++n;
        sh_n = n;
    }
    __syncthreads();
    const int l1k = sh_n;
    // P1 = Omega V Lambda^-1/2 over the kept directions (Q1 = B P1), Mq = P1^T G (= Q1^T B)
    double* P1 = place((size_t)k1 * l1k);
    for (int idx = tid; idx < k1 * l1k; idx += nth) {
        const int a = idx / l1k, j = idx - a * l1k;
        const double lam = sval[perm[j]];
        double acc = 0.0;
        for (int al = 0; al < l1; ++al) acc += Om[(size_t)a * l1 + al] * V1[al + (size_t)perm[j] * ldS];
        P1[idx] = lam > 0.0 ? acc / sqrt(lam) : 0.0;
    }
    __syncthreads();
    // second orthonormalisation of Q1 = B P1 in the Gram metric (Cholesky QR
    // twice): the rounding of Omega^T G Omega leaves eigenvector j a component
    // ~eps along the dominant directions, which 1 / sigma_j magnifies; with
    // H = P1^T G P1 = R^T R, P1 <- P1 R^-1 restores Q1^T Q1 = I to the
    // rounding of H itself
    {
        double* GP = take((size_t)k1 * l1k);
        block_mm_tiled(k1, l1k, k1, G, ldg, 1, P1, l1k, 1, GP, l1k, 1);
        __syncthreads();
        double* H = place((size_t)l1k * l1k);
        double* Rc = place((size_t)l1k * l1k);
        block_mm_tiled(l1k, l1k, k1, P1, 1, l1k, GP, l1k, 1, H, l1k, 1);
        __syncthreads();
        // right-looking Cholesky: row j of R from the current trailing block,
        // then the trailing block loses R_j^T R_j (one barrier per column)
        for (int j = 0; j < l1k; ++j) {
            const double hjj = H[(size_t)j * l1k + j];
            const double rjj = sqrt(fmax(hjj, 1e-300));
            for (int c = j + tid; c < l1k; c += nth) Rc[(size_t)j * l1k + c] = c == j ? rjj : H[(size_t)j * l1k + c] / rjj;
            const int nb = l1k - j - 1;
            for (int idx = tid; idx < nb * nb; idx += nth) {
                const int a = j + 1 + idx / nb, b = j + 1 + idx % nb;
                H[(size_t)a * l1k + b] -= H[(size_t)j * l1k + a] * H[(size_t)j * l1k + b] / fmax(hjj, 1e-300);
            }
            __syncthreads();
        }
        // P1 <- P1 R^-1: forward substitution along each row
        for (int i = tid; i < k1; i += nth) {
            double* row = P1 + (size_t)i * l1k;
            for (int c = 0; c < l1k; ++c) {
                double v = row[c];
                for (int k = 0; k < c; ++k) v -= row[k] * Rc[(size_t)k * l1k + c];
                row[c] = v / Rc[(size_t)c * l1k + c];
            }
        }
        __syncthreads();
    }
    double* Mq = take((size_t)l1k * k1);
    block_mm_tiled(l1k, k1, k1, P1, 1, l1k, G, ldg, 1, Mq, k1, 1);
    __syncthreads();
    // Theta' = Mq x_1 Q_Theta (l1k x m2, row-major = (l1k N_theta) x k2)
    double* Thp = take((size_t)l1k * m2);
    block_mm_tiled(l1k, m2, k1, Mq, k1, 1, QTh, m2, 1, Thp, m2, 1);
    __syncthreads();
    // middle-core sketch Y2 = Theta'_(2) W3 ((l1k N_theta) x l2, column-major)
    const int mY = l1k * nt;
    double* Y2 = place((size_t)mY * l2);
    double* V2 = place((size_t)l2 * l2);
    double* nrm = place((size_t)l2);
    block_mm_tiled(mY, l2, k2, Thp, k2, 1, W3, l2, 1, Y2, 1, mY);
    for (int idx = tid; idx < l2 * l2; idx += nth) V2[idx] = (idx % l2 == idx / l2) ? 1.0 : 0.0;
    __syncthreads();
    block_jacobi_1s(Y2, mY, mY, l2, V2, l2, nrm, &sh_flag, red);
    for (int j = tid; j < l2; j += nth) {
        double acc = 0.0;
        for (int i = 0; i < mY; ++i) acc += Y2[i + (size_t)j * mY] * Y2[i + (size_t)j * mY];
        sval[j] = sqrt(acc);
    }
    __syncthreads();
    block_sort_desc(sval, l2, perm);
    if (tid == 0) {
        int n = 1;
        while (n < l2 && sval[perm[n]] > kRandKeep * sval[perm[0]]) ++n;
        sh_n = n;
    }
    __syncthreads();
    const int l2k = sh_n;
    // Q2: the kept columns of Y2 V2, normalised ((l1k N_theta) x l2k, column-major)
    double* Q2 = place((size_t)mY * l2k);
    for (int idx = tid; idx < mY * l2k; idx += nth) {
        const int q = idx / mY, i = idx - q * mY;
        const double s = sval[perm[q]];
        Q2[idx] = s > 0.0 ? Y2[i + (size_t)perm[q] * mY] / s : 0.0;
    }
    __syncthreads();
    // M2 = Q2^T Theta'_(2) (l2k x k2), Phi' = M2 Q_Phi (l2k x N_phi)
    double* M2 = take((size_t)l2k * k2);
    block_mm_tiled(l2k, k2, mY, Q2, mY, 1, Thp, k2, 1, M2, k2, 1);
    __syncthreads();
    double* Php = place((size_t)l2k * npn);
    block_mm_tiled(l2k, npn, k2, M2, k2, 1, QPh, npn, 1, Php, npn, 1);
    __syncthreads();
    // right-orthogonalise the last core: Phi'^T (N_phi x l2k, column-major: the
    // same memory as Phi' row-major) = Q R, so Phi' = R^T Q^T; kk = l2k <= N_phi
    const int kk = l2k;
    double* tau = take((size_t)(k1 > npn ? k1 : npn) + nt * k2);
    block_householder_qr(Php, npn, npn, l2k, tau, red);
    double* Lf = take((size_t)l2k * kk);   // R^T (l2k x kk)
    for (int idx = tid; idx < l2k * kk; idx += nth) {
        const int q = idx / kk, c = idx - q * kk;
        Lf[idx] = c <= q ? Php[c + (size_t)q * npn] : 0.0;
    }
    __syncthreads();
    block_form_q(Php, npn, npn, kk, tau, rb.QPh, npn);   // rb.QPh[p + c np] = Q[p][c] = Q_Phi'[c][p]
    // Theta^ = Q2 x_3 R^T ((l1k N_theta) x kk row-major = l1k x (N_theta kk))
    const int mT = nt * kk;
    double* Thh = place((size_t)mY * kk);
    block_mm_tiled(mY, kk, l2k, Q2, 1, mY, Lf, kk, 1, Thh, kk, 1);
    __syncthreads();
    // Theta^ (l1k x mT) = R^T Q^T from the QR of its transpose (mT x l1k,
    // column-major: the same memory); k~1 = min(mT, l1k)
    const int kt1 = mT < l1k ? mT : l1k;
    block_householder_qr(Thh, mT, mT, l1k, tau, red);
    double* Lt = take((size_t)l1k * kt1);   // R^T (l1k x kt1)
    for (int idx = tid; idx < l1k * kt1; idx += nth) {
        const int j = idx / kt1, a = idx - j * kt1;
        Lt[idx] = a <= j ? Thh[a + (size_t)j * mT] : 0.0;
    }
    __syncthreads();
    block_form_q(Thh, mT, mT, kt1, tau, rb.QTh, mT);   // rb.QTh[i + a mT] = Q_Theta'[a][i]
    // P = P1 R^T (k1 x kt1); Gram of the compressed first core P^T G P
    block_mm_tiled(k1, kt1, l1k, P1, l1k, 1, Lt, kt1, 1, rb.P, kt1, 1);
    __syncthreads();
    double* PG = take((size_t)kt1 * k1);
    block_mm_tiled(kt1, k1, k1, rb.P, 1, kt1, G, ldg, 1, PG, k1, 1);
    __syncthreads();
    block_mm_tiled(kt1, kt1, k1, PG, k1, 1, rb.P, kt1, 1, rb.G, kp_out, 1);
    __syncthreads();
    for (int idx = tid; idx < kt1 * kt1; idx += nth) {
        const int j = idx / kt1, i = idx - j * kt1;
        if (i < j) {
            const double v = 0.5 * (rb.G[(size_t)i * kp_out + j] + rb.G[(size_t)j * kp_out + i]);
            rb.G[(size_t)i * kp_out + j] = v;
            rb.G[(size_t)j * kp_out + i] = v;
        }
    }
    __syncthreads();
    if (tid == 0) {
        st->k1 = kt1;
        st->k2 = kk;
        st->canon = 0;
        st->l1s = l1k;
        st->l2s = l2k;
    }
}

// Output operand of a randomized pass: V_eff = P V_r (k1 x r1n, V_r the sorted
// right singular vectors the chain left in Wkeep, k~1 x r1n), written as the
// chain writes V (Vout[i ldzn + a] in the contraction precision, i < ldb) and
// column-wise for k_fold (Veff[a k1 + i]); then st->k1 is the columns of B again.
template <typename TC>
__global__ __launch_bounds__(1024) void k_rand_fold(DevState* st, const double* __restrict__ P,
                                                     const double* __restrict__ Wkeep, double* __restrict__ Veff,
                                                     TC* __restrict__ Vout) {
    const int k1 = st->k1b, kt = st->k1, r1n = st->r1n, ldzn = st->ldzn, ldb = st->ldb;
    for (int idx = threadIdx.x; idx < ldb * ldzn; idx += blockDim.x) {
        const int i = idx / ldzn, a = idx - i * ldzn;
        double v = 0.0;
        if (i < k1 && a < r1n) {
            for (int j = 0; j < kt; ++j) v += P[(size_t)i * kt + j] * Wkeep[(size_t)a * kt + j];
            Veff[(size_t)a * k1 + i] = v;
        }
        Vout[idx] = (TC)v;
    }
    __syncthreads();
    if (threadIdx.x == 0) st->k1 = k1;
}

}  // namespace ttrt
