// Symmetric eigensolver of the Gram route, one 1024-thread workgroup, for the
// Gram matrix G = B^T B of the projected first core (n = k1 <= 128):
//  1. Householder tridiagonalisation T = Q^T G Q, Q = H_0 H_1 ... H_{n-3}
//     (two barriers per step, the next reflector formed by wave 0 while the
//     other waves finish the rank-2 update);
//  2. the K largest eigenvalues of T by multisection on Sturm counts (the
//     ratio recurrence q_j = d_j - x - e_{j-1}^2 / q_{j-1}), K = the rank cap;
//     the tail below them follows from trace(T) = trace(G);
//  3. an eigenvector of T per kept eigenvalue from the twisted factorisation
//     of T - lambda I (the twist at the smallest |gamma_r|), one thread each;
//  4. symmetric re-orthonormalisation Z <- Z (I - E / 2), E = Z^T Z - I,
//     twice (vectors of close eigenvalues are computed independently);
//  5. back-transformation V = Q Z, each wave holding its columns in
//     registers, the reflectors applied in reverse order.
// The work is O(n^3) once, where a Jacobi sweep moves the whole matrix and
// its rotation accumulator through LDS O(n) times.  Step 4 reports the
// largest |E| of its first pass; the caller falls back to Jacobi when it is
// not small (near-degenerate eigenvalues that the independent vectors do not
// separate).
#pragma once

namespace ttrt {

constexpr int kTrdMax = 128;                     // largest order
constexpr int kEigWaves = kSmallThreads / 64;    // 16
constexpr int kTrdPP = 1024;                     // partial products: parts x rows <= 16 x 64 = 8 x 128

// LDS words (doubles) of the scratch below.
constexpr size_t kTrdScratch = 4 * kTrdMax + 2 * kTrdMax + kTrdPP + 2 * kEigWaves + kTrdMax + 16 * kEigWaves;

struct TrdScratch {
    double* d;     // [kTrdMax] diagonal of T
    double* e;     // [kTrdMax] off-diagonal, e[k] = T[k + 1][k]; later e[k]^2 (normalised)
    double* tau;   // [kTrdMax] reflector factors
    double* lam;   // [kTrdMax] eigenvalues, descending
    double* vb;    // [2][kTrdMax] reflector of the current / next step (v[0] = 1)
    double* pp;    // [kTrdPP] partial products of A22 v by column part
    double* kp;    // [2 kEigWaves] per-wave partial sums
    double* zr;    // [kTrdMax] misc (Gershgorin bounds, reductions)
    double* wb;    // [16 kEigWaves] per-wave column values of w
    __device__ void carve(double* p) {
        d = p;
        e = d + kTrdMax;
        tau = e + kTrdMax;
        lam = tau + kTrdMax;
        vb = lam + kTrdMax;
        pp = vb + 2 * kTrdMax;
        kp = pp + kTrdPP;
        zr = kp + 2 * kEigWaves;
        wb = zr + kTrdMax;
    }
};

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
// Lane j's value (j uniform) in every lane, by v_readlane.
__device__ __forceinline__ double bcast1(double x, int j) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), j);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum / max over the wave, every lane receiving it: DPP within 16 lanes,
// then two lane exchanges.
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v = group_sum(v, 32);
    return v + __shfl_xor(v, 32, 64);
}
__device__ __forceinline__ double wave_max_dpp(double v) {
    v = fmax(v, dpp_swap<0xB1>(v));
    v = fmax(v, dpp_swap<0x4E>(v));
    v = fmax(v, dpp_swap<0x141>(v));
    v = fmax(v, dpp_swap<0x140>(v));
    v = fmax(v, __shfl_xor(v, 16, 64));
    return fmax(v, __shfl_xor(v, 32, 64));
}

__device__ __forceinline__ double block_max(double v, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double m = 0.0;
    for (int w = 0; w < nw; ++w) m = fmax(m, red[w]);
    __syncthreads();
    return m;
}

// Max / min over aligned groups of gs in {1, 2, 4, ..., 32} consecutive lanes.
__device__ __forceinline__ double group_max(double v, int gs) {
    for (int off = 1; off < gs; off <<= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double group_min(double v, int gs) {
    for (int off = 1; off < gs; off <<= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// Householder reflector of a column x[0..L) held by one wave (x[i] in lane
// i % 64, register i / 64): H = I - tau v v^T, v[0] = 1, H x = beta e_0
// (LAPACK's dlarfg convention).  The matrix is scaled to entries of at most
// 1 beforehand, so the norm needs no rescaling; the two reciprocals are
// independent.  Every lane gets tau and beta and its two entries of v (zero
// beyond L).
__device__ __forceinline__ void wave_reflector(const double xv[2], int L, double& tau, double& beta, double vv[2]) {
    const int l = threadIdx.x & 63;
    const double alpha = bcast1(xv[0], 0);
    double s = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = l + 64 * h;
        if (i >= 1 && i < L) s = fma(xv[h], xv[h], s);
    }
    s = wave_sum_dpp(s);
    if (!(s > 0.0)) {   // nothing below the leading entry: H = I
        tau = 0.0;
        beta = alpha;
        vv[0] = l == 0 ? 1.0 : 0.0;
        vv[1] = 0.0;
        return;
    }
    const double nn = fma(alpha, alpha, s);
    beta = -copysign(nn * rsq_refined(nn), alpha);
    const double rb = rcp_refined(beta), ra = rcp_refined(alpha - beta);
    tau = (beta - alpha) * rb;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = l + 64 * h;
        vv[h] = i == 0 ? 1.0 : (i < L ? xv[h] * ra : 0.0);
    }
}

// Tridiagonalise the symmetric n x n A (column-major, leading dimension ld,
// both triangles stored, in LDS; 2 <= n <= kTrdMax), scaled first by its
// largest |a_ij| (kept in ws.zr[4]): on return ws.d, ws.e hold T of the
// scaled matrix, ws.tau the reflector factors, and column k of A below its
// subdiagonal the tail v[1 ..] of reflector k (v[0] = 1 implied; H_k acts on
// rows k + 1 .. n - 1).  Ends with a barrier.
__device__ __forceinline__ void block_tridiag(double* A, int n, int ld, TrdScratch& ws, double* red) {
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    // scale to max |a_ij| = 1 (ws.zr[4] keeps the factor; T is of the scaled matrix)
    double am = 0.0;
    for (int idx = tid; idx < n * n; idx += blockDim.x) am = fmax(am, fabs(A[(idx % n) + (size_t)(idx / n) * ld]));
    am = block_max(am, red);
    const double gs = am > 0.0 && am < 1e300 ? am : 1.0, rg = 1.0 / gs;
    for (int idx = tid; idx < n * n; idx += blockDim.x) A[(idx % n) + (size_t)(idx / n) * ld] *= rg;
    if (tid == 0) ws.zr[4] = gs;
    __syncthreads();
    if (w == 0) {
        // reflector of step 0 from column 0 below the diagonal
        const int L = n - 1;
        double xv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = l + 64 * h;
            xv[h] = i < L ? A[1 + i] : 0.0;
        }
        double t, b, vv[2];
        wave_reflector(xv, L, t, b, vv);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = l + 64 * h;
            if (i < L) ws.vb[i] = vv[h];
            if (i >= 1 && i < L) A[1 + i] = vv[h];
        }
        if (l == 0) {
            ws.tau[0] = t;
            ws.e[0] = b;
            ws.d[0] = A[0];
        }
    }
    __syncthreads();
    for (int k = 0; k < n - 2; ++k) {
        const int L = n - k - 1;               // order of the trailing matrix A22 = A[k+1.., k+1..]
        const double t = ws.tau[k];
        const double* v = ws.vb + (k & 1) * kTrdMax;
        double* vn = ws.vb + ((k + 1) & 1) * kTrdMax;
        const int nrb = (L + 63) >> 6;         // row blocks of 64
        const int nparts = kEigWaves / nrb;    // column parts
        const int cw = ((L + nparts - 1) / nparts + 7) & ~7;   // columns per part, a multiple of 8
        const int rb = w % nrb, u = w / nrb;
        const int i = l + 64 * rb;             // this lane's row of A22
        const int j0 = u * cw, j1 = min(L, j0 + cw);
        double* A22 = A + (k + 1) + (size_t)(k + 1) * ld;
        const int pst = 64 * nrb;              // part stride of pp
        double vr[2];                          // v, two entries per lane
#pragma unroll
        for (int h = 0; h < 2; ++h) vr[h] = l + 64 * h < L ? v[l + 64 * h] : 0.0;
        if (t != 0.0) {
            // partial products p~ = A22 v over this wave's columns, and its
            // share of v^T A22 v (the broadcasts with every lane active; rows
            // past L read row L - 1 and are discarded)
            const int ic = i < L ? i : L - 1;
            double acc = 0.0;
            for (int jb = j0; jb < j1; jb += 8) {
                double vj[8], aj[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) vj[c] = v[min(jb + c, L - 1)];   // same address in every lane
#pragma unroll
                for (int c = 0; c < 8; ++c) aj[c] = A22[ic + (size_t)min(jb + c, L - 1) * ld];
#pragma unroll
                for (int c = 0; c < 8; ++c) acc = fma(aj[c], jb + c < j1 ? vj[c] : 0.0, acc);
            }
            if (i < L) ws.pp[u * pst + i] = acc;
            const double part = wave_sum_dpp(i < L ? acc * vr[rb] : 0.0);
            if (l == 0) ws.kp[w] = part;
        }
        __syncthreads();
        // w = t A22 v - kappa v, kappa = (t / 2) (t v^T A22 v); A22 <- A22 - v w^T - w v^T
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < kEigWaves; ++ww) s += ws.kp[ww];
        const double kap = 0.5 * t * t * s;
        // p~ of row r: the parts' sums (all loads issued together)
        auto w_at = [&](int r, double vrow) -> double {
            double p0 = 0.0, p1 = 0.0;
#pragma unroll
            for (int uu = 0; uu < 8; ++uu) p0 += ws.pp[uu * pst + r];
            if (nrb == 1) {
#pragma unroll
                for (int uu = 8; uu < 16; ++uu) p1 += ws.pp[uu * 64 + r];
            }
            return t * (p0 + p1) - kap * vrow;
        };
        if (w == 0) {
            // column 0 of A22 (global column k + 1) over both row blocks, then
            // the reflector of step k + 1 from its rows 1 .. L - 1
            double a[2];
            double wr[2] = {0.0, 0.0};
            if (t != 0.0) {
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if (l + 64 * h < L) wr[h] = w_at(l + 64 * h, vr[h]);
            }
            const double w0 = bcast1(wr[0], 0);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = l + 64 * h;
                a[h] = 0.0;
                if (r < L) {
                    a[h] = A22[r];
                    if (t != 0.0) {
                        a[h] -= vr[h] * w0 + wr[h];   // v[0] = 1
                        A22[r] = a[h];
                    }
                }
            }
            const int L1 = L - 1;              // x' = a[1 .. L - 1]
            double xv[2];
            const double up0 = __shfl(a[0], (l + 1) & 63, 64), up1 = __shfl(a[1], (l + 1) & 63, 64);
            xv[0] = l < 63 ? up0 : up1;        // row l + 1 (row 64 sits in lane 0, register 1)
            xv[1] = l < 63 ? up1 : 0.0;        // row l + 65 (< kTrdMax)
            if (l >= L1) xv[0] = 0.0;
            if (l + 64 >= L1) xv[1] = 0.0;
            double tn, bn, vv[2];
            wave_reflector(xv, L1, tn, bn, vv);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int m = l + 64 * h;
                if (m < L1) vn[m] = vv[h];
                if (m >= 1 && m < L1) A22[1 + m] = vv[h];   // rows k + 3 .. of column k + 1
            }
            if (l == 0) {
                ws.tau[k + 1] = tn;
                ws.e[k + 1] = bn;
                ws.d[k + 1] = a[0];
            }
        }
        if (t != 0.0) {
            const double vi = i < L ? vr[rb] : 0.0;
            const double wi = i < L ? w_at(i, vi) : 0.0;
            // this wave's columns (column 0 is wave 0's): w_j from lane j - j0
            // this wave's columns' w into its LDS slots (read back by the same wave)
            double* wbw = ws.wb + 16 * w;
            if (l < j1 - j0) wbw[l] = w_at(j0 + l, v[j0 + l]);
            const int js = u == 0 ? 1 : j0;   // column 0 is wave 0's
            const int ic = i < L ? i : L - 1;
            for (int jb = j0; jb < j1; jb += 8) {
                double vj[8], wj[8], aj[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    vj[c] = v[min(jb + c, L - 1)];
                    wj[c] = wbw[min(jb - j0 + c, 15)];
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) aj[c] = A22[ic + (size_t)min(jb + c, L - 1) * ld];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int j = jb + c;
                    if (i < L && j >= js && j < j1) A22[i + (size_t)j * ld] = aj[c] - fma(vi, wj[c], wi * vj[c]);
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) ws.d[n - 1] = A[(n - 1) + (size_t)(n - 1) * ld];
    __syncthreads();
}

// The K largest eigenvalues of T (ws.d, ws.e, order n) into ws.lam[0 .. K)
// in descending order, each to an absolute accuracy of a few ulps of ||T||,
// by multisection: S = 256 / K lanes per eigenvalue (at least 1) each count
// the eigenvalues below one point of the current interval per iteration.
// Also returns trace(T).  Overwrites ws.e with the squares of the scaled
// off-diagonals (negligible ones set to zero).  Ends with a barrier.
__device__ __forceinline__ double block_trd_eigvals(int n, int K, TrdScratch& ws) {
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    // scale, Gershgorin bounds and the trace (wave 0)
    if (w == 0) {
        double tr = 0.0, am = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = l + 64 * h;
            if (j < n) {
                tr += ws.d[j];
                am = fmax(am, fabs(ws.d[j]));
                if (j < n - 1) am = fmax(am, fabs(ws.e[j]));
            }
        }
        tr = wave_sum(tr);
        am = wave_max(am);
        if (l == 0) {
            ws.zr[0] = tr;
            ws.zr[1] = am;
        }
    }
    __syncthreads();
    const double tr = ws.zr[0], tn = ws.zr[1];
    if (!(tn > 0.0) || !(tn < 1e300)) {   // zero matrix (eigenvalues 0), or a non-finite one (propagated)
        for (int j = tid; j < K; j += blockDim.x) ws.lam[j] = tn == 0.0 ? 0.0 : tn;
        __syncthreads();
        return tr;
    }
    const double rs = 1.0 / tn, eps = 2.220446049250313e-16;
    // scaled T: d / tn and (e / tn)^2, off-diagonals below eps dropped (a perturbation of eps ||T||)
    __syncthreads();
    if (w == 0) {
        double gl = 1e300, gu = -1e300;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = l + 64 * h;
            if (j < n) {
                const double dj = ws.d[j] * rs;
                const double el = j > 0 ? fabs(ws.e[j - 1]) * rs : 0.0;
                const double er = j < n - 1 ? fabs(ws.e[j]) * rs : 0.0;
                gl = fmin(gl, dj - (el > eps ? el : 0.0) - (er > eps ? er : 0.0));
                gu = fmax(gu, dj + (el > eps ? el : 0.0) + (er > eps ? er : 0.0));
            }
        }
        gl = wave_min(gl);
        gu = wave_max(gu);
        if (l == 0) {
            ws.zr[2] = gl;
            ws.zr[3] = gu;
        }
    }
    __syncthreads();
    // e^2 of the scaled matrix in place (read above by wave 0 only); the
    // signed scaled off-diagonals into ws.vb for the eigenvectors
    for (int j = tid; j < n - 1; j += blockDim.x) {
        const double ej = ws.e[j] * rs;
        const bool keep = fabs(ej) > eps;
        ws.vb[j] = keep ? ej : 0.0;
        ws.e[j] = keep ? ej * ej : 0.0;
    }
    __syncthreads();
    const double atol = 4.0 * eps;            // on the scaled matrix (||T|| / tn <= 1 .. 3)
    const double gl = ws.zr[2] - 2.0 * atol, gu = ws.zr[3] + 2.0 * atol;
    int S = 1;
    while (S < 16 && S * 2 * K <= 256) S *= 2;
    const int grp = tid / S, sl = tid % S;    // eigenvalue group, lane in group
    const bool act = grp < K;
    const int idx = n - 1 - grp;              // ascending index of eigenvalue grp
    const int NP = 2 * S;                     // points per iteration (two per lane)
    const double bits = log2((gu - gl) / atol) + 1.0;
    const int its = (int)ceil(bits / log2((double)(NP + 1)));
    double lo = gl, hi = gu;
    // the scaled diagonal (4 past the end: a step that keeps the sign), the
    // squared off-diagonals shifted by one (es[j] = e_{j-1}^2, 0 at both
    // ends), and for the eigenvectors the unshifted squares and the signed
    // off-diagonals, into the free partial-product space (read as broadcasts)
    double* dsv = ws.pp;
    double* esv = ws.pp + kTrdMax;
    double* e2v = ws.pp + 2 * kTrdMax;
    double* eov = ws.pp + 3 * kTrdMax;
    for (int j = tid; j < kTrdMax; j += blockDim.x) {
        dsv[j] = j < n ? ws.d[j] * rs : 4.0;
        esv[j] = (j >= 1 && j < n) ? ws.e[j - 1] : 0.0;
        e2v[j] = j < n - 1 ? ws.e[j] : 0.0;
        eov[j] = j < n - 1 ? ws.vb[j] : 0.0;
    }
    __syncthreads();
    if (w < (K * S + 63) / 64) {   // waves holding eigenvalue groups (uniform)
        for (int it = 0; it < its; ++it) {
            // Sturm counts at two points: the leading principal minors of
            // T - x I by p_{j+1} = (d_j - x) p_j - e_{j-1}^2 p_{j-1} (no
            // division; p_0 = 1, p_{-1} = 0); the eigenvalues below x are the
            // sign changes (by the sign bit).  Eight steps per block, the
            // minors rescaled by a power of two after each (|d|, |e| <= 1,
            // |x| <= 3: growth at most 7^8 in between)
            const double h = (hi - lo) / (double)(NP + 1);
            const double xa = fma((double)(2 * sl + 1), h, lo), xb = fma((double)(2 * sl + 2), h, lo);
            double pa0 = 0.0, pb0 = 0.0, pa1 = 1.0, pb1 = 1.0;
            int sa = 0, sb = 0, ca = 0, cb = 0;
            for (int j0 = 0; j0 < n; j0 += 8) {
                double dj[8], ej[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    dj[u] = dsv[j0 + u];
                    ej[u] = esv[j0 + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double pa2 = fma(-ej[u], pa0, (dj[u] - xa) * pa1);
                    const double pb2 = fma(-ej[u], pb0, (dj[u] - xb) * pb1);
                    const int ta = __double_as_longlong(pa2) < 0, tb = __double_as_longlong(pb2) < 0;
                    ca += ta ^ sa;
                    cb += tb ^ sb;
                    sa = ta;
                    sb = tb;
                    pa0 = pa1;
                    pa1 = pa2;
                    pb0 = pb1;
                    pb1 = pb2;
                }
                const int ea = max(__builtin_amdgcn_frexp_exp(pa1), __builtin_amdgcn_frexp_exp(pa0));
                const int eb = max(__builtin_amdgcn_frexp_exp(pb1), __builtin_amdgcn_frexp_exp(pb0));
                pa0 = ldexp(pa0, -ea);
                pa1 = ldexp(pa1, -ea);
                pb0 = ldexp(pb0, -eb);
                pb1 = ldexp(pb1, -eb);
            }
            // cnt eigenvalues lie below x: x is a lower bound of eigenvalue idx when cnt <= idx
            const double lo_c = fmax(ca <= idx ? xa : -1e300, cb <= idx ? xb : -1e300);
            const double hi_c = fmin(ca <= idx ? 1e300 : xa, cb <= idx ? 1e300 : xb);
            lo = fmax(lo, group_max(lo_c, S));
            hi = fmin(hi, group_min(hi_c, S));
        }
        if (act && sl == 0) ws.lam[grp] = 0.5 * (lo + hi) * tn;
    }
    __syncthreads();
    return tr;
}

// Eigenvector of the scaled T (diagonal ds, squared off-diagonals e2 and the
// same shifted by one, es[i] = e2[i - 1], signed off-diagonals eo: LDS arrays
// read with the same address in every lane) for the scaled eigenvalue x, by
// the twisted factorisation T - x I = N_r D_r N_r^T: forward and backward
// pivots d+ and d-, twist r = argmin |gamma_r| (gamma_r = d+_r + d-_r - (d_r
// - x)), then z_r = 1 and the two bidiagonal solves outward, in the n doubles
// at z (this lane's own array).  Returns the largest residual |((T - x I)
// z)_i| after normalising z.  Selects rather than branches on the lane's own
// r keep the loops identical in every lane.
__device__ __forceinline__ double twisted_vector(int n, const double* ds, const double* es, const double* e2,
                                                 const double* eo, double x, double* z) {
    const double pivmin = 1e-290;
    auto piv = [&](double q) { return fabs(q) < pivmin ? -pivmin : q; };
    // forward pivots d+_i into z
    double dp = piv(ds[0] - x);
    z[0] = dp;
#pragma unroll 8
    for (int i = 1; i < n; ++i) {
        dp = piv(ds[i] - x - es[i] / dp);
        z[i] = dp;
    }
    // backward pivots d-_i and the twist
    double dm = piv(ds[n - 1] - x);
    double best = fabs(z[n - 1]);
    int r = n - 1;
#pragma unroll 8
    for (int i = n - 2; i >= 0; --i) {
        const double di = ds[i] - x;
        dm = piv(di - e2[i] / dm);
        const double g = fabs(z[i] + dm - di);
        r = g < best ? i : r;
        best = g < best ? g : best;
    }
    // U-_{i-1} = e_{i-1} / d-_i into z[i] for i > r (recomputed from the end)
    dm = piv(ds[n - 1] - x);
#pragma unroll 8
    for (int i = n - 1; i > 0; --i) {
        if (i < n - 1) dm = piv(ds[i] - x - e2[i] / dm);
        const double u = eo[i - 1] / dm;
        z[i] = i > r ? u : z[i];
    }
    // solve outward from z_r = 1: z_{i+1} = -U-_i z_i, z_i = -(e_i / d+_i) z_{i+1}
    double nrm = 1.0, zi = 1.0;
#pragma unroll 8
    for (int i = 0; i < n - 1; ++i) {
        const double zn = -z[i + 1] * zi;
        const bool up = i >= r;
        zi = up ? zn : zi;
        z[i + 1] = up ? zn : z[i + 1];
        nrm += up ? zn * zn : 0.0;
    }
    zi = 1.0;
#pragma unroll 8
    for (int i = n - 2; i >= 0; --i) {
        const double zn = -(eo[i] / z[i]) * zi;
        const bool dn = i < r;
        zi = dn ? zn : zi;
        z[i] = dn ? zn : z[i];
        nrm += dn ? zn * zn : 0.0;
    }
    z[r] = 1.0;
    const double sc = 1.0 / sqrt(nrm);
    double res = 0.0, zm = 0.0, z0 = z[0] * sc;
#pragma unroll 8
    for (int i = 0; i < n; ++i) {
        const double zp = i + 1 < n ? z[i + 1] * sc : 0.0;
        double ri = (ds[i] - x) * z0;
        if (i > 0) ri = fma(eo[i - 1], zm, ri);
        if (i + 1 < n) ri = fma(eo[i], zp, ri);
        res = fmax(res, fabs(ri));
        z[i] = z0;
        zm = z0;
        z0 = zp;
    }
    return res == res ? res : 1e300;
}

typedef double eig_f64x4 __attribute__((ext_vector_type(4)));

// E = Z^T Z - I (nv x nv <= 64 x 64, E[a + b lde]) on FP64 MFMA, one 16 x 16
// tile per wave (v_mfma_f64_16x16x4f64: A[i][k] in lane i + 16 k, B[k][j]
// in lane j + 16 k, D[i][j] in lane j + 16 (i % 4), register i / 4).
// Returns the largest |E| (a NaN as 1e300) over the block.
__device__ __forceinline__ double block_ztz_minus_i(const double* Z, int zs, int n, int nv, double* E, int lde,
                                                    double* red) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, m = l & 15, q = l >> 4;
    const int nt = (nv + 15) >> 4;
    double emax = 0.0;
    if (w < nt * nt) {
        const int ta = w / nt, tb = w - ta * nt;
        const int ra = 16 * ta + m, cb = 16 * tb + m;   // this lane's A row, B column
        eig_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < n; k0 += 4) {
            const int k = k0 + q;
            const double av = (ra < nv && k < n) ? Z[k + (size_t)ra * zs] : 0.0;
            const double bv = (cb < nv && k < n) ? Z[k + (size_t)cb * zs] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * ta + 4 * r + q, col = 16 * tb + m;
            if (row < nv && col < nv) {
                const double e = acc[r] - (row == col ? 1.0 : 0.0);
                E[row + (size_t)col * lde] = e;
                emax = fmax(emax, e == e ? fabs(e) : 1e300);
            }
        }
    }
    return block_max(emax, red);
}

// Z <- Z - Z E / 2 (Z n x nv, Z[i + a zs]; E symmetric nv x nv, E[b + a lde])
// on FP64 MFMA: 16 x 16 tiles of Z E, two per wave, in registers until a
// barrier, then the update.
__device__ __forceinline__ void block_sym_orth_step(double* Z, int zs, int n, int nv, const double* E, int lde) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, m = l & 15, q = l >> 4;
    const int nti = (n + 15) >> 4, ntj = (nv + 15) >> 4;
    eig_f64x4 acc[2];
    int ti[2], tj[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        acc[u] = (eig_f64x4){0.0, 0.0, 0.0, 0.0};
        const int t = w + kEigWaves * u;
        ti[u] = t < nti * ntj ? t / ntj : -1;
        tj[u] = t < nti * ntj ? t - (t / ntj) * ntj : 0;
        if (ti[u] < 0) continue;
        const int ra = 16 * ti[u] + m, cb = 16 * tj[u] + m;
        for (int b0 = 0; b0 < nv; b0 += 4) {
            const int b = b0 + q;
            const double av = (ra < n && b < nv) ? Z[ra + (size_t)b * zs] : 0.0;
            const double bv = (cb < nv && b < nv) ? E[b + (size_t)cb * lde] : 0.0;
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (ti[u] < 0) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * ti[u] + 4 * r + q, col = 16 * tj[u] + m;
            if (row < n && col < nv) Z[row + (size_t)col * zs] -= 0.5 * acc[u][r];
        }
    }
    __syncthreads();
}

// V = Q Z with Q = H_0 ... H_{n-3} (reflector k: v[0] = 1 at row k + 1, tail
// refl[i + k ldr] for rows i >= k + 2, factor tau[k]): wave w holds the
// columns a = w + 16 c (c < CPW) of Z in registers (RPL rows per lane, n <=
// 64 RPL) and applies the reflectors from the last to the first, staged
// eight at a time as whole vectors into stage[8][kTrdMax] (LDS) by the block.
template <int RPL, int CPW>
__device__ __forceinline__ void block_back_transform(int n, int nv, const double* refl, int ldr, const double* tau,
                                                     const double* Z, int zs, double* V, int ldv, double* stage) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    double z[CPW][RPL];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int h = 0; h < RPL; ++h) {
            const int a = w + kEigWaves * c, i = l + 64 * h;
            z[c][h] = (a < nv && i < n) ? Z[i + (size_t)a * zs] : 0.0;
        }
    for (int khi = n - 3; khi >= 0; khi -= 8) {
        __syncthreads();   // the previous chunk's readers are done
        for (int idx = threadIdx.x; idx < 8 * kTrdMax; idx += blockDim.x) {
            const int c = idx / kTrdMax, i = idx - c * kTrdMax, k = khi - c;
            double x = 0.0;
            if (k >= 0 && i < n) x = i == k + 1 ? 1.0 : (i > k + 1 ? refl[i + (size_t)k * ldr] : 0.0);
            stage[idx] = x;
        }
        __syncthreads();
        if (w < nv) {
            for (int c8 = 0; c8 < 8; ++c8) {
                const int k = khi - c8;
                if (k < 0) break;
                const double tk = tau[k];
                if (tk == 0.0) continue;
                double vh[RPL];
#pragma unroll
                for (int h = 0; h < RPL; ++h) vh[h] = stage[c8 * kTrdMax + l + 64 * h];
                double dots[CPW];
#pragma unroll
                for (int c = 0; c < CPW; ++c) {
                    double p = 0.0;
#pragma unroll
                    for (int h = 0; h < RPL; ++h) p = fma(vh[h], z[c][h], p);
                    dots[c] = p;
                }
#pragma unroll
                for (int c = 0; c < CPW; ++c) dots[c] = wave_sum_dpp(dots[c]) * tk;
#pragma unroll
                for (int c = 0; c < CPW; ++c)
#pragma unroll
                    for (int h = 0; h < RPL; ++h) z[c][h] = fma(-dots[c], vh[h], z[c][h]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int h = 0; h < RPL; ++h) {
            const int a = w + kEigWaves * c, i = l + 64 * h;
            if (a < nv && i < n) V[i + (size_t)a * ldv] = z[c][h];
        }
}

// The nv <= 64 kept eigenvectors (eigenvalues ws.lam[0 .. nv), descending)
// of the matrix that block_tridiag reduced and block_trd_eigvals scanned
// (scale tn), into V[i + a ldv]: twisted vectors of T in Z (Z[i + a zs], LDS,
// nv columns), two
// symmetric re-orthonormalisation passes with E in C (C[a + b ldc]), then
// V = Q Z (RPL, CPW as for block_back_transform).  Returns 0 on success, 1
// (V unwritten) when a vector of T has a scaled residual above 1e-9, 2 when
// the first pass finds |E| above 1e-3 (or a NaN); emax the first pass's |E|.
template <int RPL, int CPW>
__device__ __forceinline__ int block_trd_vectors(int n, int nv, TrdScratch& ws, double tn, const double* refl,
                                                 int ldr, double* Z, int zs, double* C, int ldc, double* V, int ldv,
                                                 double* red, double& emax) {
    const int tid = threadIdx.x;
    double bad = 0.0;
    if (tid < 64) {
        // lanes past nv repeat vector nv - 1 into its own column (the same
        // arithmetic, so they store the same values)
        const int a = tid < nv ? tid : nv - 1;
        const double res = twisted_vector(n, ws.pp, ws.pp + kTrdMax, ws.pp + 2 * kTrdMax, ws.pp + 3 * kTrdMax,
                                          ws.lam[a] / tn, Z + (size_t)a * zs);
        if (tid < nv && !(res <= 1e-9)) bad = 1.0;
    }
    emax = block_max(bad, red);
    if (emax != 0.0) return 1;
    for (int pass = 0; pass < 2; ++pass) {
        const double m = block_ztz_minus_i(Z, zs, n, nv, C, ldc, red);   // C = Z^T Z - I
        if (pass == 0) emax = m;
        if (pass == 0 && !(m <= 1e-3)) return 2;
        block_sym_orth_step(Z, zs, n, nv, C, ldc);
    }
    block_back_transform<RPL, CPW>(n, nv, refl, ldr, ws.tau, Z, zs, V, ldv, ws.pp);
    __syncthreads();
    return 0;
}

// Two-sided cyclic Jacobi on a symmetric n x n S (n <= 16, S[a + b ld]),
// accumulating the rotations into W (W[i + a ldw], caller-initialised), by
// one wave with no block barriers: per round, lane L < 8 forms the rotation
// of pair L of the tournament over 16 players (players >= n are zero rows and
// never rotate) into cs / pa / pb (LDS), then lane L applies R_p^T B R_q to the
// 2 x 2 block (p, q) = (L / 8, L % 8) of S and rotates two rows of W.  The
// wave's LDS writes precede its later reads in program order, so no barrier
// is needed.  Rotation, skipping and stopping rules as block_jacobi_sym64.
// Called by all 64 lanes of one wave; returns the sweeps.
__device__ __forceinline__ int wave_jacobi_sym16(double* S, int n, int ld, double* W, int ldw, double* cs, int* pa,
                                                 int* pb, double tconv) {
    const int l = threadIdx.x & 63, p = l >> 3, q = l & 7;
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += fabs(S[i + (size_t)i * ld]);
    const double floor_abs = 1e-15 * tr;
    for (int sweep = 0; sweep < 40; ++sweep) {
        int big = 0;
        for (int round = 0; round < 15; ++round) {
            if (l < 8) {
                int a, b;
                tournament_pair(l, round, 16, &a, &b);
                double c = 1.0, sn = 0.0;
                if (b < n) {
                    const double app = S[a + (size_t)a * ld], aqq = S[b + (size_t)b * ld], apq = S[a + (size_t)b * ld];
                    if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
                        double t;
                        jacobi_rotation(app, aqq, apq, &c, &sn, &t);
                        if (fabs(t) > tconv) big = 1;
                        if (fabs(t) <= 1e-10) {
                            c = 1.0;
                            sn = 0.0;
                        }
                    }
                }
                cs[2 * l] = c;
                cs[2 * l + 1] = sn;
                pa[l] = a;
                pb[l] = b;
            }
            const double sp = cs[2 * p + 1], sq = cs[2 * q + 1];
            const double cp = cs[2 * p], cq = cs[2 * q];
            const int ap = pa[p], bp = pb[p], aq = pa[q], bq = pb[q];
            if (sp != 0.0 || sq != 0.0) {   // both rotations identity: block unchanged
                // a rotation acts on existing rows / columns only (b < n), its partner a < b too;
                // an identity pair's second player may lie past n: that row / column is zero
                const bool vp = bp < n, vq = bq < n, up = ap < n, uq = aq < n;
                const double b00 = (up && uq) ? S[ap + (size_t)aq * ld] : 0.0;
                const double b01 = (up && vq) ? S[ap + (size_t)bq * ld] : 0.0;
                const double b10 = (vp && uq) ? S[bp + (size_t)aq * ld] : 0.0;
                const double b11 = (vp && vq) ? S[bp + (size_t)bq * ld] : 0.0;
                const double c00 = cq * b00 - sq * b01, c01 = sq * b00 + cq * b01;
                const double c10 = cq * b10 - sq * b11, c11 = sq * b10 + cq * b11;
                if (up && uq) S[ap + (size_t)aq * ld] = cp * c00 - sp * c10;
                if (up && vq) S[ap + (size_t)bq * ld] = cp * c01 - sp * c11;
                if (vp && uq) S[bp + (size_t)aq * ld] = sp * c00 + cp * c10;
                if (vp && vq) S[bp + (size_t)bq * ld] = sp * c01 + cp * c11;
            }
            if (sq != 0.0) {   // W <- W R: rows p and p + 8 of the column pair q
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = p + 8 * h;
                    if (i < n) {
                        double* wa = W + i + (size_t)aq * ldw;
                        double* wb = W + i + (size_t)bq * ldw;
                        const double u = *wa, v = *wb;
                        *wa = cq * u - sq * v;
                        *wb = sq * u + cq * v;
                    }
                }
            }
        }
        if (__ballot(big) == 0) return sweep + 1;
    }
    return 40;
}

}  // namespace ttrt
