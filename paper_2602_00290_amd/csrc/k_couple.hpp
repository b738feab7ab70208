// Coupled medium temperature (Section 2.1, the coupled source stage).
//
// Per step, around the rounding pass of the full operator:
//   k_couple_pre   the angle means J* of the intensity after streaming (from
//                  the current cores and the transport operator's TT terms,
//                  as a gather contraction with a one-column operand), the
//                  stage temperature T+ of every cell as the root of
//                      T^m - T+ - sum_g (4 pi dt kappa_g d_g / C_v) (eps_g(T+) - J*_g) = 0,
//                  d = 1 / (1 + c dt kappa) (the paper's scalar equation with
//                  the implicit J^{m+1}(T+) substituted), and eps_g(T+) where
//                  the rank-1 emission column of the operator reads it;
//   k_couple_post  the new medium temperature from total-energy conservation,
//                      C_v (T^{m+1} - T^m) = (4 pi / c) sum_g (J*_g - J_g^{m+1}),
//                  with J^{m+1} the angle means of the rounded new state.
// J = (1 / 4 pi) sum_lp w_l w_p I.  One wave per cell, lanes over groups; the
// root solve is a Newton iteration kept inside a sign-changing bracket
// (bisection when a step leaves it).  Wave sums reach every lane bitwise equal
// (each butterfly step adds the same two values), so the iteration's control
// flow is wave-uniform.
#pragma once

#include "k_big.hpp"
#include "planck.hpp"
#include "tt_common.hpp"

namespace ttrt {

constexpr int kCoupleThreads = 256;   // 4 waves, one cell each at a time

struct CoupleArgs {
    const double* edges;     // N_nu + 1 group edges (last: +inf)
    const double* wth;       // N_theta polar weights
    const double* wph;       // N_phi azimuthal weights
    const double* gtab;      // (1 + n_terms) x N_theta angular factors of the operator terms
    const double* htab;      // (1 + n_terms) x N_phi
    double* T;               // N_X medium temperature
    double* Js;              // M angle means after streaming (pre -> post)
    double* eps;             // M emission, read by the rank-1 emission column
    float* R1;               // fused rank-1 block of the full operator (or null)
    int rw1, qe1;            // its width and emission column (-1: none)
    float* R2;               // fused rank-1 block of the source operator (or null)
    int rw2, qe2;
    double heat_capacity;    // C_v = rho c_v
    double dt;
    double c;
};

// Dynamic LDS (doubles) of k_couple_pre: one-column operand (K), per-term
// angular moments of Theta (n_rblk x r1) and of Phi (n_rblk x r2).
__host__ __device__ inline size_t couple_lds_doubles(int kall_cap, int n_rblk, int r1cap, int r2cap) {
    return (size_t)kall_cap + (size_t)n_rblk * r1cap + (size_t)n_rblk * r2cap + 8;
}

template <typename T>
__global__ __launch_bounds__(kCoupleThreads) void k_couple_pre(Geom g, OpDesc op, RowData rd, const DevState* st,
                                                               const T* __restrict__ Z, const double* __restrict__ Th,
                                                               const double* __restrict__ Ph, CoupleArgs ca) {
    extern __shared__ double cl[];
    const int r1 = st->r1, r2 = st->r2, ldz = st->ldz;
    const int nt = g.nt, np = g.np, G = g.G;
    const int nrb = op.n_rblk, ng = op.n_gather, nr1 = op.n_r1;
    const int KG = ng * ldz;
    double* GJ = cl;                       // KG + nr1
    double* Mt = GJ + KG + nr1;            // nrb x r1
    double* hp = Mt + (size_t)nrb * r1;    // nrb x r2
    const double inv4pi = 0.25 / M_PI;
    // angular moment of Phi per term: hp[t][b] = sum_p w_p h_t(p) Phi[b, p]
    for (int idx = threadIdx.x; idx < nrb * r2; idx += blockDim.x) {
        const int t = idx / r2, b = idx - t * r2;
        const double* h = ca.htab + (size_t)op.rfac[t] * np;
        double s = 0.0;
        for (int p = 0; p < np; ++p) s += ca.wph[p] * h[p] * Ph[(size_t)b * np + p];
        hp[idx] = s;
    }
    __syncthreads();
    // Mt[t][a] = (1 / 4 pi) sum_l w_l g_t(l) sum_b Theta[a, l, b] hp[t][b]
    for (int idx = threadIdx.x; idx < nrb * r1; idx += blockDim.x) {
        const int t = idx / r1, a = idx - t * r1;
        const double* gt = ca.gtab + (size_t)op.rfac[t] * nt;
        const double* hpt = hp + (size_t)t * r2;
        double s = 0.0;
        for (int l = 0; l < nt; ++l) {
            const double* th = Th + ((size_t)a * nt + l) * r2;
            double u = 0.0;
            for (int b = 0; b < r2; ++b) u += th[b] * hpt[b];
            s += ca.wth[l] * gt[l] * u;
        }
        Mt[idx] = inv4pi * s;
    }
    __syncthreads();
    // one-column operand: gather block j, row a < ldz; then the rank-1 columns
    for (int idx = threadIdx.x; idx < KG; idx += blockDim.x) {
        const int j = idx / ldz, a = idx - j * ldz;
        double v = 0.0;
        if (a < r1)
            for (int t = 0; t < nrb; ++t) {
                const double m = Mt[(size_t)t * r1 + a];
                if (j == 0) v += op.rcoef0[t] * m;
                if (op.rshift[t] == j) v += op.rcoef[t] * m;
            }
        GJ[idx] = v;
    }
    for (int q = threadIdx.x; q < nr1; q += blockDim.x) {
        const double* gt = ca.gtab + (size_t)op.r1fac[q] * nt;
        const double* ht = ca.htab + (size_t)op.r1fac[q] * np;
        double sg = 0.0, sh = 0.0;
        for (int l = 0; l < nt; ++l) sg += ca.wth[l] * gt[l];
        for (int p = 0; p < np; ++p) sh += ca.wph[p] * ht[p];
        GJ[KG + q] = inv4pi * sg * sh;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long ncell = g.M / G;
    const double C = ca.heat_capacity, dt = ca.dt, cdt = g.cdt;
    for (long long cell = (long long)blockIdx.x * 4 + w; cell < ncell; cell += (long long)gridDim.x * 4) {
        const double Tm = ca.T[cell];
        double F0 = 0.0;
        for (int gg = lane; gg < G; gg += 64) {
            const long long k = cell * G + gg;
            double js = 0.0;
            for (int j = 0; j < ng; ++j) {
                const long long src = j == 0 ? k : neighbour_row(g, k, op.gaxis[j], op.gdir[j]);
                if (src < 0) continue;
                const T* zr = Z + src * ldz;
                const double* gj = GJ + (size_t)j * ldz;
                for (int a = 0; a < r1; ++a) js += (double)zr[a] * gj[a];
            }
            for (int q = 0; q < nr1; ++q) js += rank1_value(g, op, rd, k, q) * GJ[KG + q];
            ca.Js[k] = js;
            const double kap = row_kappa(g, rd, k);
            F0 += 4.0 * M_PI * dt * kap / (1.0 + cdt * kap) / C * js;
        }
        F0 = wave_sum(F0);
        // f(T) = Tm - T - sum_g coef_g (eps_g(T) - J*_g) and f'(T), summed over the wave
        auto eval = [&](double Tt, double& f, double& df) {
            double s = 0.0, ds = 0.0;
            for (int gg = lane; gg < G; gg += 64) {
                const long long k = cell * G + gg;
                const double kap = row_kappa(g, rd, k);
                const double coef = 4.0 * M_PI * dt * kap / (1.0 + cdt * kap) / C;
                double de;
                const double e = group_emission_1(ca.edges[gg], ca.edges[gg + 1], Tt, &de);
                s += coef * (e - ca.Js[k]);
                ds += coef * de;
            }
            s = wave_sum(s);
            ds = wave_sum(ds);
            f = Tm - Tt - s;
            df = -1.0 - ds;
        };
        // f(hi) <= 0 at hi = Tm + sum coef J* (eps >= 0); widen if rounding put hi below the root
        double lo = 0.0, hi = fmax(fmax(Tm + F0, Tm), 1e-300);
        double f, df;
        eval(hi, f, df);
        for (int it = 0; f > 0.0 && it < 64; ++it) {
            lo = hi;
            hi *= 2.0;
            eval(hi, f, df);
        }
        double Tc = hi;
        for (int it = 0; it < 100 && f != 0.0; ++it) {
            if (f > 0.0) lo = Tc; else hi = Tc;
            double Tn = Tc - f / df;
            if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
            const bool done = fabs(Tn - Tc) <= 1e-15 * Tn;
            Tc = Tn;
            eval(Tc, f, df);
            if (done) break;
        }
        for (int gg = lane; gg < G; gg += 64) {
            const long long k = cell * G + gg;
            const double e = group_emission_1(ca.edges[gg], ca.edges[gg + 1], Tc, nullptr);
            ca.eps[k] = e;
            const double v = cdt * row_kappa(g, rd, k) * e;
            if (ca.R1 && ca.qe1 >= 0) ca.R1[k * ca.rw1 + ca.qe1] = (float)v;
            if (ca.R2 && ca.qe2 >= 0) ca.R2[k * ca.rw2 + ca.qe2] = (float)v;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kCoupleThreads) void k_couple_post(Geom g, const DevState* st, const T* __restrict__ Z,
                                                                const double* __restrict__ Th,
                                                                const double* __restrict__ Ph, CoupleArgs ca) {
    extern __shared__ double cl[];
    const int r1 = st->r1, r2 = st->r2, ldz = st->ldz;
    const int nt = g.nt, np = g.np, G = g.G;
    double* v = cl;         // r1: angle-mean functional of the rows of Z
    double* hp = v + r1;    // r2
    for (int b = threadIdx.x; b < r2; b += blockDim.x) {
        double s = 0.0;
        for (int p = 0; p < np; ++p) s += ca.wph[p] * Ph[(size_t)b * np + p];
        hp[b] = s;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < r1; a += blockDim.x) {
        double s = 0.0;
        for (int l = 0; l < nt; ++l) {
            const double* th = Th + ((size_t)a * nt + l) * r2;
            double u = 0.0;
            for (int b = 0; b < r2; ++b) u += th[b] * hp[b];
            s += ca.wth[l] * u;
        }
        v[a] = 0.25 / M_PI * s;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long ncell = g.M / G;
    const double coefT = 4.0 * M_PI / (ca.c * ca.heat_capacity);
    for (long long cell = (long long)blockIdx.x * 4 + w; cell < ncell; cell += (long long)gridDim.x * 4) {
        double diff = 0.0;
        for (int gg = lane; gg < G; gg += 64) {
            const long long k = cell * G + gg;
            const T* zr = Z + k * ldz;
            double jn = 0.0;
            for (int a = 0; a < r1; ++a) jn += (double)zr[a] * v[a];
            diff += ca.Js[k] - jn;
        }
        diff = wave_sum(diff);
        if (lane == 0) ca.T[cell] += coefT * diff;
    }
}

}  // namespace ttrt
