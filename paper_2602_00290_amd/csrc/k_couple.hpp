// Source pre-pass: the coupled medium temperature (Section 2.1, the coupled
// source stage) and isotropic scattering (the kappa_s term of the source
// update).
//
// With scattering, J^{m+1} = (J* + a eps) / (1 + a) (a = c dt kappa; the
// scattering term drops out of the angle mean of the update) enters the
// isotropic source column c dt (kappa eps + kappa_s J^{m+1}); k_couple_pre
// writes it per row, after the stage temperature when T is coupled and from
// the fixed emission otherwise.
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
    const int* nbr;          // fused neighbour table (M x ns) or null
    int ns;
    double heat_capacity;    // C_v = rho c_v
    double dt;
    double c;
    int coupled;             // 1: solve for the stage temperature; 0: fixed emission
    double* jn;              // M angle means J^{m+1} (with scattering) or null
};

// Lanes work in segments of the next power of two >= N_nu (at most 64): a
// wave takes 64 / segment cells at once; with more groups it loops over them.
__host__ __device__ inline int couple_seg(int G) {
    int p = 1;
    while (p < G && p < 64) p <<= 1;
    return p;
}

// sum over the lanes of one aligned segment of `seg` lanes (a power of two)
__device__ inline double seg_sum(double v, int seg) {
    for (int off = seg >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum_{a < r} z[a] v[a] over a row of Z (rows start 32-byte aligned: the
// leading dimension is a multiple of 8), with 16-byte loads
template <typename T>
__device__ inline double row_dot(const T* __restrict__ zr, const double* __restrict__ v, int r) {
    double s = 0.0;
    int a = 0;
    if constexpr (sizeof(T) == 4) {
        for (; a + 4 <= r; a += 4) {
            const float4 z = *reinterpret_cast<const float4*>(zr + a);
            s += (double)z.x * v[a] + (double)z.y * v[a + 1] + (double)z.z * v[a + 2] + (double)z.w * v[a + 3];
        }
    } else {
        for (; a + 2 <= r; a += 2) {
            const double2 z = *reinterpret_cast<const double2*>(zr + a);
            s += (double)z.x * v[a] + (double)z.y * v[a + 1];
        }
    }
    for (; a < r; ++a) s += (double)zr[a] * v[a];
    return s;
}

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
                if (op.rshift2[t] == j) v += op.rcoef2[t] * m;
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
    const int Gp = couple_seg(G), cpw = 64 / Gp, seg = lane / Gp, gl = lane - seg * Gp;
    const bool one = G <= 64;   // at most one group per lane: its values stay in registers
    const long long ncell = g.M / G;
    const double C = ca.heat_capacity, dt = ca.dt, cdt = g.cdt;
    for (long long c0 = ((long long)blockIdx.x * 4 + w) * cpw; c0 < ncell; c0 += (long long)gridDim.x * 4 * cpw) {
        const long long cell = c0 + seg;
        if (cell >= ncell) continue;   // this segment has no cell (segments are independent)
        const double Tm = ca.coupled ? ca.T[cell] : 0.0;
        double F0 = 0.0, js1 = 0.0, coef1 = 0.0;
        for (int gg = gl; gg < G; gg += Gp) {
            const long long k = cell * G + gg;
            double js = row_dot(Z + k * ldz, GJ, r1);
            for (int j = 1; j < ng; ++j) {
                const long long src = ca.nbr ? (long long)ca.nbr[k * ca.ns + j - 1]
                                             : neighbour_row(g, k, op.gaxis[j], op.gdir[j]);
                if (src >= 0) js += row_dot(Z + src * ldz, GJ + (size_t)j * ldz, r1);
            }
            // inflow columns: the first columns of the fused rank-1 block when there is one
            for (int q = 0; q < nr1; ++q)
                js += (ca.R1 ? (double)ca.R1[k * ca.rw1 + q] : rank1_value(g, op, rd, k, q)) * GJ[KG + q];
            ca.Js[k] = js;
            js1 = js;
            if (ca.coupled) {
                const double kap = row_kappa(g, rd, k);
                const double coef = 4.0 * M_PI * dt * kap / (1.0 + cdt * kap) / C;
                F0 += coef * js;
                coef1 = coef;
            }
        }
        double e1 = 0.0, de1 = 0.0, Te = 0.0, Tc = 0.0;
        if (ca.coupled) {
            F0 = seg_sum(F0, Gp);
            // f(T) = Tm - T - sum_g coef_g (eps_g(T) - J*_g) and f'(T), summed over the segment;
            // the lane keeps its last emission and derivative (e1, de1 at Te)
            auto eval = [&](double Tt, double& f, double& df) {
                double s = 0.0, ds = 0.0;
                if (one) {
                    if (gl < G) {
                        e1 = group_emission_1(ca.edges[gl], ca.edges[gl + 1], Tt, &de1);
                        s = coef1 * (e1 - js1);
                        ds = coef1 * de1;
                    }
                } else {
                    for (int gg = gl; gg < G; gg += Gp) {
                        const long long k = cell * G + gg;
                        const double kap = row_kappa(g, rd, k);
                        const double coef = 4.0 * M_PI * dt * kap / (1.0 + cdt * kap) / C;
                        double de;
                        const double e = group_emission_1(ca.edges[gg], ca.edges[gg + 1], Tt, &de);
                        s += coef * (e - ca.Js[k]);
                        ds += coef * de;
                    }
                }
                Te = Tt;
                s = seg_sum(s, Gp);
                ds = seg_sum(ds, Gp);
                f = Tm - Tt - s;
                df = -1.0 - ds;
            };
            // Newton from T^m (the stage temperature is usually close to it) inside
            // a bracket: f(0) >= 0, and f <= 0 at Tm + sum coef J* (eps >= 0), up to
            // rounding, which the step-size stop below absorbs
            const double Thi = fmax(fmax(Tm + F0, Tm), 1e-300);
            Tc = fmax(Tm, 1e-300);
            double f, df;
            eval(Tc, f, df);
            double lo = f > 0.0 ? Tc : 0.0, hi = f > 0.0 ? fmax(Thi, Tc) : Tc;
            for (int it = 0; it < 100 && f != 0.0; ++it) {
                if (f > 0.0) lo = fmax(lo, Tc); else hi = fmin(hi, Tc);
                const double step = f / df;
                // a Newton step below 1e-14 of T is at the level of the rounding in
                // f: take it and stop (testing it against the bracket instead would
                // turn rounding noise into a bisection step)
                if (fabs(step) <= 1e-14 * Tc) {
                    Tc -= step;
                    break;
                }
                double Tn = Tc - step;
                if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
                Tc = Tn;
                eval(Tc, f, df);
                if (hi - lo <= 1e-15 * hi) break;
            }
        }
        // emission at T+: the last evaluation moved to T+ to first order
        // (|T+ - Te| <= 1e-14 T+, so the neglected term is ~1e-28 relative)
        for (int gg = gl; gg < G; gg += Gp) {
            const long long k = cell * G + gg;
            double e;
            if (ca.coupled) {
                e = one ? e1 + de1 * (Tc - Te) : group_emission_1(ca.edges[gg], ca.edges[gg + 1], Tc, nullptr);
                ca.eps[k] = e;
            } else {
                e = rd.eps[k];
            }
            const double ka = row_kappa(g, rd, k);
            double v = cdt * ka * e;
            if (rd.kscat) {
                const double jsk = one ? js1 : ca.Js[k];
                const double jn = (jsk + cdt * ka * e) / (1.0 + cdt * ka);
                ca.jn[k] = jn;
                v += cdt * rd.kscat[k] * jn;
            }
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
    const int Gp = couple_seg(G), cpw = 64 / Gp, seg = lane / Gp, gl = lane - seg * Gp;
    const long long ncell = g.M / G;
    const double coefT = 4.0 * M_PI / (ca.c * ca.heat_capacity);
    for (long long c0 = ((long long)blockIdx.x * 4 + w) * cpw; c0 < ncell; c0 += (long long)gridDim.x * 4 * cpw) {
        const long long cell = c0 + seg;
        if (cell >= ncell) continue;
        double diff = 0.0;
        for (int gg = gl; gg < G; gg += Gp) {
            const long long k = cell * G + gg;
            diff += ca.Js[k] - row_dot(Z + k * ldz, v, r1);
        }
        diff = seg_sum(diff, Gp);
        if (gl == 0) ca.T[cell] += coefT * diff;
    }
}

}  // namespace ttrt
