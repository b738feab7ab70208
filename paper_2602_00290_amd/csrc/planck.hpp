// Group emission coefficients eps_g(T) and their temperature derivative
// (Section 2, group emission), FP64, for host setup and device kernels.
//
// eps_g(T) = 2 T^4 * int_{nu_{g-1}/T}^{nu_g/T} t^3/(e^t - 1) dt   (h = k = c_light = 1)
//
// The incomplete Bose integral is evaluated with two convergent series, a
// method of this library's own (the paper uses polylogarithm routines):
//   * x <= XS:  int_0^x t^3/(e^t-1) dt = x^3/3 - x^4/8 + sum_{j>=1} B_{2j} x^{2j+3} / ((2j+3)(2j)!)
//               (the generating function t/(e^t-1) = sum B_n t^n / n!, radius 2 pi);
//   * x >  XS:  int_x^inf t^3/(e^t-1) dt = sum_{k>=1} e^{-kx} (x^3/k + 3x^2/k^2 + 6x/k^3 + 6/k^4)
//               (expanding 1/(e^t-1) = sum_k e^{-kt} and integrating term by term).
// A group [a, b) is formed as low(b) - low(a), tail(a) - tail(b), or a mix
// across XS, which avoids subtracting from the total pi^4/15.
//
// With a = nu_{g-1}/T and b = nu_g/T,
//   d eps_g / dT = 8 T^3 int_a^b t^3/(e^t-1) dt + 2 T^3 (a^4/(e^a-1) - b^4/(e^b-1)),
// since d a / dT = -a / T (and the same for b).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace ttrt {

constexpr double kPlanckXS = 1.5;

constexpr int kPlanckTailTerms = 200;

// Compile-time coefficient tables (no division is left for run time):
//   c[j] = B_{2j} / ((2j)! (2j + 3)) for j = 1..14 (Bernoulli numbers B_2 .. B_28
//   as exact rationals), and inv[k] = 1 / k for the tail series.
struct PlanckSeries {
    double c[15];
    double inv[kPlanckTailTerms + 1];
    constexpr PlanckSeries() : c{}, inv{} {
        const double num[15] = {0.0, 1.0, -1.0, 1.0, -1.0, 5.0, -691.0, 7.0, -3617.0, 43867.0,
                                -174611.0, 854513.0, -236364091.0, 8553103.0, -23749461029.0};
        const double den[15] = {1.0, 6.0, 30.0, 42.0, 30.0, 66.0, 2730.0, 6.0, 510.0, 798.0,
                                330.0, 138.0, 2730.0, 6.0, 870.0};
        double fact = 1.0;   // (2j)!
        for (int j = 1; j <= 14; ++j) {
            fact *= (double)(2 * j - 1) * (double)(2 * j);
            c[j] = (num[j] / den[j]) / fact / (double)(2 * j + 3);
        }
        for (int k = 1; k <= kPlanckTailTerms; ++k) inv[k] = 1.0 / (double)k;
    }
};
constexpr PlanckSeries kPlanckSeries{};

__host__ __device__ inline double planck_low(double x) {   // int_0^x t^3/(e^t-1) dt, 0 <= x <= XS
    const PlanckSeries& S = kPlanckSeries;
    if (x <= 0.0) return 0.0;
    const double x2 = x * x;
    double sum = x2 * x * (1.0 / 3.0) - x2 * x2 * 0.125;
    double p = x2 * x;   // x^{2j+3} built incrementally
    for (int j = 1; j <= 14; ++j) {
        p *= x2;
        const double term = S.c[j] * p;
        sum += term;
        if (fabs(term) < 1e-18 * fabs(sum)) break;
    }
    return sum;
}

__host__ __device__ inline double planck_tail(double x) {  // int_x^inf t^3/(e^t-1) dt, x >= XS
    if (__builtin_isinf(x)) return 0.0;
    const PlanckSeries& S = kPlanckSeries;
    double sum = 0.0;
    const double q = exp(-x);
    const double x2 = x * x, x3 = x2 * x;
    double ek = 1.0;
    for (int k = 1; k <= kPlanckTailTerms; ++k) {
        ek *= q;
        const double ik = S.inv[k];
        // e^{-kx} (x^3/k + 3x^2/k^2 + 6x/k^3 + 6/k^4), Horner in 1/k
        const double term = ek * ik * (x3 + ik * (3.0 * x2 + ik * (6.0 * x + 6.0 * ik)));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

// int_a^b t^3/(e^t-1) dt, 0 <= a < b <= inf
__host__ __device__ inline double bose3_integral(double a, double b) {
    if (!(b > a)) return 0.0;
    if (a >= kPlanckXS) return planck_tail(a) - planck_tail(b);
    if (b <= kPlanckXS) return planck_low(b) - planck_low(a);
    return (planck_low(kPlanckXS) - planck_low(a)) + (planck_tail(kPlanckXS) - planck_tail(b));
}

// x^4 / (e^x - 1), zero at x = 0 and x = inf
__host__ __device__ inline double planck_x4(double x) {
    if (!(x > 0.0) || __builtin_isinf(x)) return 0.0;
    return x * x * x * x * exp(-x) / -expm1(-x);
}

// eps of the group [nu_lo, nu_hi) at T and, if deps is non-null, d eps / dT
__host__ __device__ inline double group_emission_1(double nu_lo, double nu_hi, double T, double* deps) {
    if (!(T > 0.0)) {
        if (deps) *deps = 0.0;
        return 0.0;
    }
    const double a = nu_lo / T;
    const double b = __builtin_isinf(nu_hi) ? INFINITY : nu_hi / T;
    const double I = bose3_integral(a, b);
    const double T3 = T * T * T;
    if (deps) *deps = 8.0 * T3 * I + 2.0 * T3 * (planck_x4(a) - planck_x4(b));
    return 2.0 * T3 * T * I;
}

inline void group_emission(const double* edges, int n_groups, double T, double* out) {
    for (int g = 0; g < n_groups; ++g) out[g] = group_emission_1(edges[g], edges[g + 1], T, nullptr);
}

}  // namespace ttrt
