// Group emission coefficients eps_g(T) (Section 2, group emission), host FP64.
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
#include <cmath>
#include <limits>

namespace ttrt {

namespace {

constexpr double XS = 1.5;

// c_j = B_{2j} / (2j)! for j = 1..14 from the Bernoulli numbers
// B_2 .. B_28 (exact rationals), divided by (2j)! in double precision.
struct BernoulliTable {
    double c[15];
    BernoulliTable() {
        static const double num[15] = {0.0, 1.0, -1.0, 1.0, -1.0, 5.0, -691.0, 7.0, -3617.0, 43867.0,
                                       -174611.0, 854513.0, -236364091.0, 8553103.0, -23749461029.0};
        static const double den[15] = {1.0, 6.0, 30.0, 42.0, 30.0, 66.0, 2730.0, 6.0, 510.0, 798.0,
                                       330.0, 138.0, 2730.0, 6.0, 870.0};
        double fact = 1.0;  // (2j)!
        c[0] = 0.0;
        for (int j = 1; j <= 14; ++j) {
            fact *= (double)(2 * j - 1) * (double)(2 * j);
            c[j] = (num[j] / den[j]) / fact;
        }
    }
};

const BernoulliTable& bern() {
    static BernoulliTable t;
    return t;
}

// int_0^x t^3/(e^t-1) dt for 0 <= x <= XS
double low_part(double x) {
    if (x <= 0.0) return 0.0;
    const BernoulliTable& b = bern();
    const double x2 = x * x;
    double sum = x2 * x / 3.0 - x2 * x2 / 8.0;
    double p = x2 * x;  // x^{2j+3} built incrementally
    for (int j = 1; j <= 14; ++j) {
        p *= x2;
        double term = b.c[j] * p / (2 * j + 3);
        sum += term;
        if (std::fabs(term) < 1e-18 * std::fabs(sum)) break;
    }
    return sum;
}

// int_x^inf t^3/(e^t-1) dt for x >= XS
double tail_part(double x) {
    if (std::isinf(x)) return 0.0;
    double sum = 0.0;
    const double q = std::exp(-x);
    double ek = 1.0;
    for (int k = 1; k <= 200; ++k) {
        ek *= q;
        const double kk = (double)k;
        const double term = ek * (x * x * x / kk + 3.0 * x * x / (kk * kk) + 6.0 * x / (kk * kk * kk) +
                                  6.0 / (kk * kk * kk * kk));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

}  // namespace

// int_a^b t^3/(e^t-1) dt, 0 <= a < b <= inf
double bose3_integral(double a, double b) {
    if (!(b > a)) return 0.0;
    if (a >= XS) return tail_part(a) - tail_part(b);
    if (b <= XS) return low_part(b) - low_part(a);
    return (low_part(XS) - low_part(a)) + (tail_part(XS) - tail_part(b));
}

void group_emission(const double* edges, int n_groups, double T, double* out) {
    for (int g = 0; g < n_groups; ++g) {
        if (!(T > 0.0)) {
            out[g] = 0.0;
            continue;
        }
        const double a = edges[g] / T;
        const double b = std::isinf(edges[g + 1]) ? std::numeric_limits<double>::infinity()
                                                  : edges[g + 1] / T;
        out[g] = 2.0 * T * T * T * T * bose3_integral(a, b);
    }
}

}  // namespace ttrt
