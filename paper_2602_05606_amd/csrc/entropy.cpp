// entropy.cpp -- the Monte Carlo relative entropy of the paper's second test
// (Sec. 5, eq:KL) from a speed histogram: exact bin probabilities of the Kappa
// distribution and the sum of eq:KL, on the host (the nbins + 1 counts come
// from kappa_speed_histogram on the GPU).
//
// The speed CDF in x = (v/theta)^2 is the regularized incomplete beta
// function F(x) = I_{x/(x+kappa)}(3/2, kappa - 1/2) (eq:CDF; its derivative
// is eq:kappax), and for kappa = inf (the Maxwell limit) the regularized
// incomplete gamma function P(3/2, x).  Both are evaluated with the textbook
// methods (DLMF 8.17(v) for the beta function: its continued fraction,
// evaluated by the modified Lentz algorithm, with the symmetry
// I_x(a, b) = 1 - I_{1-x}(b, a) beyond the fraction's fast-converging range;
// DLMF 8.7 and 8.9 for the gamma function: the series of P below x = a + 1,
// the continued fraction of Q = 1 - P above), each to about 1e-15 relative.
#include <cmath>
#include <cstdint>
#include <limits>

#include "kappa_internal.hpp"

namespace kappa {

namespace {

constexpr double kTiny = 1e-300;
constexpr double kEps = 1e-16;
constexpr int kMaxIter = 10000;

// Continued fraction of I_x(a, b) x^-a (1-x)^-b a B(a, b) (DLMF 8.17.22),
// modified Lentz; fast for x < (a + 1) / (a + b + 2).
double beta_cf(double a, double b, double x)
{
    double c = 1.0;
    double d = 1.0 - (a + b) * x / (a + 1.0);
    if (std::fabs(d) < kTiny) d = kTiny;
    d = 1.0 / d;
    double h = d;
    for (int m = 1; m <= kMaxIter; ++m) {
        // even step: d_{2m} = m (b - m) x / ((a + 2m - 1)(a + 2m))
        double num = m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
        d = 1.0 + num * d;
        if (std::fabs(d) < kTiny) d = kTiny;
        c = 1.0 + num / c;
        if (std::fabs(c) < kTiny) c = kTiny;
        d = 1.0 / d;
        h *= d * c;
        // odd step: d_{2m+1} = -(a + m)(a + b + m) x / ((a + 2m)(a + 2m + 1))
        num = -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0));
        d = 1.0 + num * d;
        if (std::fabs(d) < kTiny) d = kTiny;
        c = 1.0 + num / c;
        if (std::fabs(c) < kTiny) c = kTiny;
        d = 1.0 / d;
        const double delta = d * c;
        h *= delta;
        if (std::fabs(delta - 1.0) < kEps) break;
    }
    return h;
}

// I_x(a, b) and 1 - I_x(a, b), each computed directly (no cancellation).
void incomplete_beta(double a, double b, double x, double &ix, double &one_minus)
{
    if (x <= 0.0) {
        ix = 0.0;
        one_minus = 1.0;
        return;
    }
    if (x >= 1.0) {
        ix = 1.0;
        one_minus = 0.0;
        return;
    }
    const double lbeta = std::lgamma(a) + std::lgamma(b) - std::lgamma(a + b);
    const double front = std::exp(a * std::log(x) + b * std::log1p(-x) - lbeta);
    if (x < (a + 1.0) / (a + b + 2.0)) {
        ix = front * beta_cf(a, b, x) / a;
        one_minus = 1.0 - ix;
        if (ix > 0.5) one_minus = front * beta_cf(b, a, 1.0 - x) / b;  // the other side is then in range
    } else {
        one_minus = front * beta_cf(b, a, 1.0 - x) / b;
        ix = 1.0 - one_minus;
    }
}

// P(a, x) and Q(a, x) = 1 - P(a, x), the regularized incomplete gamma functions.
void incomplete_gamma(double a, double x, double &p, double &q)
{
    if (x <= 0.0) {
        p = 0.0;
        q = 1.0;
        return;
    }
    const double front = std::exp(a * std::log(x) - x - std::lgamma(a));
    if (x < a + 1.0) {
        // P = x^a e^-x / Gamma(a + 1) sum_n x^n / ((a + 1)...(a + n))  (DLMF 8.7.1)
        double term = 1.0 / a, sum = term;
        for (int n = 1; n <= kMaxIter; ++n) {
            term *= x / (a + n);
            sum += term;
            if (std::fabs(term) < std::fabs(sum) * kEps) break;
        }
        p = front * sum;
        q = 1.0 - p;
    } else {
        // Q by its continued fraction (DLMF 8.9.2), modified Lentz
        double b = x + 1.0 - a, c = 1.0 / kTiny, d = 1.0 / b, h = d;
        for (int n = 1; n <= kMaxIter; ++n) {
            const double an = -n * (n - a);
            b += 2.0;
            d = an * d + b;
            if (std::fabs(d) < kTiny) d = kTiny;
            c = b + an / c;
            if (std::fabs(c) < kTiny) c = kTiny;
            d = 1.0 / d;
            const double delta = d * c;
            h *= delta;
            if (std::fabs(delta - 1.0) < kEps) break;
        }
        q = front * h;
        p = 1.0 - q;
    }
}

}  // namespace

void speed_cdf(double kappa, double x, double &F, double &one_minus_F)
{
    if (std::isinf(kappa)) {
        incomplete_gamma(1.5, x, F, one_minus_F);
        return;
    }
    // x / (x + kappa) and kappa / (x + kappa) both exact to rounding: the two tails
    incomplete_beta(1.5, kappa - 0.5, x / (x + kappa), F, one_minus_F);
}

}  // namespace kappa

using namespace kappa;

extern "C" kappa_status kappa_relative_entropy(double kappa, const uint64_t *counts, uint32_t nbins, double bin_width,
                                               double eps, double *D, double *prob)
{
    if (!(kappa > 1.5) || std::isnan(kappa)) return fail(KAPPA_EINVAL, "kappa must be > 3/2 or +inf (got %g)", kappa);
    if (!counts || !D) return fail(KAPPA_EINVAL, "null counts or D pointer");
    if (nbins < 1 || nbins > 2047) return fail(KAPPA_ERANGE, "nbins must be in [1, 2047] (got %u)", nbins);
    if (!(bin_width > 0.0) || !std::isfinite(bin_width)) return fail(KAPPA_EINVAL, "bin_width must be positive");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(KAPPA_EINVAL, "eps must be finite and >= 0");
    double total = 0.0;
    for (uint32_t i = 0; i <= nbins; ++i) total += static_cast<double>(counts[i]);
    if (!(total > 0.0)) return fail(KAPPA_EINVAL, "the histogram is empty");
    double sum = 0.0, F_prev = 0.0, R_prev = 1.0;  // F and 1 - F at the previous edge
    for (uint32_t i = 0; i <= nbins; ++i) {
        double p;
        if (i < nbins) {
            const double e = (i + 1) * bin_width;
            double F, R;
            speed_cdf(kappa, e * e, F, R);
            // the bin's probability from the side that does not cancel
            p = F < 0.5 ? F - F_prev : R_prev - R;
            F_prev = F;
            R_prev = R;
        } else {
            p = R_prev;  // the open last bin: 1 - F at the last edge
        }
        if (prob) prob[i] = p;
        const double q = static_cast<double>(counts[i]) / total;
        sum += (p + eps) * std::log((p + eps) / (q + eps));
    }
    *D = sum;
    return KAPPA_OK;
}
