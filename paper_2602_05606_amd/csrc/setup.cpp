// setup.cpp -- host-side per-species setup of the approximate Kappa generator
// (Zenitani & Umeda, arXiv 2602.05606): the first four rows of Table 1, which
// the paper computes once per species, in FP64.
#include <cmath>

#include "kappa_internal.hpp"
#include "kappa_params.hpp"

namespace kappa {

// Digamma: shift the argument up with psi(x) = psi(x + 1) - 1/x until x >= 10,
// then the asymptotic expansion psi(x) = ln x - 1/(2x) - sum_k B_2k / (2k x^2k)
// (Abramowitz & Stegun 6.3.5, 6.3.18), truncated after B_14.
double digamma(double x)
{
    double acc = 0.0;
    for (; x < 10.0; x += 1.0) acc -= 1.0 / x;
    const double r = 1.0 / (x * x);
    // B_2k / (2k) for k = 1..7
    const double t = r * (1.0 / 12 + r * (-1.0 / 120 + r * (1.0 / 252 + r * (-1.0 / 240 + r * (1.0 / 132 +
                     r * (-691.0 / 32760 + r * (1.0 / 12)))))));
    return acc + std::log(x) - 0.5 / x - t;
}

Setup make_setup(double kappa)
{
    Setup s{};
    s.kappa = kappa;
    if (std::isinf(kappa)) {
        // Maxwell limit: exp_q* -> exp, ln_q* -> ln; a and b/c at their kappa -> inf
        // limits (Sec. 3); c minimises the relative entropy against the Maxwell density.
        s.kstar = kappa;
        s.lnbeta = -kappa;
        s.a = std::pow(4.0 / (3.0 * std::sqrt(M_PI)), 2.0 / 3.0);
        s.c = kMaxwellC;
        s.b_over_c = 1.0;
        s.b = s.c;
        return s;  // derivatives stay 0: kappa = inf is not differentiated
    }
    // kappa* = kappa - 1/2 (eq:k2)
    s.kstar = kappa - 0.5;
    // ln B(3/2, kappa*) with B(x, y) = Gamma(x) Gamma(y) / Gamma(x + y) (Sec. 6)
    s.lnbeta = std::lgamma(1.5) + std::lgamma(s.kstar) - std::lgamma(kappa + 1.0);
    // a = (1/kappa) (2 / (3B))^{2/3} (eq:a), in logs
    s.a = std::exp((2.0 / 3.0) * (std::log(2.0 / 3.0) - s.lnbeta) - std::log(kappa));
    // c = (0.123 k^2 - 1.12 k + 2.56) / (k^2 - 7.89 k + 15.6) (eq:c)
    const double num = (0.123 * kappa - 1.12) * kappa + 2.56;
    const double den = (kappa - 7.89) * kappa + 15.6;
    s.c = num / den;
    // b/c = {kappa* (3/2) B}^{1/kappa*} kappa*/kappa (eq:b), b = (b/c) c
    const double ln_q = std::log(1.5 * s.kstar) + s.lnbeta;
    s.b_over_c = std::exp(ln_q / s.kstar + std::log(s.kstar) - std::log(kappa));
    s.b = s.b_over_c * s.c;

    // Derivatives.  d ln B / d kappa = psi(kappa*) - psi(kappa + 1).
    const double dlnbeta = digamma(s.kstar) - digamma(kappa + 1.0);
    s.da = s.a * ((-2.0 / 3.0) * dlnbeta - 1.0 / kappa);
    const double dnum = 0.246 * kappa - 1.12;
    const double dden = 2.0 * kappa - 7.89;
    s.dc = (dnum * den - num * dden) / (den * den);
    // d ln(b/c) / d kappa = -ln_q / kappa*^2 + (1/kappa* + dlnB) / kappa* + 1/kappa* - 1/kappa
    const double dln_ratio = -ln_q / (s.kstar * s.kstar) + (1.0 / s.kstar + dlnbeta) / s.kstar + 1.0 / s.kstar -
                             1.0 / kappa;
    s.db = s.b * dln_ratio + s.b_over_c * s.dc;
    return s;
}

// The kernels evaluate L = -kappa* expm1(-lT / kappa*).  For kappa = inf they
// get kappa* = 2^60: then L = lT (1 + O(|lT| 2^-61)), lT within (-38, 0), which
// is lT to below half an ulp in FP64 and FP32, with no special case on the GPU.
static double kernel_kstar(const Setup &s) { return std::isinf(s.kstar) ? 0x1p60 : s.kstar; }

SpeciesF64 species_f64(const Setup &s, double theta)
{
    SpeciesF64 p{};
    p.kstar = kernel_kstar(s);
    p.inv_kstar = 1.0 / p.kstar;
    p.a = s.a;
    p.b = s.b;
    p.c = s.c;
    p.two_b = 2.0 * s.b;
    p.neg_four_b = -4.0 * s.b;
    p.theta = theta;
    p.da = s.da;
    p.db = s.db;
    p.dc = s.dc;
    return p;
}

SpeciesF32 species_f32(const Setup &s, double theta)
{
    SpeciesF32 p{};
    const double ks = kernel_kstar(s);
    p.kstar = static_cast<float>(ks);
    p.inv_kstar = static_cast<float>(1.0 / ks);
    p.a = static_cast<float>(s.a);
    p.b = static_cast<float>(s.b);
    p.c = static_cast<float>(s.c);
    p.half_inv_b = static_cast<float>(0.5 / s.b);
    p.theta = static_cast<float>(theta);
    p.two_b = static_cast<float>(2.0 * s.b);
    p.two_kstar = static_cast<float>(2.0 * ks);
    p.neg_c_kstar = static_cast<float>(-s.c * ks);
    p.four_b_kstar = static_cast<float>(4.0 * s.b * ks);
    p.da = static_cast<float>(s.da);
    p.db = static_cast<float>(s.db);
    p.dc = static_cast<float>(s.dc);
    return p;
}

}  // namespace kappa
