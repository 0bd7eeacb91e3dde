// kappa_params.hpp -- per-species parameter blocks passed to the kernels, and
// the host-side setup of Table 1 (rows 1-4) that fills them.
#pragma once

#include <stdint.h>

namespace kappa {

// Setup of one species in FP64 (Table 1, first four rows; eq:k2, eq:a, eq:c,
// eq:b), plus the kappa-derivatives used by the backward pass.
struct Setup {
    double kappa, kstar, a, b, c, b_over_c, da, db, dc, lnbeta;
};

// Host: computes the setup block.  Requires kappa > 3/2 and finite.
Setup make_setup(double kappa);

// Digamma on the host (recurrence + asymptotic series); used for the
// kappa-derivative of ln B(3/2, kappa*).
double digamma(double x);

// Kernel-side copies, FP64 and FP32.
struct SpeciesF64 {
    double kstar, inv_kstar, a, b, c;
    double two_b, neg_four_b;  // 2b, -4b
    double theta;
    double da, db, dc;  // kappa-derivatives (backward only)
};

struct SpeciesF32 {
    float kstar, inv_kstar, a, b, c, half_inv_b, theta;
    float two_b, two_kstar, neg_c_kstar, four_b_kstar;  // 2b, 2 kappa*, -c kappa*, 4b kappa*
    float da, db, dc;
};

SpeciesF64 species_f64(const Setup &s, double theta);
SpeciesF32 species_f32(const Setup &s, double theta);

}  // namespace kappa
