/*
 * kappa_oracle.c -- FP64 CPU oracle of the approximate Kappa velocity sampler
 * of Zenitani & Umeda, "An approximate Kappa generator for particle
 * simulations" (arXiv 2602.05606).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code with the HIP library: its Philox, uniform maps, parameter
 * setup, digamma and inversion are written here from the published
 * definitions, and nothing here is used by the product path.
 *
 * Citations name the paper's sections, its LaTeX equation labels (eq:...)
 * and Table 1 (label table:kappa).
 *
 * Everything is FP64 and uses the C library's log, log1p, exp, expm1, sqrt,
 * sin and cos.  Compile with -O2 -ffp-contract=off and without fast-math.
 *
 * Parity pins: every function here is pinned by a CPU test (limits of a and
 * b/c, asymptotic matching against the exact Beta-prime CDF, the G round
 * trip, the KS test against the exact CDF, the paper's statements on the
 * relative entropy and the energy error, finite differences of the adjoint,
 * and Philox against an independent library implementation).  None is
 * "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition: Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11.  Ten rounds; each
 * round multiplies counter words 0 and 2 by two fixed 32-bit multipliers,
 * and the key is advanced by the two Weyl constants between rounds.        */
/* ------------------------------------------------------------------------ */

#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t prod_a = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t y0 = hi_b ^ x1 ^ k0;
        uint32_t y1 = lo_b;
        uint32_t y2 = hi_a ^ x3 ^ k1;
        uint32_t y3 = lo_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The block drawn for particle i of segment seg, draw d:
 * counter = (low word of i, high word of i, seg, d), key = (low, high word of seed). */
static void particle_block(uint64_t seed, uint64_t i, uint32_t seg, uint32_t draw, uint32_t r[4])
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), seg, draw};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, r);
}

void oracle_philox_blocks(uint64_t n, uint64_t seed, uint64_t counter_offset, uint32_t seg,
                          uint32_t draw, uint32_t *out)
{
    for (uint64_t j = 0; j < n; ++j)
        particle_block(seed, counter_offset + j, seg, draw, out + 4 * j);
}

/* ------------------------------------------------------------------------ */
/* Digamma, needed only for the derivative of the setup parameters with
 * respect to kappa.  Recurrence psi(x) = psi(x+1) - 1/x up to x >= 12, then
 * the standard asymptotic series psi(x) ~ ln x - 1/(2x) - sum B_2k/(2k x^2k)
 * (Abramowitz & Stegun 6.3.5 and 6.3.18).                                  */
/* ------------------------------------------------------------------------ */
double oracle_digamma(double x)
{
    double shift = 0.0;
    while (x < 12.0) {
        shift -= 1.0 / x;
        x += 1.0;
    }
    double inv = 1.0 / x, inv2 = inv * inv;
    /* Bernoulli numbers B2..B12 divided by 2k */
    double series = inv2 * (1.0 / 12.0 - inv2 * (1.0 / 120.0 - inv2 * (1.0 / 252.0 -
                    inv2 * (1.0 / 240.0 - inv2 * (1.0 / 132.0 - inv2 * (691.0 / 32760.0))))));
    return shift + log(x) - 0.5 * inv - series;
}

/* ------------------------------------------------------------------------ */
/* Per-species setup (Table 1, first four rows, "required only once").      */
/*   kappa* = kappa - 1/2                                      (eq:k2)      */
/*   a = (1/kappa) * (2 / (3 B(3/2, kappa*)))^(2/3)            (eq:a)       */
/*   c = (0.123 k^2 - 1.12 k + 2.56) / (k^2 - 7.89 k + 15.6)   (eq:c)       */
/*   b = {kappa* (3/2) B(3/2, kappa*)}^(1/kappa*) (kappa* / kappa) c  (eq:b)  */
/* with B(x, y) = Gamma(x) Gamma(y) / Gamma(x + y) (Sec. 6).                */
/* Also the kappa-derivatives of a, b, c used by the adjoint.               */
/* ------------------------------------------------------------------------ */

enum {
    OP_KSTAR = 0, OP_A, OP_B, OP_C, OP_B_OVER_C, OP_DA, OP_DB, OP_DC, OP_LNBETA, OP_COUNT
};

/* The Maxwell limit, kappa = +inf (a variant on the same construction; the
 * paper gives no constants for it): q* -> 1, so exp_q* -> exp in eq:G and
 * the q-logarithm of eq:L -> ln; a and b/c take the limits Sec. 3 states,
 * a = (4 / (3 sqrt(pi)))^(2/3) and b/c = 1; c is the value that minimises
 * the relative entropy of eq:relative_entropy with the Maxwell density
 * 2/sqrt(pi) x^(1/2) e^-x in place of eq:kappax (0.078998 by a 30-digit
 * quadrature), rounded to three figures as eq:c's constants are. */
#define ORACLE_C_MAXWELL 0.079

void oracle_params(double kappa, double *p)
{
    if (isinf(kappa) && kappa > 0) {
        p[OP_KSTAR] = INFINITY;
        p[OP_A] = pow(4.0 / (3.0 * sqrt(M_PI)), 2.0 / 3.0);
        p[OP_C] = ORACLE_C_MAXWELL;
        p[OP_B_OVER_C] = 1.0;
        p[OP_B] = ORACLE_C_MAXWELL;
        p[OP_DA] = p[OP_DB] = p[OP_DC] = 0.0;
        p[OP_LNBETA] = -INFINITY;
        return;
    }
    double ks = kappa - 0.5;
    double lnB = lgamma(1.5) + lgamma(ks) - lgamma(kappa + 1.0);
    double a = (1.0 / kappa) * pow(2.0 / (3.0 * exp(lnB)), 2.0 / 3.0);
    double cn = 0.123 * kappa * kappa - 1.12 * kappa + 2.56;
    double cd = kappa * kappa - 7.89 * kappa + 15.6;
    double c = cn / cd;
    double ln_inner = log(ks * 1.5) + lnB; /* ln{kappa* (3/2) B} */
    double b_over_c = exp(ln_inner / ks) * ks / kappa;
    double b = b_over_c * c;

    /* d lnB / d kappa = psi(kappa*) - psi(kappa + 1) */
    double dlnB = oracle_digamma(ks) - oracle_digamma(kappa + 1.0);
    double da = a * (-1.0 / kappa - (2.0 / 3.0) * dlnB);
    double dcn = 0.246 * kappa - 1.12, dcd = 2.0 * kappa - 7.89;
    double dc = (dcn * cd - cn * dcd) / (cd * cd);
    double dln_boc = -ln_inner / (ks * ks) + (1.0 / ks) * (1.0 / ks + dlnB) + 1.0 / ks - 1.0 / kappa;
    double db = b * dln_boc + b_over_c * dc;

    p[OP_KSTAR] = ks;
    p[OP_A] = a;
    p[OP_B] = b;
    p[OP_C] = c;
    p[OP_B_OVER_C] = b_over_c;
    p[OP_DA] = da;
    p[OP_DB] = db;
    p[OP_DC] = dc;
    p[OP_LNBETA] = lnB;
}

/* ------------------------------------------------------------------------ */
/* Uniform maps.  The paper draws U1, U2, U3 ~ Uniform(0,1) (Table 1) and
 * warns against a zero uniform (Sec. 6).  Reading used here: open midpoint
 * dyadics, with U1 carried as (side, small value) so that both U1 and 1-U1
 * are exact, and the same uniforms in every precision mode:
 *   m = top 53 bits of (r0:r3).  m < 2^52: U1 = (2m+1) 2^-54 on the low
 *   side; else W1 = 1 - U1 = (2^54-2m-1) 2^-54.  U2 = (r1 + 1/2) 2^-32,
 *   U3 = (r2 + 1/2) 2^-32.
 * The modes differ only in the arithmetic the GPU uses (the oracle always
 * computes in FP64): mode 0 FP64; mode 1 FP32 with an FP64 inversion when
 * W1 < 2^-20 (r0 >= 0xFFFFF000, probability exactly 2^-20), reported as
 * "tail"; mode 2 FP32 throughout (diagnostics).                            */
/* ------------------------------------------------------------------------ */

enum { SIDE_LOW = 0, SIDE_HIGH = 1 };
enum { MODE_FP64 = 0, MODE_FP32 = 1, MODE_FP32_NOTAIL = 2 };

/* Returns 1 when mode 1 takes the FP64 tail inversion for this particle. */
int oracle_speed_uniform(int mode, uint32_t r0, uint32_t r3, int *side, double *u)
{
    uint64_t m53 = ((((uint64_t)r0) << 32) | (uint64_t)r3) >> 11;
    if (m53 < (1ull << 52)) {
        *side = SIDE_LOW;
        *u = ldexp((double)(2 * m53 + 1), -54);
    } else {
        *side = SIDE_HIGH;
        *u = ldexp((double)((1ull << 54) - 2 * m53 - 1), -54);
    }
    return mode == MODE_FP32 && r0 >= 0xFFFFF000u;
}

/* cos(theta) = 2 U2 - 1 and U2 (1 - U2), both from the integer word. */
static void polar_uniform(uint32_t r1, double *cos_t, double *u2_1mu2)
{
    double lo = (double)r1 + 0.5;                /* U2 * 2^32 */
    double hi = 4294967296.0 - (double)r1 - 0.5; /* (1 - U2) * 2^32 */
    *cos_t = ldexp((double)(2 * (int64_t)r1 + 1 - 4294967296LL), -32);
    *u2_1mu2 = ldexp(lo * hi, -64);
}

static double azimuth_uniform(uint32_t r2)
{
    return ldexp((double)r2 + 0.5, -32);
}

/* ------------------------------------------------------------------------ */
/* Inversion of G (Sec. 4).  Solving G(x) = U1 (eq:GU) with the q-logarithm
 * (eq:qlog) gives
 *   L = ln_{q*}(1 - U1^(2/3)) = -kappa* {(1 - U1^(2/3))^(-1/kappa*) - 1}  (eq:L)
 *   x = (V/theta)^2 = root of b x^2 + (a + cL) x + L = 0                   (eq:v)
 * Written with lT = ln(1 - U1^(2/3)) so that no step subtracts nearly equal
 * numbers:
 *   low side : lT = log1p(-exp((2/3) ln U1))
 *   high side: lT = ln(-expm1((2/3) log1p(-W1)))
 *   L = -kappa* expm1(-lT / kappa*)
 * and the two printed forms of the root (eq:v) chosen by the sign of
 * A = a + cL:  x = -2L / (A + D) if A >= 0, else (D - A) / (2b), with
 * D = sqrt(A^2 - 4bL).                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lT, z, L, A, D, x;
} inversion;

static void invert(const double *p, int side, double u, inversion *r)
{
    double ks = p[OP_KSTAR], a = p[OP_A], b = p[OP_B], c = p[OP_C];
    double lT;
    if (side == SIDE_LOW) {
        double t = exp((2.0 / 3.0) * log(u)); /* U1^(2/3) */
        lT = log1p(-t);
    } else {
        double lnU1 = log1p(-u);               /* ln(1 - W1) = ln U1 */
        lT = log(-expm1((2.0 / 3.0) * lnU1));  /* ln(1 - U1^(2/3)) */
    }
    double z = -lT / ks;
    double L = isinf(ks) ? lT : -ks * expm1(z);  /* ln_q -> ln as q* -> 1 */
    double A = a + c * L;
    double D = sqrt(A * A - 4.0 * b * L);
    double x = (A >= 0.0) ? (-2.0 * L) / (A + D) : (D - A) / (2.0 * b);
    r->lT = lT; r->z = z; r->L = L; r->A = A; r->D = D; r->x = x;
}

/* Speed V / theta at a given (side, small uniform). */
double oracle_speed(double kappa, int side, double u)
{
    double p[OP_COUNT];
    inversion r;
    oracle_params(kappa, p);
    invert(p, side, u, &r);
    return sqrt(r.x);
}

/* The approximate CDF G(x) of eq:G with exp_q from eq:qexp and q* = 1 + 1/kappa*:
 * exp_{q*}(-w) = (1 + w/kappa*)^(-kappa*), w = (a x + b x^2) / (1 + c x).
 * Returns G and 1 - G, each computed without cancellation. */
void oracle_G(double kappa, double x, double *G, double *one_minus_G)
{
    double p[OP_COUNT];
    oracle_params(kappa, p);
    double ks = p[OP_KSTAR], a = p[OP_A], b = p[OP_B], c = p[OP_C];
    double w = (a * x + b * x * x) / (1.0 + c * x);
    double ln_e = isinf(ks) ? -w : -ks * log1p(w / ks);  /* ln exp_{q*}(-w) */
    double inner = -expm1(ln_e);             /* 1 - exp_{q*}(-w) */
    *G = exp(1.5 * log(inner));
    *one_minus_G = -expm1(1.5 * log1p(-exp(ln_e)));
}

/* The approximate speed density g(x) of eq:approx_x. */
double oracle_g_pdf(double kappa, double x)
{
    double p[OP_COUNT];
    oracle_params(kappa, p);
    double ks = p[OP_KSTAR], a = p[OP_A], b = p[OP_B], c = p[OP_C];
    double pre = 3.0 * (a + 2.0 * b * x + b * c * x * x) / (2.0 * (1.0 + c * x) * (1.0 + c * x));
    if (isinf(ks)) {
        double w = (a * x + b * x * x) / (1.0 + c * x);
        return pre * sqrt(-expm1(-w)) * exp(-w);
    }
    double ratio = 1.0 + (a * x + b * x * x) / (ks * (1.0 + c * x));
    return pre * sqrt(1.0 - pow(ratio, -ks)) * pow(ratio, -(ks + 1.0));
}

/* ------------------------------------------------------------------------ */
/* One particle of Table 1: speed from U1, direction from U2 and U3:
 *   v_x = V (2U2 - 1), v_y = 2V sqrt(U2(1-U2)) cos(2 pi U3),
 *   v_z = 2V sqrt(U2(1-U2)) sin(2 pi U3), then the drift is added.        */
/* ------------------------------------------------------------------------ */

static int one_particle(const double *p, double theta, const double *drift, int mode,
                        const uint32_t r[4], double v[3])
{
    int side;
    double u;
    inversion inv;
    int tail = oracle_speed_uniform(mode, r[0], r[3], &side, &u);
    invert(p, side, u, &inv);
    double V = theta * sqrt(inv.x);
    double cos_t, u2prod;
    polar_uniform(r[1], &cos_t, &u2prod);
    double sin_t = 2.0 * sqrt(u2prod);
    double phi = 2.0 * M_PI * azimuth_uniform(r[2]);
    v[0] = V * cos_t + drift[0];
    v[1] = V * sin_t * cos(phi) + drift[1];
    v[2] = V * sin_t * sin(phi) + drift[2];
    return tail;
}

/* Samples particles counter_offset .. counter_offset + n - 1 of segment seg.
 * Returns the number of particles that took the FP64 tail (mode 1). */
uint64_t oracle_sample(double kappa, double theta, const double *drift, uint64_t n, uint64_t seed,
                       uint64_t counter_offset, uint32_t seg, int mode, double *vx, double *vy,
                       double *vz)
{
    double p[OP_COUNT];
    double zero[3] = {0.0, 0.0, 0.0};
    const double *d = drift ? drift : zero;
    uint64_t tails = 0;
    oracle_params(kappa, p);
#pragma omp parallel for schedule(static) reduction(+ : tails)
    for (int64_t j = 0; j < (int64_t)n; ++j) {
        uint32_t r[4];
        double v[3];
        particle_block(seed, counter_offset + (uint64_t)j, seg, 0, r);
        tails += (uint64_t)one_particle(p, theta, d, mode, r, v);
        vx[j] = v[0]; vy[j] = v[1]; vz[j] = v[2];
    }
    return tails;
}

/* Particle positions for fused particle loading (not in the paper, which
 * samples velocities only): particle i of a segment takes the Philox block
 * with counter (i, seg, draw 1) and sits at lo[k] + u_k size[k] on axis k,
 * where u_k is the open midpoint dyadic of word r_k (k = 0, 1, 2):
 * (r_k + 1/2) 2^-32 in FP64 mode and (floor(r_k / 2^9) + 1/2) 2^-23 in the
 * FP32 modes (24 significant bits: exact in float, below 1).  FP64
 * arithmetic.
 *
 * The box is half-open, [lo, lo + size).  u < 1, but lo + u size rounded to
 * the nearest double can still reach lo + size when |lo| is large against
 * size (lo = 1e8, size = 1, u = 1 - 2^-33), so the result is capped at the
 * largest double strictly below the real number lo + size.  A box of size 0
 * places every particle at lo. */

/* Largest double strictly below the real lo + size (size > 0), never below
 * lo: the rounded sum s and its exact rounding error (Knuth's two-sum) tell
 * whether s lies below the real sum (then s is the answer) or not (then the
 * double just below s is). */
static double box_upper(double lo, double size)
{
    if (!(size > 0.0)) return lo;
    const double s = lo + size;
    const double t = s - lo;
    const double err = (lo - (s - t)) + (size - t);
    const double hi = err > 0.0 ? s : nextafter(s, -INFINITY);
    return hi > lo ? hi : lo;
}

/* Coordinate of one axis from the Philox word r. */
double oracle_position_coord(double lo, double size, uint32_t r, int mode)
{
    const double u = mode == MODE_FP64 ? ldexp((double)r + 0.5, -32) : ldexp((double)(r >> 9) + 0.5, -23);
    const double p = lo + u * size;
    const double hi = box_upper(lo, size);
    return p < hi ? p : hi;
}

void oracle_positions(const double *lo, const double *size, uint64_t n, uint64_t seed,
                      uint64_t counter_offset, uint32_t seg, int mode, double *px, double *py,
                      double *pz)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)n; ++j) {
        uint32_t r[4];
        particle_block(seed, counter_offset + (uint64_t)j, seg, 1, r);
        px[j] = oracle_position_coord(lo[0], size[0], r[0], mode);
        py[j] = oracle_position_coord(lo[1], size[1], r[1], mode);
        pz[j] = oracle_position_coord(lo[2], size[2], r[2], mode);
    }
}

/* Same as oracle_sample, for an arbitrary list of particle indices. */
void oracle_sample_indices(double kappa, double theta, const double *drift, const uint64_t *idx,
                           uint64_t m, uint64_t seed, uint32_t seg, int mode, double *vx,
                           double *vy, double *vz)
{
    double p[OP_COUNT];
    double zero[3] = {0.0, 0.0, 0.0};
    const double *d = drift ? drift : zero;
    oracle_params(kappa, p);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)m; ++j) {
        uint32_t r[4];
        double v[3];
        particle_block(seed, idx[j], seg, 0, r);
        one_particle(p, theta, d, mode, r, v);
        vx[j] = v[0]; vy[j] = v[1]; vz[j] = v[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the sampler at fixed uniforms (reparameterisation gradient).
 * Not in the paper; derived from its equations:
 *   dv/dtheta = v / theta  (v is linear in theta, Table 1)
 *   x solves P(x) = b x^2 + (a + cL) x + L = 0 (eq:v), and dP/dx = 2bx + A = D,
 *   so dx/dkappa = -(b' x^2 + (a' + c' L + c L') x + L') / D,
 *   with L = -kappa* expm1(z), z = -lT/kappa*, lT independent of kappa:
 *   L' = -expm1(z) + z e^z;  dv/dkappa = v (dx/dkappa) / (2x).
 * Returns sum_i g_i . dv_i/dkappa and sum_i g_i . dv_i/dtheta (drift-free). */
/* ------------------------------------------------------------------------ */
void oracle_backward(double kappa, double theta, uint64_t n, uint64_t seed, uint64_t counter_offset,
                     uint32_t seg, int mode, const float *gx, const float *gy, const float *gz,
                     double out[2])
{
    double p[OP_COUNT];
    oracle_params(kappa, p);
    double c = p[OP_C], da = p[OP_DA], db = p[OP_DB], dc = p[OP_DC];
    double sum_k = 0.0, sum_t = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : sum_k, sum_t)
    for (int64_t j = 0; j < (int64_t)n; ++j) {
        uint32_t r[4];
        int side;
        double u;
        inversion inv;
        particle_block(seed, counter_offset + (uint64_t)j, seg, 0, r);
        oracle_speed_uniform(mode, r[0], r[3], &side, &u);
        invert(p, side, u, &inv);
        double V = theta * sqrt(inv.x);
        double cos_t, u2prod;
        polar_uniform(r[1], &cos_t, &u2prod);
        double sin_t = 2.0 * sqrt(u2prod);
        double phi = 2.0 * M_PI * azimuth_uniform(r[2]);
        double v0 = V * cos_t, v1 = V * sin_t * cos(phi), v2 = V * sin_t * sin(phi);
        double s = (double)gx[j] * v0 + (double)gy[j] * v1 + (double)gz[j] * v2;
        double dL = -expm1(inv.z) + inv.z * exp(inv.z);
        double x = inv.x, L = inv.L;
        double dx = -(db * x * x + (da + dc * L + c * dL) * x + dL) / inv.D;
        sum_k += s * dx / (2.0 * x);
        sum_t += s / theta;
    }
    out[0] = sum_k;
    out[1] = sum_t;
}

/* Indices j in [counter_offset, counter_offset + n) for which the FP32 mode
 * takes the FP64 tail inversion (1 - U1 < 2^-20), in increasing order; at
 * most max_out are written.  Returns how many there are. */
uint64_t oracle_find_tails(uint64_t n, uint64_t seed, uint64_t counter_offset, uint32_t seg, uint64_t *out,
                           uint64_t max_out)
{
    uint64_t found = 0;
    const int64_t chunk = 1 << 20;
    const int64_t nchunks = (int64_t)((n + (uint64_t)chunk - 1) / (uint64_t)chunk);
    for (int64_t c0 = 0; c0 < nchunks; c0 += 64) {
        uint64_t hits[64][16];
        int counts[64] = {0};
        int64_t c1 = c0 + 64 < nchunks ? c0 + 64 : nchunks;
#pragma omp parallel for schedule(dynamic)
        for (int64_t c = c0; c < c1; ++c) {
            uint64_t lo = (uint64_t)c * (uint64_t)chunk, hi = lo + (uint64_t)chunk;
            if (hi > n) hi = n;
            for (uint64_t j = lo; j < hi; ++j) {
                uint32_t r[4];
                particle_block(seed, counter_offset + j, seg, 0, r);
                if (r[0] >= 0xFFFFF000u && counts[c - c0] < 16)
                    hits[c - c0][counts[c - c0]++] = counter_offset + j;
            }
        }
        for (int64_t c = c0; c < c1; ++c)
            for (int k = 0; k < counts[c - c0]; ++k) {
                if (found < max_out) out[found] = hits[c - c0][k];
                ++found;
            }
    }
    return found;
}

/* Loss sum_i g_i . v_i of the samples (drift-free), for finite differences. */
double oracle_dot(double kappa, double theta, uint64_t n, uint64_t seed, uint64_t counter_offset, uint32_t seg,
                  int mode, const float *gx, const float *gy, const float *gz)
{
    double p[OP_COUNT];
    double zero[3] = {0.0, 0.0, 0.0};
    double sum = 0.0;
    oracle_params(kappa, p);
#pragma omp parallel for schedule(static) reduction(+ : sum)
    for (int64_t j = 0; j < (int64_t)n; ++j) {
        uint32_t r[4];
        double v[3];
        particle_block(seed, counter_offset + (uint64_t)j, seg, 0, r);
        one_particle(p, theta, zero, mode, r, v);
        sum += (double)gx[j] * v[0] + (double)gy[j] * v[1] + (double)gz[j] * v[2];
    }
    return sum;
}

/* ------------------------------------------------------------------------ */
/* Speed histogram for the Monte Carlo relative entropy of the paper's second
 * test (Sec. 5, eq:KL): counts[k] += #{particles with
 * edge2[k] <= s2 < edge2[k+1]} for k < nbins, counts[nbins] += the rest, where
 * s2 = (vx*vx + vy*vy) + vz*vz in the data's precision and
 * edge2[k] = (k * (bin_width * theta))^2 in FP64, rounded once to that
 * precision.  Plain loop, binary search over the edges.                    */
/* ------------------------------------------------------------------------ */
static uint32_t bin_of_f32(const float *edge2, uint32_t nbins, float s2)
{
    uint32_t lo = 0, hi = nbins; /* edge2[lo] <= s2 holds for lo = 0 */
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (edge2[mid] <= s2)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

void oracle_speed_histogram_f32(const float *vx, const float *vy, const float *vz, uint64_t n, double theta,
                                double bin_width, uint32_t nbins, uint64_t *counts)
{
    double width = bin_width * theta;
    float edge2[2048];
    for (uint32_t k = 0; k <= nbins; ++k) {
        double e = (double)k * width;
        edge2[k] = (float)(e * e);
    }
    for (uint64_t j = 0; j < n; ++j) {
        float s2 = (vx[j] * vx[j] + vy[j] * vy[j]) + vz[j] * vz[j];
        counts[bin_of_f32(edge2, nbins, s2)] += 1;
    }
}

static uint32_t bin_of_f64(const double *edge2, uint32_t nbins, double s2)
{
    uint32_t lo = 0, hi = nbins;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (edge2[mid] <= s2)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

void oracle_speed_histogram_f64(const double *vx, const double *vy, const double *vz, uint64_t n, double theta,
                                double bin_width, uint32_t nbins, uint64_t *counts)
{
    double width = bin_width * theta;
    double edge2[2048];
    for (uint32_t k = 0; k <= nbins; ++k) {
        double e = (double)k * width;
        edge2[k] = e * e;
    }
    for (uint64_t j = 0; j < n; ++j) {
        double s2 = (vx[j] * vx[j] + vy[j] * vy[j]) + vz[j] * vz[j];
        counts[bin_of_f64(edge2, nbins, s2)] += 1;
    }
}

/* Number of worker threads the oracle's parallel loops use. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
