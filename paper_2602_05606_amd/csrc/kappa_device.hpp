// kappa_device.hpp -- device-side building blocks of the approximate Kappa
// generator (Zenitani & Umeda, arXiv 2602.05606, Sec. 4 and Table 1) for
// gfx950: the Philox4x32-10 counter RNG, the uniform maps, the closed-form
// inversion of the approximate CDF G in FP64 and FP32, and the isotropic
// direction.  Everything lives in registers; nothing here touches memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kappa_params.hpp"

namespace kappa {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key schedule is
// uniform across the wave, so the compiler keeps it in scalar registers; each
// round costs two 32x32->64 multiplies and two three-input XORs per lane.
// ---------------------------------------------------------------------------
struct Block4 {
    uint32_t r0, r1, r2, r3;
};

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96 is the three-input XOR).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;

__device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(kMulA) * c0;
        const uint64_t pb = static_cast<uint64_t>(kMulB) * c2;
        const uint32_t n0 = xor3(static_cast<uint32_t>(pb >> 32), c1, k0);
        const uint32_t n2 = xor3(static_cast<uint32_t>(pa >> 32), c3, k1);
        c1 = static_cast<uint32_t>(pb);
        c3 = static_cast<uint32_t>(pa);
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return Block4{c0, c1, c2, c3};
}

// Philox4x32-10 of a counter (c0, u1, u2, u3) whose words u1, u2, u3 are the
// same in every lane of a launch (the high word of the particle index, seg and
// draw): the words of philox4x32_10, with the first three rounds grouped so
// that every product or XOR of uniform words runs on the scalar unit.  The
// first product M_A c0 comes in as pa1, so that a caller can fold c0 = base + k
// into one multiply-add.
__device__ __forceinline__ Block4 philox4x32_10_lane(uint64_t pa1, uint32_t u1, uint32_t u2, uint32_t u3,
                                                     uint32_t k0, uint32_t k1)
{
    // round 1: M_B u2 and the new c0 are uniform
    const uint64_t pb1 = static_cast<uint64_t>(kMulB) * u2;
    uint32_t c0 = static_cast<uint32_t>(pb1 >> 32) ^ u1 ^ k0;
    uint32_t c1 = static_cast<uint32_t>(pb1);
    uint32_t c2 = static_cast<uint32_t>(pa1 >> 32) ^ (u3 ^ k1);
    uint32_t c3 = static_cast<uint32_t>(pa1);
    k0 += kWeylA;
    k1 += kWeylB;
    {  // round 2: c0 and c1 uniform, so M_A c0 is too
        const uint64_t pa = static_cast<uint64_t>(kMulA) * c0;
        const uint64_t pb = static_cast<uint64_t>(kMulB) * c2;
        const uint32_t n0 = static_cast<uint32_t>(pb >> 32) ^ (c1 ^ k0);
        const uint32_t n2 = c3 ^ (static_cast<uint32_t>(pa >> 32) ^ k1);
        c1 = static_cast<uint32_t>(pb);
        c3 = static_cast<uint32_t>(pa);
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    {  // round 3: c3 uniform
        const uint64_t pa = static_cast<uint64_t>(kMulA) * c0;
        const uint64_t pb = static_cast<uint64_t>(kMulB) * c2;
        const uint32_t n0 = xor3(static_cast<uint32_t>(pb >> 32), c1, k0);
        const uint32_t n2 = static_cast<uint32_t>(pa >> 32) ^ (c3 ^ k1);
        c1 = static_cast<uint32_t>(pb);
        c3 = static_cast<uint32_t>(pa);
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(kMulA) * c0;
        const uint64_t pb = static_cast<uint64_t>(kMulB) * c2;
        const uint32_t n0 = xor3(static_cast<uint32_t>(pb >> 32), c1, k0);
        const uint32_t n2 = xor3(static_cast<uint32_t>(pa >> 32), c3, k1);
        c1 = static_cast<uint32_t>(pb);
        c3 = static_cast<uint32_t>(pa);
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return Block4{c0, c1, c2, c3};
}

// The words a segment's counters (c0, 0, seg, draw) share through Philox's
// first two rounds: after round 1, c0 = hi(M_B seg) ^ k0 and c1 = lo(M_B seg),
// and round 2's product M_A c0 (hi, lo).  They depend on seg and the key only,
// so a batched plan computes them once per segment on the host.
struct SegWords {
    uint32_t c0, c1, pa_hi, pa_lo;
};

// Philox4x32-10 of the counter (c0, 0, seg, draw) from its segment's words:
// per particle, round 1 takes one product and round 2 one, against two each in
// philox4x32_10.  The words are the same.
__device__ __forceinline__ Block4 philox4x32_10_seg(uint32_t c0_in, uint32_t draw, const SegWords &w, uint32_t k0,
                                                    uint32_t k1)
{
    // round 1: M_B seg and the new c0, c1 come from the segment's words
    const uint64_t pa1 = static_cast<uint64_t>(kMulA) * c0_in;
    uint32_t c2 = static_cast<uint32_t>(pa1 >> 32) ^ draw ^ k1;
    uint32_t c3 = static_cast<uint32_t>(pa1);
    k0 += kWeylA;
    k1 += kWeylB;
    uint32_t c0, c1;
    {  // round 2: M_A c0 is the segment's (pa_hi, pa_lo)
        const uint64_t pb = static_cast<uint64_t>(kMulB) * c2;
        c0 = xor3(static_cast<uint32_t>(pb >> 32), w.c1, k0);
        c2 = xor3(w.pa_hi, c3, k1);
        c1 = static_cast<uint32_t>(pb);
        c3 = w.pa_lo;
        k0 += kWeylA;
        k1 += kWeylB;
    }
#pragma unroll
    for (int r = 2; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(kMulA) * c0;
        const uint64_t pb = static_cast<uint64_t>(kMulB) * c2;
        const uint32_t n0 = xor3(static_cast<uint32_t>(pb >> 32), c1, k0);
        const uint32_t n2 = xor3(static_cast<uint32_t>(pa >> 32), c3, k1);
        c1 = static_cast<uint32_t>(pb);
        c3 = static_cast<uint32_t>(pa);
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return Block4{c0, c1, c2, c3};
}

// Block of particle i (global counter index) in segment seg, draw d.
__device__ __forceinline__ Block4 particle_block(uint64_t i, uint32_t seg, uint32_t draw, uint32_t k0, uint32_t k1)
{
    return philox4x32_10(static_cast<uint32_t>(i), static_cast<uint32_t>(i >> 32), seg, draw, k0, k1);
}

// ---------------------------------------------------------------------------
// Speed inversion (Sec. 4).  G(x) = U1 (eq:GU) is solved with the q-logarithm
// (eq:qlog): L = ln_{q*}(1 - U1^{2/3}) (eq:L), then x = (V/theta)^2 is the
// positive root of b x^2 + (a + cL) x + L = 0 (eq:v).
//
// Evaluation order, chosen so that no step subtracts nearly equal numbers and
// so that both sides of U1 run the same instructions (no divergence):
//   l1 = ln U1            low side: ln(u);   high side (u = 1-U1): ln(1-u)
//   p  = (2/3) l1         ln U1^{2/3}
//   lT = ln(1 - e^p)      low side: log1p(-e^p); high side: ln(-expm1(p))
//   L  = -kappa* expm1(-lT / kappa*)          (= eq:L)
//   A = a + cL,  D = sqrt(A^2 - 4bL)
//   x = -2L / (A + D) if A >= 0 else (D - A) / (2b)   (the two forms of eq:v)
// A logarithm of a value known as y + d with |d| << y (d exact) is taken as
// ln(y) + d/y, which is how one log call serves both sides.
// ---------------------------------------------------------------------------

// e^p and e^p - 1 from one argument reduction (the textbook method: Cody and
// Waite's two-part ln 2, then a polynomial on |r| <= ln2/2): p = k ln2 + r,
// q = expm1(r) = r + r^2 t(r) with t a degree-10 near-minimax fit (Chebyshev
// nodes, 60-digit arithmetic; 1.1e-16 relative for q with FP64 evaluation),
// e^p = 2^k (1 + q), e^p - 1 = 2^k q + (2^k - 1).  The last form has no
// harmful cancellation for any k (|q| <= 0.42).  2^k is assembled from its
// exponent bits: the callers' |p| stay far inside the normal range.
__device__ __forceinline__ void exp_expm1_f64(double p, double &e, double &em1)
{
    constexpr double kLog2e = 0x1.71547652b82fep+0;
    constexpr double kLn2Hi = 0x1.62e42fefa3800p-1, kLn2Lo = 0x1.ef35793c76730p-45;
    const double k = rint(p * kLog2e);
    double r = fma(-k, kLn2Hi, p);
    r = fma(-k, kLn2Lo, r);
    double t = 0x1.1f72fc730b4ffp-29;
    t = fma(t, r, 0x1.af4ddd84882fep-26);
    t = fma(t, r, 0x1.27e4db67b4303p-22);
    t = fma(t, r, 0x1.71de02375656cp-19);
    t = fma(t, r, 0x1.a01a01a6d7808p-16);
    t = fma(t, r, 0x1.a01a01abe62ddp-13);
    t = fma(t, r, 0x1.6c16c16c162d6p-10);
    t = fma(t, r, 0x1.11111111100dfp-7);
    t = fma(t, r, 0x1.5555555555556p-5);
    t = fma(t, r, 0x1.5555555555557p-3);
    t = fma(t, r, 0.5);
    const double q = fma(r * r, t, r);        // expm1(r)
    const double pk = __hiloint2double((static_cast<int>(k) + 1023) << 20, 0);  // 2^k
    e = fma(q, pk, pk);
    em1 = fma(q, pk, pk - 1.0);
}

// Natural log of x in (0, 1] (normal doubles), within a few ulp: x = m 2^e
// with m in [sqrt(1/2), sqrt(2)), f = m - 1 (exact), and
// log(1 + f) = 2 atanh(s) = 2s + s z Q(z), s = f / (2 + f), z = s^2 <= 0.0295,
// Q a degree-6 near-minimax fit of (2 atanh(s)/s - 2)/z (1.1e-16 relative for
// the log with FP64 evaluation).  The division is one v_rcp_f64 step refined
// by a Newton correction.
__device__ __forceinline__ double log_unit_f64(double x)
{
    constexpr double kLn2Hi = 0x1.62e42fefa3800p-1, kLn2Lo = 0x1.ef35793c76730p-45;
    double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    const bool low = m < 0x1.6a09e667f3bcdp-1;   // sqrt(1/2)
    m = low ? 2.0 * m : m;
    e = low ? e - 1 : e;
    const double f = m - 1.0;
    const double den = 2.0 + f;
    const double rc = __builtin_amdgcn_rcp(den);
    double sv = f * rc;
    sv = fma(fma(-sv, den, f), rc, sv);          // one Newton correction of f / den
    const double z = sv * sv;
    double q = 0x1.2b584aae78a57p-3;
    q = fma(q, z, 0x1.39fe606542ddep-3);
    q = fma(q, z, 0x1.7462b4ab2ef6bp-3);
    q = fma(q, z, 0x1.c71c62e5800a1p-3);
    q = fma(q, z, 0x1.2492492df148dp-2);
    q = fma(q, z, 0x1.99999999952e2p-2);
    q = fma(q, z, 0x1.5555555555558p-1);
    const double ed = static_cast<double>(e);
    const double lo = fma(ed, kLn2Lo, sv * z * q);
    return fma(ed, kLn2Hi, fma(2.0, sv, lo));
}

// sin(pi x) and cos(pi x) for x = (2 r + 1) 2^-32 in (0, 2), exact in double:
// n = rint(2x), r = x - n/2 in [-1/4, 1/4] (exact), t = pi r, then
// sin t = t - t^3 S(t^2) and cos t = 1 - t^2 C(t^2) with S and C degree-6
// near-minimax fits on |t| <= pi/4 (1.1e-16 relative with FP64 evaluation);
// the quadrant n mod 4 swaps and signs the pair.
__device__ __forceinline__ void sincospi_f64(double x, double &sn, double &cs)
{
    const double n = rint(2.0 * x);
    const double r = fma(-0.5, n, x);
    const double t = r * 0x1.921fb54442d18p+1;   // pi r, |t| <= pi/4
    const double t2 = t * t;
    double ps = 0x1.ab17d404de5b3p-41;
    ps = fma(ps, t2, -0x1.61217f0b800d5p-33);
    ps = fma(ps, t2, 0x1.ae645412c560cp-26);
    ps = fma(ps, t2, -0x1.71de3a546095bp-19);
    ps = fma(ps, t2, 0x1.a01a01a019938p-13);
    ps = fma(ps, t2, -0x1.1111111111110p-7);
    ps = fma(ps, t2, 0x1.5555555555555p-3);
    const double sr = fma(-t * t2, ps, t);       // sin(pi r)
    double pc = 0x1.8ff9d439a204ap-37;
    pc = fma(pc, t2, -0x1.1eea7f259b344p-29);
    pc = fma(pc, t2, 0x1.27e4f8e4a2e74p-22);
    pc = fma(pc, t2, -0x1.a01a019de131fp-16);
    pc = fma(pc, t2, 0x1.6c16c16c15d79p-10);
    pc = fma(pc, t2, -0x1.5555555555551p-5);
    pc = fma(pc, t2, 0.5);
    const double cr = fma(-t2, pc, 1.0);         // cos(pi r)
    const int q = static_cast<int>(n) & 3;
    const double a = (q & 1) ? cr : sr;
    const double b = (q & 1) ? sr : cr;
    sn = (q & 2) ? -a : a;
    cs = ((q + 1) & 2) ? -b : b;
}

// 1/sqrt(a) and sqrt(a) for positive normal doubles (every caller's argument
// is one): v_rsq_f64's estimate y with relative error e0, refined by one step
// of the second-order iteration y (1 + e/2 + 3e^2/8), e = 1 - a y^2, which
// leaves O(e0^3); sqrt(a) = a y, then one Newton correction (a - g^2)/(2g).
__device__ __forceinline__ double rsqrt_pos_f64(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    const double e = fma(-a * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ double sqrt_pos_f64(double a)
{
    const double y = rsqrt_pos_f64(a);
    const double g = a * y;
    return fma(fma(-g, g, a), 0.5 * y, g);
}

struct InvF64 {
    double z;    // -lT / kappa*
    double ez;   // e^z
    double em1;  // e^z - 1
    double L;    // q-logarithm of 1 - U1^{2/3}
    double D;    // sqrt(A^2 - 4bL)
    double num, den;  // x = (V/theta)^2 = num / den, both > 0
    __device__ __forceinline__ double x() const { return num / den; }
    __device__ __forceinline__ double sqrt_x() const { return num * rsqrt_pos_f64(num * den); }
};

__device__ __forceinline__ InvF64 invert_f64(bool high, double u, const SpeciesF64 &s)
{
    // l1 = ln U1.  High side: U1 = 1 - u = y1 + d1 exactly, y1 = fl(1 - u); the
    // correction d1/y1 is taken as d1 (|d1| <= 2^-54 and y1 >= 1/2, so this
    // changes ln U1 by less than 2^-53 relative).
    const double y1 = high ? 1.0 - u : u;
    const double d1 = high ? (1.0 - y1) - u : 0.0;
    const double l1 = log_unit_f64(y1) + d1;
    const double p = (2.0 / 3.0) * l1;
    // 1 - U1^{2/3} = y2 + d2.  Low side: t = e^p, y2 = fl(1 - t), d2 = (1 - y2) - t.
    // High side: y2 = -expm1(p), d2 = 0.
    double t, em1;
    exp_expm1_f64(p, t, em1);
    const double y2 = high ? -em1 : 1.0 - t;
    const double d2 = high ? 0.0 : (1.0 - y2) - t;
    const double lT = log_unit_f64(y2) + d2;
    InvF64 r;
    r.z = -lT * s.inv_kstar;
    exp_expm1_f64(r.z, r.ez, r.em1);
    r.L = -s.kstar * r.em1;
    const double A = fma(s.c, r.L, s.a);
    r.D = sqrt_pos_f64(fma(A, A, s.neg_four_b * r.L));
    const bool pos = A >= 0.0;
    r.num = pos ? -2.0 * r.L : r.D - A;
    r.den = pos ? A + r.D : s.two_b;
    return r;
}

// FP32 path.  It runs on the hardware base-2 transcendentals (v_log_f32,
// v_exp_f32), v_sqrt_f32 and v_rsq_f32, each within 2 ulp, in base 2
// throughout: with t = p / ln 2, e^p - 1 = 2^t - 1 is taken by a degree-4
// polynomial for (2^t - 1) / t where |t| is small (two near-minimax fits at
// Chebyshev nodes, one per argument range; approximation error <= 1.0e-7,
// <= 1.8e-7 with FP32 evaluation).  Same evaluation order as invert_f64.

// 2^t - 1 for t in [-2/3, 0] (the high side's U1^{2/3} - 1).
__device__ __forceinline__ float exp2m1_neg(float t)
{
    float p = fmaf(0x1.20ec64p-10f, t, 0x1.36e5bep-7f);
    p = fmaf(p, t, 0x1.c6708p-5f);
    p = fmaf(p, t, 0x1.ebfa8cp-3f);
    p = fmaf(p, t, 0x1.62e42ep-1f);
    return t * p;
}

// 2^t - 1 for t in [0, 1 / (2 ln 2)] (expm1(z) for z < 1/2).
__device__ __forceinline__ float exp2m1_pos(float t)
{
    float p = fmaf(0x1.af907ep-10f, t, 0x1.34741cp-7f);
    p = fmaf(p, t, 0x1.c7211p-5f);
    p = fmaf(p, t, 0x1.ebf952p-3f);
    p = fmaf(p, t, 0x1.62e432p-1f);
    return t * p;
}

// Threshold of the small-argument branch: z = t ln 2 < 1/2.
constexpr float kExp2m1Small = 0x1.715476p-1f;  // 1 / (2 ln 2)

struct InvF32 {
    float w;         // -log2(1 - U1^{2/3}) / kappa* = z / ln 2
    float z;         // -lT / kappa*
    float ez;        // e^z
    float em1;       // e^z - 1
    float L, D;
    float num, den;  // x = (V/theta)^2 = num / den, both > 0
    __device__ __forceinline__ float x() const { return num * __builtin_amdgcn_rcpf(den); }
    // sqrt(x) = num / sqrt(num den): one transcendental instead of rcp and sqrt
    __device__ __forceinline__ float sqrt_x() const { return num * __builtin_amdgcn_rsqf(num * den); }
};

// The species constants enter premultiplied (SpeciesF32): with L = -kappa* em1,
// A = a + cL = a - (c kappa*) em1, A^2 - 4bL = A^2 + (4b kappa*) em1 and
// -2L = (2 kappa*) em1, so L itself is formed only for the backward pass.
__device__ __forceinline__ InvF32 invert_f32(bool high, float y1, float d1, const SpeciesF32 &s)
{
    constexpr float kLog2e = 0x1.715476p+0f, kLn2 = 0x1.62e430p-1f;
    // log2 U1 = log2(y1 + d1): one hardware log for both sides; the residual
    // (|d1| <= 2^-25, y1 >= 1/2 where it is non-zero) enters as d1 log2(e),
    // whose missing 1/y1 factor changes log2 U1 by less than 2^-24 relative.
    const float l1 = fmaf(d1, kLog2e, __builtin_amdgcn_logf(y1));
    const float p2 = l1 * (2.0f / 3.0f);               // log2 U1^{2/3}
    const float e = __builtin_amdgcn_exp2f(p2);         // U1^{2/3} (low side)
    const float em1q = exp2m1_neg(p2);                  // U1^{2/3} - 1 (high side, p2 in [-2/3, 0])
    const float y2 = high ? -em1q : 1.0f - e;
    const float d2 = high ? 0.0f : (1.0f - y2) - e;
    const float lT2 = fmaf(d2, kLog2e, __builtin_amdgcn_logf(y2));  // log2(1 - U1^{2/3})
    InvF32 r;
    r.w = -lT2 * s.inv_kstar;
    r.z = r.w * kLn2;
    r.ez = __builtin_amdgcn_exp2f(r.w);
    r.em1 = (r.w < kExp2m1Small) ? exp2m1_pos(r.w) : r.ez - 1.0f;
    r.L = -s.kstar * r.em1;
    const float A = fmaf(r.em1, s.neg_c_kstar, s.a);
    r.D = __builtin_amdgcn_sqrtf(fmaf(r.em1, s.four_b_kstar, A * A));
    const bool pos = A >= 0.0f;
    r.num = pos ? r.em1 * s.two_kstar : r.D - A;
    r.den = pos ? A + r.D : s.two_b;
    return r;
}

// ---------------------------------------------------------------------------
// Uniform maps: open midpoint dyadics.  U1 is carried as (side, small value)
// so that both U1 and 1 - U1 are exact; cos(theta) = 2 U2 - 1 is formed
// exactly from the integer word.
// ---------------------------------------------------------------------------

// FP64: m = top 53 bits of (r0:r3).
__device__ __forceinline__ void speed_uniform_f64(uint32_t r0, uint32_t r3, bool &high, double &u)
{
    const uint64_t m = ((static_cast<uint64_t>(r0) << 32) | r3) >> 11;
    high = m >= (1ull << 52);
    const uint64_t k = high ? (1ull << 54) - 2 * m - 1 : 2 * m + 1;  // < 2^53: exact in double
    u = static_cast<double>(k) * 0x1p-54;
}

// FP32 bulk: m24 = r0 >> 8.  Tail when m24 >= 2^24 - 16 (1 - U1 < 2^-20).
// FP32 mode draws the FP64 mode's uniforms.  With R = (r0:r3) and its low 11
// bits replaced by the midpoint bit 2^10, U1 = R 2^-64 exactly.  The small
// side value s (U1 on the low side, 1 - U1 = (~r0, 2^32 - lo) 2^-64 on the
// high side, taken from the integers without cancellation) is rounded to
// float; then y1 = fl(U1) and the exact float residual d1 = (1 - y1) - s on
// the high side give ln U1 = ln(y1 + d1) to float precision for any U1.
__device__ __forceinline__ void speed_uniform_f32(uint32_t r0, uint32_t r3, bool &high, float &y1, float &d1)
{
    const uint32_t mask = static_cast<uint32_t>(static_cast<int32_t>(r0) >> 31);  // ones on the high side
    high = mask != 0u;
    const uint32_t lo = (r3 & 0xFFFFF800u) | 0x400u;
    const uint32_t hw = r0 ^ mask;         // high side: ~r0
    const uint32_t lw = (lo ^ mask) - mask;  // high side: 2^32 - lo
    const float s = fmaf(static_cast<float>(lw), 0x1p-32f, static_cast<float>(hw)) * 0x1p-32f;
    y1 = high ? 1.0f - s : s;
    d1 = high ? (1.0f - y1) - s : 0.0f;
}

__device__ __forceinline__ bool in_fp64_tail(uint32_t r0)
{
    return r0 >= ((1u << 24) - 16u) << 8;
}

// Direction (Table 1, last three rows): cos(theta) = 2U2 - 1,
// sin(theta) = 2 sqrt(U2 (1 - U2)) = sqrt((1 - cos)(1 + cos)), phi = 2 pi U3.
struct DirF64 {
    double cx, cy, cz;  // unit vector
};

__device__ __forceinline__ DirF64 direction_f64(uint32_t r1, uint32_t r2)
{
    const double ct = static_cast<double>(static_cast<int64_t>(2 * static_cast<uint64_t>(r1) + 1) - (1ll << 32)) * 0x1p-32;
    const double st = sqrt_pos_f64((1.0 - ct) * (1.0 + ct));  // both factors exact
    const double u3x2 = static_cast<double>(2 * static_cast<uint64_t>(r2) + 1) * 0x1p-32;  // 2 U3
    double sp, cp;
    sincospi_f64(u3x2, sp, cp);
    DirF64 d;
    d.cx = ct;
    d.cy = st * cp;
    d.cz = st * sp;
    return d;
}

struct DirF32 {
    float cx, cy, cz;  // unit vector
    float st, cphi, sphi;  // sin(theta), cos(phi), sin(phi): cy = st cphi, cz = st sphi
};

// v_sin_f32 / v_cos_f32 take their argument in revolutions, so sin(2 pi U3)
// needs no range reduction (absolute error 1.3e-7 on gfx950).  The uniforms
// are the FP64 mode's: 1 + cos = 2 U2 = (r1 + 1/2) 2^-31 and
// 1 - cos = 2 (1 - U2) = (~r1 + 1/2) 2^-31 each come from the integer word
// without cancellation, so sin = sqrt((1 - cos)(1 + cos)) stays accurate at
// the poles; U3 = (r2 + 1/2) 2^-32 is rounded to float (error <= 2^-24 U3).
__device__ __forceinline__ DirF32 direction_f32(uint32_t r1, uint32_t r2)
{
    const float opc = fmaf(static_cast<float>(r1), 0x1p-31f, 0x1p-32f);
    const float omc = fmaf(static_cast<float>(~r1), 0x1p-31f, 0x1p-32f);
    const float st = __builtin_amdgcn_sqrtf(opc * omc);
    const float u3 = fmaf(static_cast<float>(r2), 0x1p-32f, 0x1p-33f);
    DirF32 d;
    d.cx = 0.5f * (opc - omc);
    d.st = st;
    d.cphi = __builtin_amdgcn_cosf(u3);
    d.sphi = __builtin_amdgcn_sinf(u3);
    d.cy = st * d.cphi;
    d.cz = st * d.sphi;
    return d;
}

// ---------------------------------------------------------------------------
// One particle, all modes.  Returns V/theta-scaled components in (vx, vy, vz).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void particle_f64(const Block4 &b, const SpeciesF64 &s, double &vx, double &vy,
                                             double &vz)
{
    bool high;
    double u;
    speed_uniform_f64(b.r0, b.r3, high, u);
    const InvF64 inv = invert_f64(high, u, s);
    const double V = s.theta * inv.sqrt_x();
    const DirF64 d = direction_f64(b.r1, b.r2);
    vx = V * d.cx;
    vy = V * d.cy;
    vz = V * d.cz;
}

// FP32 bulk particle (no tail handling).
__device__ __forceinline__ void particle_f32(const Block4 &b, const SpeciesF32 &s, float &vx, float &vy, float &vz)
{
    bool high;
    float y1, d1;
    speed_uniform_f32(b.r0, b.r3, high, y1, d1);
    const InvF32 inv = invert_f32(high, y1, d1, s);
    const float V = s.theta * inv.sqrt_x();
    const DirF32 d = direction_f32(b.r1, b.r2);
    const float Vs = V * d.st;  // V sin(theta), shared by vy and vz
    vx = V * d.cx;
    vy = Vs * d.cphi;
    vz = Vs * d.sphi;
}

// FP32-mode particle whose 1 - U1 is below 2^-20: the speed is inverted in
// FP64 from the 53-bit 1 - U1 of the FP64 map and rounded to float; the
// direction is the FP32 one.  Callers take this branch rarely (probability
// 2^-20 per particle) after the bulk pass, so it costs no occupancy there.
__device__ __forceinline__ void tail_particle_f32(const Block4 &b, const SpeciesF64 &s64, float &vx, float &vy,
                                                  float &vz)
{
    bool high;
    double u;
    speed_uniform_f64(b.r0, b.r3, high, u);
    const InvF64 inv = invert_f64(high, u, s64);
    const float V = static_cast<float>(s64.theta * inv.sqrt_x());
    const DirF32 d = direction_f32(b.r1, b.r2);
    vx = V * d.cx;
    vy = V * d.cy;
    vz = V * d.cz;
}

}  // namespace kappa
