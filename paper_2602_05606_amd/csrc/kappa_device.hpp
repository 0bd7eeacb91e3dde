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

__device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(kMulA) * c0;
        const uint64_t pb = static_cast<uint64_t>(kMulB) * c2;
        const uint32_t n0 = static_cast<uint32_t>(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(pa >> 32) ^ c3 ^ k1;
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

struct InvF64 {
    double z;  // -lT / kappa*
    double L;  // q-logarithm of 1 - U1^{2/3}
    double D;  // sqrt(A^2 - 4bL)
    double x;  // (V/theta)^2
};

__device__ __forceinline__ InvF64 invert_f64(bool high, double u, const SpeciesF64 &s)
{
    // l1 = ln U1.  High side: U1 = 1 - u = y1 + d1 exactly, y1 = fl(1 - u).
    const double y1 = high ? 1.0 - u : u;
    const double d1 = high ? (1.0 - y1) - u : 0.0;
    const double l1 = log(y1) + d1 / y1;
    const double p = (2.0 / 3.0) * l1;
    // 1 - U1^{2/3} = y2 + d2.  Low side: t = e^p, y2 = fl(1 - t), d2 = (1 - y2) - t.
    // High side: y2 = -expm1(p), d2 = 0.
    const double t = exp(p);
    const double em1 = expm1(p);
    const double y2 = high ? -em1 : 1.0 - t;
    const double d2 = high ? 0.0 : (1.0 - y2) - t;
    const double lT = log(y2) + d2 / y2;
    InvF64 r;
    r.z = -lT * s.inv_kstar;
    r.L = -s.kstar * expm1(r.z);
    const double A = fma(s.c, r.L, s.a);
    r.D = sqrt(fma(A, A, -4.0 * s.b * r.L));
    r.x = (A >= 0.0) ? (-2.0 * r.L) / (A + r.D) : (r.D - A) * s.half_inv_b;
    return r;
}

struct InvF32 {
    float z, L, D, x;
};

__device__ __forceinline__ InvF32 invert_f32(bool high, float u, const SpeciesF32 &s)
{
    const float y1 = high ? 1.0f - u : u;
    const float d1 = high ? (1.0f - y1) - u : 0.0f;
    const float l1 = logf(y1) + d1 / y1;
    const float p = (2.0f / 3.0f) * l1;
    const float t = expf(p);
    const float em1 = expm1f(p);
    const float y2 = high ? -em1 : 1.0f - t;
    const float d2 = high ? 0.0f : (1.0f - y2) - t;
    const float lT = logf(y2) + d2 / y2;
    InvF32 r;
    r.z = -lT * s.inv_kstar;
    r.L = -s.kstar * expm1f(r.z);
    const float A = fmaf(s.c, r.L, s.a);
    r.D = sqrtf(fmaf(A, A, -4.0f * s.b * r.L));
    r.x = (A >= 0.0f) ? (-2.0f * r.L) / (A + r.D) : (r.D - A) * s.half_inv_b;
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
__device__ __forceinline__ void speed_uniform_f32(uint32_t r0, bool &high, float &u)
{
    const uint32_t m = r0 >> 8;
    high = m >= (1u << 23);
    const uint32_t k = high ? (1u << 25) - 2 * m - 1 : 2 * m + 1;  // < 2^24: exact in float
    u = static_cast<float>(k) * 0x1p-25f;
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
    const double st = sqrt((1.0 - ct) * (1.0 + ct));  // both factors exact
    const double u3x2 = static_cast<double>(2 * static_cast<uint64_t>(r2) + 1) * 0x1p-32;  // 2 U3
    double sp, cp;
    sincospi(u3x2, &sp, &cp);
    DirF64 d;
    d.cx = ct;
    d.cy = st * cp;
    d.cz = st * sp;
    return d;
}

struct DirF32 {
    float cx, cy, cz;
};

__device__ __forceinline__ DirF32 direction_f32(uint32_t r1, uint32_t r2)
{
    const int32_t k = static_cast<int32_t>(2 * (r1 >> 8) + 1) - (1 << 24);  // |k| < 2^24
    const float ct = static_cast<float>(k) * 0x1p-24f;
    const float st = sqrtf((1.0f - ct) * (1.0f + ct));
    const float u3x2 = static_cast<float>(2 * (r2 >> 8) + 1) * 0x1p-24f;  // 2 U3
    float sp, cp;
    sincospif(u3x2, &sp, &cp);
    DirF32 d;
    d.cx = ct;
    d.cy = st * cp;
    d.cz = st * sp;
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
    const double V = s.theta * sqrt(inv.x);
    const DirF64 d = direction_f64(b.r1, b.r2);
    vx = V * d.cx;
    vy = V * d.cy;
    vz = V * d.cz;
}

// FP32 bulk particle (no tail handling).
__device__ __forceinline__ void particle_f32(const Block4 &b, const SpeciesF32 &s, float &vx, float &vy, float &vz)
{
    bool high;
    float u;
    speed_uniform_f32(b.r0, high, u);
    const InvF32 inv = invert_f32(high, u, s);
    const float V = s.theta * sqrtf(inv.x);
    const DirF32 d = direction_f32(b.r1, b.r2);
    vx = V * d.cx;
    vy = V * d.cy;
    vz = V * d.cz;
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
    const float V = static_cast<float>(s64.theta * sqrt(inv.x));
    const DirF32 d = direction_f32(b.r1, b.r2);
    vx = V * d.cx;
    vy = V * d.cy;
    vz = V * d.cz;
}

}  // namespace kappa
