// baselines.hip -- exact Kappa generators with rejection loops, run on the
// same GPU and the same Philox4x32-10 stream as the approximate generator, as
// the comparators of the paper's third test (Sec. 5) and its SIMT discussion
// (Sec. 6).  Neither is the paper's method; both sample eq:kappa exactly.
//
// Counter use: particle i, loop iteration t (t >= 1) draws the block with
// counter (i, 0, t); the block with t = 0 holds the uniforms drawn outside the
// loop.  Every loop is capped at kMaxIters iterations so that each wave
// finishes (the cap is reached with probability below 1e-40 and is then
// reported through `iters`).
#include "kappa_device.hpp"
#include "kappa_internal.hpp"
#include "kappa_store.hpp"

namespace kappa {

namespace {

constexpr uint32_t kMaxIters = 64;

// Elementary functions of the two precisions.  FP32 takes the hardware
// instructions the approximate generator uses (v_log_f32 and v_exp_f32 in
// base 2, v_sqrt_f32, v_sin_f32 and v_cos_f32 in revolutions, each within
// 2 ulp), so that both sides of the comparison are built alike; FP64 takes
// the device library's double functions.
template <typename T>
struct Math;

template <>
struct Math<double> {
    // (r + 1/2) 2^-32
    static __device__ __forceinline__ double unit(uint32_t r) { return (static_cast<double>(r) + 0.5) * 0x1p-32; }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    // e^x - 1 for x >= 0
    static __device__ __forceinline__ double expm1_pos(double x) { return ::expm1(x); }
    // sin and cos of 2 pi u
    static __device__ __forceinline__ void sincos_rev(double u, double &s, double &c) { sincospi(2.0 * u, &s, &c); }
};

template <>
struct Math<float> {
    // (floor(r / 2^8) + 1/2) 2^-24, exact in float
    static __device__ __forceinline__ float unit(uint32_t r)
    {
        return fmaf(static_cast<float>(r >> 8), 0x1p-24f, 0x1p-25f);
    }
    static __device__ __forceinline__ float log(float x) { return __builtin_amdgcn_logf(x) * 0x1.62e430p-1f; }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    // e^x - 1 for x >= 0: 2^t - 1 with t = x log2(e), by the generator's
    // polynomial below t = 1/(2 ln 2) and from v_exp_f32 above it
    static __device__ __forceinline__ float expm1_pos(float x)
    {
        const float t = x * 0x1.715476p+0f;
        return t < kExp2m1Small ? exp2m1_pos(t) : __builtin_amdgcn_exp2f(t) - 1.0f;
    }
    static __device__ __forceinline__ void sincos_rev(float u, float &s, float &c)
    {
        s = __builtin_amdgcn_sinf(u);
        c = __builtin_amdgcn_cosf(u);
    }
};

// Philox block of particle i at loop iteration t (counter (i, 0, t)).  With
// HI_UNIFORM the launch's particle indices share their high word hi, so the
// first rounds run partly on the scalar unit, as in the generator.
template <bool HI_UNIFORM>
__device__ __forceinline__ Block4 exact_block(uint64_t i, uint32_t hi, uint32_t t, uint32_t k0, uint32_t k1)
{
    if constexpr (HI_UNIFORM)
        return philox4x32_10_lane(static_cast<uint64_t>(kMulA) * static_cast<uint32_t>(i), hi, 0, t, k0, k1);
    else
        return particle_block(i, 0, t, k0, k1);
}

// Box-Muller (Box & Muller 1958): two uniforms -> two independent normals.
template <typename T>
__device__ __forceinline__ void box_muller(uint32_t ra, uint32_t rb, T &z0, T &z1)
{
    const T rad = Math<T>::sqrt(T(-2) * Math<T>::log(Math<T>::unit(ra)));
    T s, c;
    Math<T>::sincos_rev(Math<T>::unit(rb), s, c);
    z0 = rad * c;
    z1 = rad * s;
}

// Kappa as a multivariate t with 2 kappa - 1 degrees of freedom:
// v = theta sqrt(kappa / (2 G)) (Z1, Z2, Z3), G ~ Gamma(kappa - 1/2), drawn
// with Marsaglia & Tsang (2000) (shape kappa - 1/2 > 1, so no boost step).
// Each thread produces U consecutive particles, one after the other, and
// stores them as the generator does.
template <typename T, int U, bool HI_UNIFORM>
__global__ void __launch_bounds__(256) exact_t_kernel(ExactArgs a)
{
    const uint64_t ngroups = (a.n + U - 1) / U;
    const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    const T shape = static_cast<T>(a.kappa - 0.5);
    const T d = shape - T(1) / T(3);
    const T cmt = Math<T>::rsqrt(T(9) * d);
    const T scale = static_cast<T>(a.theta * sqrt(0.5 * a.kappa));
    const uint64_t j0 = g * U;
    T x[U], y[U], z[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const uint64_t l = j0 + k;  // position in this launch's outputs
        const uint64_t i = a.first + l;  // particle index: the counter
        x[k] = y[k] = z[k] = T(0);
        if (l >= a.n) continue;
        const Block4 b0 = exact_block<HI_UNIFORM>(i, a.hi, 0, a.k0, a.k1);
        T z1, z2, z3, spare;
        box_muller<T>(b0.r0, b0.r1, z1, z2);
        box_muller<T>(b0.r2, b0.r3, z3, spare);
        (void)spare;
        T gam = d;
        uint32_t t = 1;
        for (; t <= kMaxIters; ++t) {
            const Block4 bt = exact_block<HI_UNIFORM>(i, a.hi, t, a.k0, a.k1);
            T nx, unused;
            box_muller<T>(bt.r0, bt.r1, nx, unused);
            (void)unused;
            const T w = T(1) + cmt * nx;
            if (w <= T(0)) continue;
            const T v = w * w * w;
            const T u = Math<T>::unit(bt.r2);
            const T x2 = nx * nx;
            gam = d * v;
            if (u < T(1) - T(0.0331) * x2 * x2) break;
            if (Math<T>::log(u) < T(0.5) * x2 + d * (T(1) - v + Math<T>::log(v))) break;
        }
        const T f = scale * Math<T>::rsqrt(gam);
        x[k] = f * z1;
        y[k] = f * z2;
        z[k] = f * z3;
        if (a.iters) a.iters[l] = t > kMaxIters ? kMaxIters : t;
    }
    store_or_tail<T, U>(static_cast<T *>(a.vx), j0, a.n, x);
    store_or_tail<T, U>(static_cast<T *>(a.vy), j0, a.n, y);
    store_or_tail<T, U>(static_cast<T *>(a.vz), j0, a.n, z);
}

// Speed by rejection from a Type II Pareto (Lomax) proposal with index
// n = kappa/2: s^2 = kappa (W^{-2/kappa} - 1), W uniform, proposal density
// q(s) = s (1 + s^2/kappa)^{-(kappa/2 + 1)} against the target
// f(s) ~ s^2 (1 + s^2/kappa)^{-(kappa+1)} of eq:kappa.  f/q is proportional
// to s (1 + s^2/kappa)^{-kappa/2} = s W, which peaks at s^2 = kappa/(kappa-1);
// the acceptance test is U <= s W (kappa/(kappa-1))^{(kappa-1)/2}.  Its
// acceptance rate is the p2 of eq:pareto_eff.  Direction from the two
// uniforms drawn outside the loop, as in Table 1.
template <typename T, int U, bool HI_UNIFORM>
__global__ void __launch_bounds__(256) exact_pareto_kernel(ExactArgs a)
{
    const uint64_t ngroups = (a.n + U - 1) / U;
    const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    const T kap = static_cast<T>(a.kappa);
    const T neg2k = static_cast<T>(-2.0 / a.kappa);
    const T ln_m = static_cast<T>(0.5 * (a.kappa - 1.0) * log(a.kappa / (a.kappa - 1.0)));
    const T theta = static_cast<T>(a.theta);
    const uint64_t j0 = g * U;
    T x[U], y[U], z[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const uint64_t l = j0 + k;  // position in this launch's outputs
        const uint64_t i = a.first + l;  // particle index: the counter
        x[k] = y[k] = z[k] = T(0);
        if (l >= a.n) continue;
        const Block4 b0 = exact_block<HI_UNIFORM>(i, a.hi, 0, a.k0, a.k1);
        T sp2 = T(0);
        uint32_t t = 1;
        for (; t <= kMaxIters; ++t) {
            const Block4 bt = exact_block<HI_UNIFORM>(i, a.hi, t, a.k0, a.k1);
            const T lw = Math<T>::log(Math<T>::unit(bt.r0));
            sp2 = kap * Math<T>::expm1_pos(neg2k * lw);  // s^2
            const T u = Math<T>::unit(bt.r1);
            // U <= s W M, in logarithms: ln U <= ln(s^2)/2 + ln W + ln M
            if (Math<T>::log(u) <= T(0.5) * Math<T>::log(sp2) + lw + ln_m) break;
        }
        const T ct = T(2) * Math<T>::unit(b0.r1) - T(1);
        const T st = Math<T>::sqrt((T(1) - ct) * (T(1) + ct));
        T sp, cp;
        Math<T>::sincos_rev(Math<T>::unit(b0.r2), sp, cp);
        const T V = theta * Math<T>::sqrt(sp2);
        x[k] = V * ct;
        y[k] = V * st * cp;
        z[k] = V * st * sp;
        if (a.iters) a.iters[l] = t > kMaxIters ? kMaxIters : t;
    }
    store_or_tail<T, U>(static_cast<T *>(a.vx), j0, a.n, x);
    store_or_tail<T, U>(static_cast<T *>(a.vy), j0, a.n, y);
    store_or_tail<T, U>(static_cast<T *>(a.vz), j0, a.n, z);
}

// One thread per group of U particles (U = 4 in FP32 and 2 in FP64 when the
// outputs are 16-byte aligned, else 1), the generator's launch shape.

template <typename T, int U>
hipError_t launch_exact(void (*kernel)(ExactArgs), const ExactArgs &a, hipStream_t stream)
{
    const uint64_t groups = (a.n + U - 1) / U;
    const uint64_t grid = (groups + 255) / 256;
    log_launch("exact_kernel", sizeof(T) == 8 ? kModeF64 : kModeF32, a.n, Shape{256, U, static_cast<int>(grid)},
               stream);
    hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(grid > 0 ? grid : 1)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

bool aligned16(const ExactArgs &a)
{
    return reinterpret_cast<uintptr_t>(a.vx) % 16 == 0 && reinterpret_cast<uintptr_t>(a.vy) % 16 == 0 &&
           reinterpret_cast<uintptr_t>(a.vz) % 16 == 0;
}

template <bool PARETO, typename T, int U>
hipError_t launch_one(const ExactArgs &a, bool hi_uniform, hipStream_t stream)
{
    if (PARETO)
        return hi_uniform ? launch_exact<T, U>(exact_pareto_kernel<T, U, true>, a, stream)
                          : launch_exact<T, U>(exact_pareto_kernel<T, U, false>, a, stream);
    return hi_uniform ? launch_exact<T, U>(exact_t_kernel<T, U, true>, a, stream)
                      : launch_exact<T, U>(exact_t_kernel<T, U, false>, a, stream);
}

template <bool PARETO>
hipError_t launch_generator(int mode, const ExactArgs &args, hipStream_t stream)
{
    const bool vec = aligned16(args);
    const uint64_t per_thread = mode == kModeF64 ? (vec ? 2 : 1) : (vec ? 4 : 1);
    const size_t esz = mode == kModeF64 ? 8 : 4;
    // launches of at most 2^23 workgroups of 256 threads (2^31 work-items);
    // each starts on a multiple of the group size, so alignment carries over
    const uint64_t chunk = (1ull << 31) * per_thread;
    for (uint64_t first = 0; first < args.n; first += chunk) {
        ExactArgs a = args;
        a.first = first;
        a.n = args.n - first < chunk ? args.n - first : chunk;
        a.vx = static_cast<char *>(args.vx) + first * esz;
        a.vy = static_cast<char *>(args.vy) + first * esz;
        a.vz = static_cast<char *>(args.vz) + first * esz;
        a.iters = args.iters ? args.iters + first : nullptr;
        a.hi = static_cast<uint32_t>(first >> 32);
        const bool hi_uniform = (first >> 32) == ((first + a.n - 1) >> 32);
        hipError_t err;
        if (mode == kModeF64)
            err = vec ? launch_one<PARETO, double, 2>(a, hi_uniform, stream)
                      : launch_one<PARETO, double, 1>(a, hi_uniform, stream);
        else
            err = vec ? launch_one<PARETO, float, 4>(a, hi_uniform, stream)
                      : launch_one<PARETO, float, 1>(a, hi_uniform, stream);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_exact_t(int mode, const ExactArgs &args, hipStream_t stream)
{
    return launch_generator<false>(mode, args, stream);
}

hipError_t launch_exact_pareto(int mode, const ExactArgs &args, hipStream_t stream)
{
    return launch_generator<true>(mode, args, stream);
}

}  // namespace kappa
