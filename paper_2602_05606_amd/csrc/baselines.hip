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

namespace kappa {

namespace {

constexpr uint32_t kMaxIters = 64;

template <typename T>
__device__ __forceinline__ T unit_open(uint32_t r);  // (r + 1/2) 2^-32

template <>
__device__ __forceinline__ double unit_open<double>(uint32_t r)
{
    return (static_cast<double>(r) + 0.5) * 0x1p-32;
}

template <>
__device__ __forceinline__ float unit_open<float>(uint32_t r)
{
    return (static_cast<float>(r >> 8) + 0.5f) * 0x1p-24f;
}

__device__ __forceinline__ double log_t(double x) { return log(x); }
__device__ __forceinline__ float log_t(float x) { return logf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(x); }
__device__ __forceinline__ void sincospi_t(double x, double *s, double *c) { sincospi(x, s, c); }
__device__ __forceinline__ void sincospi_t(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ double exp_t(double x) { return exp(x); }
__device__ __forceinline__ float exp_t(float x) { return expf(x); }
__device__ __forceinline__ double expm1_t(double x) { return expm1(x); }
__device__ __forceinline__ float expm1_t(float x) { return expm1f(x); }

// Box-Muller (Box & Muller 1958): two uniforms -> two independent normals.
template <typename T>
__device__ __forceinline__ void box_muller(uint32_t ra, uint32_t rb, T &z0, T &z1)
{
    const T rad = sqrt_t(T(-2) * log_t(unit_open<T>(ra)));
    T s, c;
    sincospi_t(T(2) * unit_open<T>(rb), &s, &c);
    z0 = rad * c;
    z1 = rad * s;
}

// Kappa as a multivariate t with 2 kappa - 1 degrees of freedom:
// v = theta sqrt(kappa / (2 G)) (Z1, Z2, Z3), G ~ Gamma(kappa - 1/2), drawn
// with Marsaglia & Tsang (2000) (shape kappa - 1/2 > 1, so no boost step).
template <typename T>
__global__ void __launch_bounds__(256) exact_t_kernel(ExactArgs a)
{
    T *vx = static_cast<T *>(a.vx);
    T *vy = static_cast<T *>(a.vy);
    T *vz = static_cast<T *>(a.vz);
    const T shape = static_cast<T>(a.kappa - 0.5);
    const T d = shape - T(1) / T(3);
    const T cmt = T(1) / sqrt_t(T(9) * d);
    const T scale = static_cast<T>(a.theta * sqrt(0.5 * a.kappa));
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const Block4 b0 = particle_block(i, 0, 0, a.k0, a.k1);
        T z1, z2, z3, spare;
        box_muller<T>(b0.r0, b0.r1, z1, z2);
        box_muller<T>(b0.r2, b0.r3, z3, spare);
        (void)spare;
        T g = d;
        uint32_t t = 1;
        for (; t <= kMaxIters; ++t) {
            const Block4 bt = particle_block(i, 0, t, a.k0, a.k1);
            T x, unused;
            box_muller<T>(bt.r0, bt.r1, x, unused);
            (void)unused;
            const T w = T(1) + cmt * x;
            if (w <= T(0)) continue;
            const T v = w * w * w;
            const T u = unit_open<T>(bt.r2);
            const T x2 = x * x;
            g = d * v;
            if (u < T(1) - T(0.0331) * x2 * x2) break;
            if (log_t(u) < T(0.5) * x2 + d * (T(1) - v + log_t(v))) break;
        }
        const T f = scale / sqrt_t(g);
        vx[i] = f * z1;
        vy[i] = f * z2;
        vz[i] = f * z3;
        if (a.iters) a.iters[i] = t > kMaxIters ? kMaxIters : t;
    }
}

// Speed by rejection from a Type II Pareto (Lomax) proposal with index
// n = kappa/2: s^2 = kappa (W^{-2/kappa} - 1), W uniform, proposal density
// q(s) = s (1 + s^2/kappa)^{-(kappa/2 + 1)} against the target
// f(s) ~ s^2 (1 + s^2/kappa)^{-(kappa+1)} of eq:kappa.  f/q is proportional
// to s (1 + s^2/kappa)^{-kappa/2} = s W, which peaks at s^2 = kappa/(kappa-1);
// the acceptance test is U <= s W (kappa/(kappa-1))^{(kappa-1)/2}.  Its
// acceptance rate is the p2 of eq:pareto_eff.  Direction from the two
// uniforms drawn outside the loop, as in Table 1.
template <typename T>
__global__ void __launch_bounds__(256) exact_pareto_kernel(ExactArgs a)
{
    T *vx = static_cast<T *>(a.vx);
    T *vy = static_cast<T *>(a.vy);
    T *vz = static_cast<T *>(a.vz);
    const T kap = static_cast<T>(a.kappa);
    const T neg2k = static_cast<T>(-2.0 / a.kappa);
    const T ln_m = static_cast<T>(0.5 * (a.kappa - 1.0) * log(a.kappa / (a.kappa - 1.0)));
    const T theta = static_cast<T>(a.theta);
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const Block4 b0 = particle_block(i, 0, 0, a.k0, a.k1);
        T s = T(0);
        uint32_t t = 1;
        for (; t <= kMaxIters; ++t) {
            const Block4 bt = particle_block(i, 0, t, a.k0, a.k1);
            const T lw = log_t(unit_open<T>(bt.r0));
            s = sqrt_t(kap * expm1_t(neg2k * lw));
            const T u = unit_open<T>(bt.r1);
            if (log_t(u) <= log_t(s) + lw + ln_m) break;
        }
        const T ct = T(2) * unit_open<T>(b0.r1) - T(1);
        const T st = sqrt_t((T(1) - ct) * (T(1) + ct));
        T sp, cp;
        sincospi_t(T(2) * unit_open<T>(b0.r2), &sp, &cp);
        const T V = theta * s;
        vx[i] = V * ct;
        vy[i] = V * st * cp;
        vz[i] = V * st * sp;
        if (a.iters) a.iters[i] = t > kMaxIters ? kMaxIters : t;
    }
}

int exact_grid(uint64_t n)
{
    const uint64_t need = (n + 255) / 256;
    const uint64_t cap = static_cast<uint64_t>(device_cu_count()) * 16;
    return static_cast<int>(need < cap ? (need > 0 ? need : 1) : cap);
}

}  // namespace

hipError_t launch_exact_t(int mode, const ExactArgs &args, hipStream_t stream)
{
    const int grid = exact_grid(args.n);
    if (mode == kModeF64)
        hipLaunchKernelGGL(exact_t_kernel<double>, dim3(grid), dim3(256), 0, stream, args);
    else
        hipLaunchKernelGGL(exact_t_kernel<float>, dim3(grid), dim3(256), 0, stream, args);
    return hipGetLastError();
}

hipError_t launch_exact_pareto(int mode, const ExactArgs &args, hipStream_t stream)
{
    const int grid = exact_grid(args.n);
    if (mode == kModeF64)
        hipLaunchKernelGGL(exact_pareto_kernel<double>, dim3(grid), dim3(256), 0, stream, args);
    else
        hipLaunchKernelGGL(exact_pareto_kernel<float>, dim3(grid), dim3(256), 0, stream, args);
    return hipGetLastError();
}

}  // namespace kappa
