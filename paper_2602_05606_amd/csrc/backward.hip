// backward.hip -- reparameterisation gradient of the approximate Kappa
// generator (Zenitani & Umeda, arXiv 2602.05606) with respect to kappa and
// theta, at fixed uniforms.
//
// Per particle the kernel regenerates the Philox block, redoes the inversion
// of Sec. 4, and differentiates it: v is linear in theta (Table 1), so
// dv/dtheta = v/theta; x = (V/theta)^2 is the root of P(x) = b x^2 + (a+cL) x
// + L (eq:v) with dP/dx = 2bx + a + cL = D, so dx/dkappa = -dP/dkappa / D with
// dP/dkappa = b' x^2 + (a' + c'L + cL') x + L'; L = -kappa* expm1(z) with
// z = -lT/kappa* and lT independent of kappa gives L' = -expm1(z) + z e^z;
// then dv/dkappa = v (dx/dkappa) / (2x).
//
// The kernel reads the upstream gradient (3 x sizeof(T) bytes per particle)
// and writes one pair of FP64 partial sums per block; a second one-block
// kernel adds the partials in a fixed order.
#include <cstdlib>
#include <mutex>

#include "kappa_device.hpp"
#include "kappa_internal.hpp"

namespace kappa {

namespace {

constexpr int kBwdBlock = 256;
constexpr int kBwdMaxGrid = 4096;

// Partial sums of kappa_sample_backward_noalloc: one FP64 pair per workgroup
// of the default grid (at most kBwdMaxGrid), 64 KiB per device, held from the
// library's load until the process ends.  Host code never passes this name
// to a kernel: it is a host-side stand-in for the device array, whose address
// on each device comes from hipGetSymbolAddress (backward_scratch).
static __device__ __align__(256) double scratch[2 * kBwdMaxGrid];
static_assert(sizeof(scratch) == KAPPA_BACKWARD_SCRATCH_BYTES, "the header states the scratch size");

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kScratchDevices] = {};

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Loads U consecutive values of T from p (aligned to U * sizeof(T) bytes, a
// multiple of 16) with 16-byte nontemporal loads: the upstream gradient is
// read once (1.2-1.4% faster than ordinary loads at 2^26 particles).
template <typename T, int U>
__device__ __forceinline__ void load_group(const T *p, T (&v)[U])
{
    static_assert((U * sizeof(T)) % 16 == 0, "vector loads need 16-byte groups");
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int c = 0; c < U / 4; ++c) {
            typedef float v4f __attribute__((ext_vector_type(4)));
            const v4f q = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(p) + c);
            v[4 * c] = q.x;
            v[4 * c + 1] = q.y;
            v[4 * c + 2] = q.z;
            v[4 * c + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int c = 0; c < U / 2; ++c) {
            typedef double v2d __attribute__((ext_vector_type(2)));
            const v2d q = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(p) + c);
            v[2 * c] = q.x;
            v[2 * c + 1] = q.y;
        }
    }
}

// dP/dkappa at the root x of P (eq:v differentiated at fixed U1), in FP64:
// b' x^2 + (a' + c' L + c L') x + L' with L' = z e^z - expm1(z).
__device__ __forceinline__ double dP_dkappa_f64(const InvF64 &inv, const SpeciesF64 &s, double x)
{
    const double dL = fma(inv.z, inv.ez, -inv.em1);
    return fma(fma(s.db, x, fma(s.c, dL, fma(s.dc, inv.L, s.da))), x, dL);
}

// 1/a for a positive normal a: the hardware estimate and two Newton steps
// (the error of the estimate squares with each step), within an ulp or two.
__device__ __forceinline__ double rcp_pos_f64(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    y = fma(y, fma(-a, y, 1.0), y);
    return fma(y, fma(-a, y, 1.0), y);
}

// dL/dkappa at fixed U1 in FP32: z e^z - expm1(z), z = w ln 2.  For z < 1/2
// the two terms cancel to z^2/2, so there it is taken as w^2 Q(w) with Q a
// degree-4 near-minimax fit of (z e^z - expm1(z)) / w^2 on [0, 1/(2 ln 2)]
// (Chebyshev nodes; 2.6e-7 relative with FP32 evaluation).
__device__ __forceinline__ float dL_dkappa_f32(const InvF32 &inv)
{
    const float w = inv.w;
    float q = fmaf(0x1.f58396p-11f, w, 0x1.558744p-8f);
    q = fmaf(q, w, 0x1.d9463cp-6f);
    q = fmaf(q, w, 0x1.c6ad82p-4f);
    q = fmaf(q, w, 0x1.ebfbe6p-3f);
    return w < kExp2m1Small ? (w * w) * q : fmaf(inv.z, inv.ez, -inv.em1);
}

// The generator's Philox block of particle counter_offset + j0 + k, as in the
// forward kernel: with HI_UNIFORM the launch's counters share their high word,
// taken from the kernel argument so that the first rounds run partly on the
// scalar unit, and the first product M_A (base + k) is one multiply-add; the
// words are the same.
template <bool HI_UNIFORM>
__device__ __forceinline__ Block4 bwd_block(const BwdArgs &a, uint64_t j0, int k)
{
    if constexpr (HI_UNIFORM) {
        const uint32_t base = static_cast<uint32_t>(a.counter_offset) + static_cast<uint32_t>(j0);
        const uint64_t pa1 = static_cast<uint64_t>(kMulA) * base + static_cast<uint64_t>(kMulA) * static_cast<uint32_t>(k);
        return philox4x32_10_lane(pa1, static_cast<uint32_t>(a.counter_offset >> 32), a.seg, 0, a.k0, a.k1);
    } else {
        return particle_block(a.counter_offset + j0 + k, a.seg, 0, a.k0, a.k1);
    }
}

template <int MODE, int U, bool VEC, bool HI_UNIFORM>
__global__ void __launch_bounds__(kBwdBlock) backward_kernel(BwdArgs a)
{
    using T = typename std::conditional<MODE == kModeF64, double, float>::type;
    const T *gx = static_cast<const T *>(a.gx);
    const T *gy = static_cast<const T *>(a.gy);
    const T *gz = static_cast<const T *>(a.gz);
    // Per particle, with sx = V / theta, g.d the upstream gradient along the
    // direction and dx/dkappa = -dP/dkappa / D: d(g.v)/dtheta = sx (g.d) and
    // d(g.v)/dkappa = -(theta / 2) (g.d) (dP/dkappa) / (sx D).  sum_s and sum_k
    // add sx (g.d) and (g.d) (dP/dkappa) / (sx D); their factors theta and
    // -theta/2 are applied once per thread.  acc_s and acc_k take theta times
    // dLoss/dtheta and dLoss/dkappa directly (the FP32 mode's FP64-tail
    // particles, and the block sums).
    double acc_k = 0.0, acc_s = 0.0, sum_k = 0.0, sum_s = 0.0;
    const float neg_dc_kstar = static_cast<float>(-a.s64.dc * a.s64.kstar);  // dc L = -dc kappa* expm1(z)
    const uint64_t ngroups = (a.n + U - 1) / U;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < ngroups; g += stride) {
        const uint64_t j0 = g * U;
        T ux[U], uy[U], uz[U];
        if (VEC && j0 + U <= a.n) {
            load_group<T, U>(gx + j0, ux);
            load_group<T, U>(gy + j0, uy);
            load_group<T, U>(gz + j0, uz);
        } else {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const bool in = j0 + k < a.n;
                ux[k] = in ? gx[j0 + k] : T(0);
                uy[k] = in ? gy[j0 + k] : T(0);
                uz[k] = in ? gz[j0 + k] : T(0);
            }
        }
        uint32_t tails = 0;
        float tail_dot[U];
        float grp_s = 0.0f, grp_k = 0.0f;  // FP32 sums of this group's U terms
#pragma unroll
        for (int k = 0; k < U; ++k) {
            tail_dot[k] = 0.0f;
            const Block4 b = bwd_block<HI_UNIFORM>(a, j0, k);
            if constexpr (MODE == kModeF64) {
                bool high;
                double u;
                speed_uniform_f64(b.r0, b.r3, high, u);
                const InvF64 inv = invert_f64(high, u, a.s64);
                const DirF64 d = direction_f64(b.r1, b.r2);
                const double sx = inv.sqrt_x();
                const double gd = fma(d.cz, uz[k], fma(d.cy, uy[k], d.cx * ux[k]));
                sum_s = fma(sx, gd, sum_s);
                sum_k = fma(gd * dP_dkappa_f64(inv, a.s64, sx * sx), rcp_pos_f64(sx * inv.D), sum_k);
            } else {
                bool high;
                float y1, d1;
                speed_uniform_f32(b.r0, b.r3, high, y1, d1);
                const InvF32 inv = invert_f32(high, y1, d1, a.s32);
                const DirF32 d = direction_f32(b.r1, b.r2);
                // g . direction with cy = sin(theta) cos(phi), cz = sin(theta) sin(phi)
                const float dot = fmaf(d.st, fmaf(d.cphi, uy[k], d.sphi * uz[k]), d.cx * ux[k]);
                // Every lane takes the FP32 terms (straight-line code over the U particles);
                // the rare tail lanes drop them and are redone in FP64 below.
                const bool tail = MODE == kModeF32 && in_fp64_tail(b.r0);
                tail_dot[k] = dot;
                tails |= static_cast<uint32_t>(tail) << k;
                const float sx = inv.sqrt_x();
                const float x = sx * sx;
                const float dL = dL_dkappa_f32(inv);
                const float dP = fmaf(fmaf(a.s32.db, x, fmaf(a.s32.c, dL, fmaf(neg_dc_kstar, inv.em1, a.s32.da))), x, dL);
                const float gd = tail ? 0.0f : dot;
                grp_s = fmaf(sx, gd, grp_s);
                grp_k = fmaf(gd * dP, __builtin_amdgcn_rcpf(sx * inv.D), grp_k);
            }
        }
        if constexpr (MODE != kModeF64) {
            sum_s += static_cast<double>(grp_s);
            sum_k += static_cast<double>(grp_k);
        }
        if constexpr (MODE == kModeF32) {
            // rare: 1 - U1 < 2^-20, the speed comes from the FP64 inversion
            if (__builtin_expect(tails != 0, 0)) {
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    if ((tails >> k) & 1u) {
                        const Block4 b = particle_block(a.counter_offset + j0 + k, a.seg, 0, a.k0, a.k1);
                        bool h64;
                        double u64;
                        speed_uniform_f64(b.r0, b.r3, h64, u64);
                        const InvF64 i64 = invert_f64(h64, u64, a.s64);
                        const double sx = i64.sqrt_x();
                        const double x = sx * sx;
                        // the sampler's output speed is the FP64 speed rounded to float
                        const double V = static_cast<double>(static_cast<float>(a.s64.theta * sx));
                        const double vg = V * static_cast<double>(tail_dot[k]);
                        acc_s += vg;
                        acc_k -= 0.5 * vg * dP_dkappa_f64(i64, a.s64, x) / (x * i64.D);
                    }
                }
            }
        }
    }
    acc_s = fma(sum_s, a.s64.theta, acc_s);
    acc_k = fma(sum_k, -0.5 * a.s64.theta, acc_k);
    // block reduction: waves, then LDS across the 4 waves, in a fixed order
    __shared__ double red[2][kBwdBlock / 64];
    acc_k = wave_sum(acc_k);
    acc_s = wave_sum(acc_s);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = acc_k;
        red[1][wave] = acc_s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sk = 0.0, ss = 0.0;
        for (int w = 0; w < kBwdBlock / 64; ++w) {
            sk += red[0][w];
            ss += red[1][w];
        }
        a.partials[2 * blockIdx.x] = sk;
        a.partials[2 * blockIdx.x + 1] = ss;
    }
}

constexpr int kFinBlock = 256;
constexpr int kFinBatch = kBwdMaxGrid / kFinBlock;  // partial pairs per thread in one pass of the default grid

// Adds the per-block partial pairs in a fixed order: each thread loads a batch
// of kFinBatch pairs (all loads in flight together) and sums them in index
// order, then the waves and the 4 waves of the block are summed as in the
// main kernel.
__global__ void __launch_bounds__(kFinBlock) backward_finalize(const double *partials, int nblocks,
                                                               double inv_theta, double *grad)
{
    double sk = 0.0, ss = 0.0;
    for (int base = 0; base < nblocks; base += kFinBlock * kFinBatch) {
        double pk[kFinBatch], ps[kFinBatch];
#pragma unroll
        for (int i = 0; i < kFinBatch; ++i) {
            const int j = base + i * kFinBlock + static_cast<int>(threadIdx.x);
            const bool in = j < nblocks;
            pk[i] = in ? partials[2 * j] : 0.0;
            ps[i] = in ? partials[2 * j + 1] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kFinBatch; ++i) {
            sk += pk[i];
            ss += ps[i];
        }
    }
    __shared__ double red[2][kFinBlock / 64];
    sk = wave_sum(sk);
    ss = wave_sum(ss);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = sk;
        red[1][wave] = ss;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tk = 0.0, ts = 0.0;
        for (int w = 0; w < kFinBlock / 64; ++w) {
            tk += red[0][w];
            ts += red[1][w];
        }
        grad[0] = tk;
        grad[1] = ts * inv_theta;
    }
}

constexpr int unroll_for(int mode)
{
    return mode == kModeF64 ? 2 : 4;
}

template <int MODE, bool HI_UNIFORM>
hipError_t launch_mode(const BwdArgs &a, bool vec, hipStream_t stream)
{
    constexpr int U = unroll_for(MODE);
    const int grid = backward_grid(a.n);
    log_launch("backward_kernel", MODE, a.n, Shape{kBwdBlock, vec ? U : 1, grid}, stream);
    if (vec)
        hipLaunchKernelGGL((backward_kernel<MODE, U, true, HI_UNIFORM>), dim3(grid), dim3(kBwdBlock), 0, stream, a);
    else
        hipLaunchKernelGGL((backward_kernel<MODE, U, false, HI_UNIFORM>), dim3(grid), dim3(kBwdBlock), 0, stream, a);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(const BwdArgs &a, bool vec, hipStream_t stream)
{
    const bool uniform_hi = a.n == 0 || (a.counter_offset >> 32) == ((a.counter_offset + a.n - 1) >> 32);
    return uniform_hi ? launch_mode<MODE, true>(a, vec, stream) : launch_mode<MODE, false>(a, vec, stream);
}

}  // namespace

// Fixed for a given n (independent of the device) so the summation order, and
// hence the result, is reproducible.  KAPPA_BACKWARD_GRID=<blocks> overrides
// the cap for tuning (0: one thread per group, up to 2^20 blocks); a
// different grid changes only the order of the FP64 sums.
int backward_grid(uint64_t n)
{
    const uint64_t per_block = static_cast<uint64_t>(kBwdBlock) * 4;
    const uint64_t need = (n + per_block - 1) / per_block;
    uint64_t cap = kBwdMaxGrid;
    if (const char *env = std::getenv("KAPPA_BACKWARD_GRID")) {
        const long v = std::strtol(env, nullptr, 10);
        if (v == 0) cap = 1u << 20;
        else if (v > 0 && v <= (1 << 20)) cap = static_cast<uint64_t>(v);
    }
    return static_cast<int>(need < 1 ? 1 : (need > cap ? cap : need));
}

size_t backward_scratch_bytes() { return sizeof(scratch); }

hipError_t backward_scratch(double **ptr)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        // with dev current: each device holds its own copy of the array
        void *p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess) return err;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_backward(int mode, const BwdArgs &args, double *grad, hipStream_t stream)
{
    const size_t esz = mode == kModeF64 ? 8 : 4;
    const bool vec = (reinterpret_cast<uintptr_t>(args.gx) % (esz * unroll_for(mode)) == 0) &&
                     (reinterpret_cast<uintptr_t>(args.gy) % (esz * unroll_for(mode)) == 0) &&
                     (reinterpret_cast<uintptr_t>(args.gz) % (esz * unroll_for(mode)) == 0);
    hipError_t err;
    switch (mode) {
    case kModeF64: err = launch_mode<kModeF64>(args, vec, stream); break;
    case kModeF32: err = launch_mode<kModeF32>(args, vec, stream); break;
    case kModeF32NoTail: err = launch_mode<kModeF32NoTail>(args, vec, stream); break;
    default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(backward_finalize, dim3(1), dim3(kFinBlock), 0, stream, args.partials,
                       backward_grid(args.n), 1.0 / args.s64.theta, grad);
    return hipGetLastError();
}

}  // namespace kappa
