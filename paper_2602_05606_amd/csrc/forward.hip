// forward.hip -- single-species forward kernels of the approximate Kappa
// generator (Table 1 of Zenitani & Umeda, arXiv 2602.05606) for gfx950, plus
// the raw Philox dump and the store/copy measurement probes.
//
// The forward pass is a pure streaming write: 3 x sizeof(T) bytes per particle
// and no reads.  Each thread produces `U` consecutive particles entirely in
// registers and writes them with one 16-byte store per output array.
#include <cstdio>
#include <cstdlib>

#include "kappa_device.hpp"
#include "kappa_internal.hpp"
#include "kappa_store.hpp"

namespace kappa {

// Philox block of particle counter_offset + j0 + k.  When the launch's counter
// range stays inside one block of 2^32 (HI_UNIFORM, nearly every launch), the
// counter's high word is the same for all its particles and comes from the
// kernel argument, the first rounds run partly on the scalar unit, and the low
// word base + k of the group's particles never carries, so its first product
// M_A (base + k) = M_A base + M_A k is one multiply-add.  The words are the same.
template <bool HI_UNIFORM>
__device__ __forceinline__ Block4 fwd_block(const FwdArgs &a, uint64_t j0, int k)
{
    if constexpr (HI_UNIFORM) {
        const uint32_t base = static_cast<uint32_t>(a.counter_offset) + static_cast<uint32_t>(j0);
        const uint64_t pa1 = static_cast<uint64_t>(kMulA) * base + static_cast<uint64_t>(kMulA) * static_cast<uint32_t>(k);
        return philox4x32_10_lane(pa1, static_cast<uint32_t>(a.counter_offset >> 32), a.seg, 0, a.k0, a.k1);
    } else {
        return particle_block(a.counter_offset + j0 + k, a.seg, 0, a.k0, a.k1);
    }
}

// CLOCK = true is the clock probe's instantiation: the same kernel, plus
// per-workgroup stamps of the shader-clock counter (s_memtime, core clock
// cycles) and the constant-rate counter (s_memrealtime) at entry and exit of
// wave 0, written by its thread 0 to stamps[4w .. 4w+3] for workgroup w.
// Product launches instantiate CLOCK = false and pass no stamps.
template <int MODE, int U, bool HI_UNIFORM, bool CLOCK>
__global__ void __launch_bounds__(256) forward_kernel(FwdArgs a, uint64_t *stamps)
{
    using T = typename std::conditional<MODE == kModeF64, double, float>::type;
    if constexpr (CLOCK) {
        // stored at once, so that no registers are held across the kernel
        const uint64_t clk0 = __builtin_amdgcn_s_memtime();
        const uint64_t rt0 = __builtin_amdgcn_s_memrealtime();
        if (threadIdx.x == 0) {
            stamps[4 * static_cast<uint64_t>(blockIdx.x)] = clk0;
            stamps[4 * static_cast<uint64_t>(blockIdx.x) + 1] = rt0;
        }
    }
    T *vx = static_cast<T *>(a.vx);
    T *vy = static_cast<T *>(a.vy);
    T *vz = static_cast<T *>(a.vz);
    // One group of U particles per thread and no loop: the launcher's grid
    // covers every group, and with no loop the compiler keeps no constants
    // live across one (on the FP64 path that spared every SGPR spill).
    const uint64_t ngroups = (a.n + U - 1) / U;
    if (const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < ngroups) {
        const uint64_t j0 = g * U;
        T x[U], y[U], z[U];
        uint32_t tails = 0;
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const Block4 b = fwd_block<HI_UNIFORM>(a, j0, k);
            if constexpr (MODE == kModeF64) {
                particle_f64(b, a.s64, x[k], y[k], z[k]);
            } else {
                particle_f32(b, a.s32, x[k], y[k], z[k]);
                if constexpr (MODE == kModeF32) tails |= static_cast<uint32_t>(in_fp64_tail(b.r0)) << k;
            }
        }
        if constexpr (MODE == kModeF32) {
            if (__builtin_expect(tails != 0, 0)) {
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    if ((tails >> k) & 1u) {
                        const Block4 b = particle_block(a.counter_offset + j0 + k, a.seg, 0, a.k0, a.k1);
                        tail_particle_f32(b, a.s64, x[k], y[k], z[k]);
                    }
                }
            }
        }
        if (j0 + U <= a.n) {
            store_group<T, U>(vx + j0, x);
            store_group<T, U>(vy + j0, y);
            store_group<T, U>(vz + j0, z);
        } else {
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (j0 + k < a.n) {
                    vx[j0 + k] = x[k];
                    vy[j0 + k] = y[k];
                    vz[j0 + k] = z[k];
                }
            }
        }
    }
    if constexpr (CLOCK) {
        const uint64_t clk1 = __builtin_amdgcn_s_memtime();
        const uint64_t rt1 = __builtin_amdgcn_s_memrealtime();
        if (threadIdx.x == 0) {
            stamps[4 * static_cast<uint64_t>(blockIdx.x) + 2] = clk1;
            stamps[4 * static_cast<uint64_t>(blockIdx.x) + 3] = rt1;
        }
    }
}

namespace {

template <int MODE, bool HI_UNIFORM>
hipError_t launch_mode(const Shape &sh, const FwdArgs &a, hipStream_t stream)
{
    log_launch("forward_kernel", MODE, a.n, sh, stream);
    dim3 grid(sh.grid), block(sh.block);
    switch (sh.unroll) {
    case 1: hipLaunchKernelGGL((forward_kernel<MODE, 1, HI_UNIFORM, false>), grid, block, 0, stream, a, nullptr); break;
    case 2: hipLaunchKernelGGL((forward_kernel<MODE, 2, HI_UNIFORM, false>), grid, block, 0, stream, a, nullptr); break;
    case 4: hipLaunchKernelGGL((forward_kernel<MODE, 4, HI_UNIFORM, false>), grid, block, 0, stream, a, nullptr); break;
    case 8: hipLaunchKernelGGL((forward_kernel<MODE, 8, HI_UNIFORM, false>), grid, block, 0, stream, a, nullptr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(const Shape &sh, const FwdArgs &a, hipStream_t stream)
{
    const bool uniform_hi = a.n == 0 || (a.counter_offset >> 32) == ((a.counter_offset + a.n - 1) >> 32);
    return uniform_hi ? launch_mode<MODE, true>(sh, a, stream) : launch_mode<MODE, false>(sh, a, stream);
}

// Clock probe: the kernel of the default vector-store shape (unroll 2 for
// FP64, 4 otherwise) with stamps; stamps holds 4 entries per workgroup.
template <int MODE>
hipError_t launch_clock_mode(const Shape &sh, const FwdArgs &a, uint64_t *stamps, hipStream_t stream)
{
    constexpr int U = MODE == kModeF64 ? 2 : 4;
    if (sh.unroll != U) return hipErrorInvalidValue;
    dim3 grid(sh.grid), block(sh.block);
    const bool uniform_hi = a.n == 0 || (a.counter_offset >> 32) == ((a.counter_offset + a.n - 1) >> 32);
    if (uniform_hi)
        hipLaunchKernelGGL((forward_kernel<MODE, U, true, true>), grid, block, 0, stream, a, stamps);
    else
        hipLaunchKernelGGL((forward_kernel<MODE, U, false, true>), grid, block, 0, stream, a, stamps);
    return hipGetLastError();
}

}  // namespace

int forward_default_unroll(int mode) { return mode == kModeF64 ? 2 : 4; }

hipError_t launch_forward_clock(int mode, const Shape &shape, const FwdArgs &args, uint64_t *stamps,
                                hipStream_t stream)
{
    switch (mode) {
    case kModeF64: return launch_clock_mode<kModeF64>(shape, args, stamps, stream);
    case kModeF32: return launch_clock_mode<kModeF32>(shape, args, stamps, stream);
    case kModeF32NoTail: return launch_clock_mode<kModeF32NoTail>(shape, args, stamps, stream);
    default: return hipErrorInvalidValue;
    }
}

// One thread per group of particles: consecutive workgroups write
// consecutive address ranges, which measured faster for streaming stores on
// gfx950 than a grid capped at a few workgroups per CU striding over the
// arrays.  A launch holds at most max_grid workgroups (2^23, so that its
// work-items fit the dispatch packet's 32-bit grid size; the environment
// variable KAPPA_FORWARD_MAX_GRID lowers it, for tests): launch_forward splits
// larger calls into consecutive chunks.  KAPPA_FORWARD_SHAPE="block,unroll"
// overrides the shape for tuning (block in {64,128,256}, unroll in {1,2,4,8}).
// Results never depend on either.
uint64_t forward_max_grid()
{
    uint64_t cap = 1ull << 23;
    if (const char *env = std::getenv("KAPPA_FORWARD_MAX_GRID")) {
        const long long v = std::strtoll(env, nullptr, 10);
        if (v > 0 && v < static_cast<long long>(cap)) cap = static_cast<uint64_t>(v);
    }
    return cap;
}

Shape forward_shape(int mode, uint64_t n, bool vec, bool tuned)
{
    Shape s;
    s.block = 256;
    s.unroll = vec ? forward_default_unroll(mode) : 1;
    Shape t{};
    if (const char *env = std::getenv("KAPPA_FORWARD_SHAPE")) {
        int b = 0, u = 0;
        if (std::sscanf(env, "%d,%d", &b, &u) == 2 && (b == 64 || b == 128 || b == 256) &&
            (u == 1 || u == 2 || u == 4 || u == 8)) {
            s.block = b;
            s.unroll = vec ? u : 1;
        }
    } else if (tuned && vec && forward_tuned(mode, n, t) && (t.block == 64 || t.block == 128 || t.block == 256) &&
               (t.unroll == 1 || t.unroll == 2 || t.unroll == 4 || t.unroll == 8)) {
        // a shape kappa_sample_autotune chose for this precision and size
        s.block = t.block;
        s.unroll = t.unroll;
    }
    const uint64_t groups = (n + s.unroll - 1) / s.unroll;
    const uint64_t need = (groups + s.block - 1) / s.block;
    const uint64_t cap = forward_max_grid();
    s.grid = static_cast<int>(need < cap ? (need > 0 ? need : 1) : cap);
    return s;
}

hipError_t launch_forward(int mode, const Shape &shape, bool vec, const FwdArgs &args, hipStream_t stream)
{
    Shape sh = shape;
    if (!vec) sh.unroll = 1;
    // chunks of at most sh.grid workgroups; each starts on a multiple of
    // block * unroll particles, so 16-byte alignment carries over
    const uint64_t chunk = static_cast<uint64_t>(sh.grid) * sh.block * sh.unroll;
    const size_t esz = mode == kModeF64 ? 8 : 4;
    for (uint64_t first = 0; first < args.n || first == 0; first += chunk) {
        FwdArgs a = args;
        a.n = args.n - first < chunk ? args.n - first : chunk;
        a.counter_offset = args.counter_offset + first;
        a.vx = static_cast<char *>(args.vx) + first * esz;
        a.vy = static_cast<char *>(args.vy) + first * esz;
        a.vz = static_cast<char *>(args.vz) + first * esz;
        Shape c = sh;
        const uint64_t need = ((a.n + sh.unroll - 1) / sh.unroll + sh.block - 1) / sh.block;
        c.grid = static_cast<int>(need > 0 ? need : 1);
        hipError_t err;
        switch (mode) {
        case kModeF64: err = launch_mode<kModeF64>(c, a, stream); break;
        case kModeF32: err = launch_mode<kModeF32>(c, a, stream); break;
        case kModeF32NoTail: err = launch_mode<kModeF32NoTail>(c, a, stream); break;
        default: return hipErrorInvalidValue;
        }
        if (err != hipSuccess) return err;
        if (args.n - first <= chunk) break;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Raw Philox dump: out[4j .. 4j+3] = block of particle counter_offset + j.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) philox_kernel(uint64_t n, uint64_t off, uint32_t seg, uint32_t draw,
                                                     uint32_t k0, uint32_t k1, uint4 *out)
{
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += stride) {
        const Block4 b = particle_block(off + j, seg, draw, k0, k1);
        out[j] = make_uint4(b.r0, b.r1, b.r2, b.r3);
    }
}

hipError_t launch_philox(uint64_t n, uint64_t counter_offset, uint32_t seg, uint32_t draw, uint32_t k0, uint32_t k1,
                         uint32_t *out, hipStream_t stream)
{
    const uint64_t need = (n + 255) / 256;
    const uint64_t cap = static_cast<uint64_t>(device_cu_count()) * 16;
    const int grid = static_cast<int>(need < cap ? need : cap);
    hipLaunchKernelGGL(philox_kernel, dim3(grid), dim3(256), 0, stream, n, counter_offset, seg, draw, k0, k1,
                       reinterpret_cast<uint4 *>(out));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Store-only probe: the generator's store path with the arithmetic removed.
// ---------------------------------------------------------------------------
template <typename T, int U>
__global__ void __launch_bounds__(256) fill_kernel(uint64_t n, T *vx, T *vy, T *vz)
{
    const uint64_t ngroups = (n + U - 1) / U;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < ngroups; g += stride) {
        const uint64_t j0 = g * U;
        T x[U], y[U], z[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            x[k] = T(1);
            y[k] = T(2);
            z[k] = T(3);
        }
        if (j0 + U <= n) {
            store_group<T, U>(vx + j0, x);
            store_group<T, U>(vy + j0, y);
            store_group<T, U>(vz + j0, z);
        } else {
            for (int k = 0; k < U; ++k) {
                if (j0 + k < n) {
                    vx[j0 + k] = x[k];
                    vy[j0 + k] = y[k];
                    vz[j0 + k] = z[k];
                }
            }
        }
    }
}

hipError_t launch_fill_probe(int mode, uint64_t n, void *vx, void *vy, void *vz, hipStream_t stream)
{
    const Shape s = forward_shape(mode, n, true, false);
    if (mode == kModeF64) {
        hipLaunchKernelGGL((fill_kernel<double, 2>), dim3(s.grid), dim3(s.block), 0, stream, n,
                           static_cast<double *>(vx), static_cast<double *>(vy), static_cast<double *>(vz));
    } else {
        hipLaunchKernelGGL((fill_kernel<float, 4>), dim3(s.grid), dim3(s.block), 0, stream, n,
                           static_cast<float *>(vx), static_cast<float *>(vy), static_cast<float *>(vz));
    }
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) copy_kernel(const float4 *src, float4 *dst, uint64_t n16)
{
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n16; j += stride)
        dst[j] = src[j];
}

hipError_t launch_copy_probe(const void *src, void *dst, uint64_t bytes, hipStream_t stream)
{
    const uint64_t n16 = bytes / 16;
    const uint64_t need = (n16 + 255) / 256;
    const uint64_t cap = static_cast<uint64_t>(device_cu_count()) * 16;
    const int grid = static_cast<int>(need < cap ? (need > 0 ? need : 1) : cap);
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, stream, static_cast<const float4 *>(src),
                       static_cast<float4 *>(dst), n16);
    return hipGetLastError();
}

}  // namespace kappa
