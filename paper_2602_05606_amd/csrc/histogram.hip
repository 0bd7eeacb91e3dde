// histogram.hip -- speed histogram of sampled velocities, the data of the
// paper's Monte Carlo relative-entropy test (Sec. 5, second test, eq:KL):
// counts of |v| in bins of width w theta, plus one overflow bin.
//
// Bin membership is decided without division or square root: bin k holds the
// particles with edge2[k] <= |v|^2 < edge2[k+1], where |v|^2 = (vx^2 + vy^2)
// + vz^2 in the data's precision and edge2[k] = (k w theta)^2 computed in
// FP64 and rounded once to that precision.  Any implementation that follows
// these IEEE operations gets the same counts.
//
// Each block keeps one sub-histogram per wave in LDS (fewer atomic
// collisions), walks the arrays with a grid stride (16-byte loads when the
// arrays are 16-byte aligned), and adds its counts to the caller's uint64
// counters with one atomic per bin at the end.
#include "kappa_internal.hpp"

namespace kappa {

namespace {

constexpr int kHistBlock = 256;
constexpr int kHistWaves = kHistBlock / 64;

// Bin of one squared speed: an estimate from sqrt, then the exact decision
// against the squared edges.
template <typename T>
__device__ __forceinline__ uint32_t bin_of(T s2, const T *edge2, T inv_w, uint32_t nbins)
{
    const T est = sqrt(s2) * inv_w;
    uint32_t k = est < static_cast<T>(nbins) ? static_cast<uint32_t>(est) : nbins;
    while (k > 0 && s2 < edge2[k]) --k;
    while (k < nbins && s2 >= edge2[k + 1]) ++k;
    return k;
}

template <typename T>
struct Vec;
template <>
struct Vec<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <>
struct Vec<double> {
    using type = double2;
    static constexpr int n = 2;
};

// VEC: 16-byte nontemporal loads of Vec<T>::n particles per array (outputs
// 16-byte aligned; each velocity is read once: 7% faster than ordinary loads
// at 1e8 FP32 particles); otherwise one particle per load.  The counts do not
// depend on it.
template <typename T, bool VEC>
__global__ void __launch_bounds__(kHistBlock) histogram_kernel(const T *vx, const T *vy, const T *vz, uint64_t n,
                                                               double width, uint32_t nbins,
                                                               unsigned long long *counts)
{
    extern __shared__ unsigned char smem[];
    T *edge2 = reinterpret_cast<T *>(smem);                                     // nbins + 1
    uint32_t *bins = reinterpret_cast<uint32_t *>(smem + sizeof(T) * (nbins + 1));  // kHistWaves x (nbins + 1)
    const uint32_t nb = nbins + 1;
    for (uint32_t k = threadIdx.x; k < nb; k += kHistBlock) {
        const double e = static_cast<double>(k) * width;
        edge2[k] = static_cast<T>(e * e);
    }
    for (uint32_t k = threadIdx.x; k < kHistWaves * nb; k += kHistBlock) bins[k] = 0u;
    __syncthreads();
    uint32_t *mine = bins + (threadIdx.x >> 6) * nb;
    const T inv_w = static_cast<T>(1.0 / width);
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    const uint64_t first = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if constexpr (VEC) {
        using V = typename Vec<T>::type;
        constexpr int W = Vec<T>::n;
        const uint64_t ngroups = n / W;
        for (uint64_t g = first; g < ngroups; g += stride) {
            typedef T vt __attribute__((ext_vector_type(W)));
            const vt xv = __builtin_nontemporal_load(reinterpret_cast<const vt *>(vx) + g);
            const vt yv = __builtin_nontemporal_load(reinterpret_cast<const vt *>(vy) + g);
            const vt zv = __builtin_nontemporal_load(reinterpret_cast<const vt *>(vz) + g);
            V x, y, z;
            __builtin_memcpy(&x, &xv, sizeof(V));
            __builtin_memcpy(&y, &yv, sizeof(V));
            __builtin_memcpy(&z, &zv, sizeof(V));
            T xs[W], ys[W], zs[W];
            __builtin_memcpy(xs, &x, sizeof(V));
            __builtin_memcpy(ys, &y, sizeof(V));
            __builtin_memcpy(zs, &z, sizeof(V));
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const T s2 = (xs[k] * xs[k] + ys[k] * ys[k]) + zs[k] * zs[k];
                atomicAdd(&mine[bin_of(s2, edge2, inv_w, nbins)], 1u);
            }
        }
        // the ragged tail (fewer than W particles)
        for (uint64_t j = ngroups * W + first; j < n; j += stride) {
            const T s2 = (vx[j] * vx[j] + vy[j] * vy[j]) + vz[j] * vz[j];
            atomicAdd(&mine[bin_of(s2, edge2, inv_w, nbins)], 1u);
        }
    } else {
        for (uint64_t j = first; j < n; j += stride) {
            const T x = vx[j], y = vy[j], z = vz[j];
            const T s2 = (x * x + y * y) + z * z;
            atomicAdd(&mine[bin_of(s2, edge2, inv_w, nbins)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nb; k += kHistBlock) {
        unsigned long long c = 0;
        for (int w = 0; w < kHistWaves; ++w) c += bins[w * nb + k];
        if (c) atomicAdd(&counts[k], c);
    }
}

}  // namespace

size_t histogram_lds_bytes(int mode, uint32_t nbins)
{
    const size_t esz = mode == kModeF64 ? 8 : 4;
    return esz * (nbins + 1) + sizeof(uint32_t) * kHistWaves * (nbins + 1);
}

hipError_t launch_histogram(int mode, const void *vx, const void *vy, const void *vz, uint64_t n, double width,
                            uint32_t nbins, uint64_t *counts, hipStream_t stream)
{
    const uint64_t need = (n + kHistBlock - 1) / kHistBlock;
    const uint64_t cap = static_cast<uint64_t>(device_cu_count()) * 8;
    const int grid = static_cast<int>(need < cap ? (need > 0 ? need : 1) : cap);
    const size_t lds = histogram_lds_bytes(mode, nbins);
    auto *c = reinterpret_cast<unsigned long long *>(counts);
    auto a16 = [](const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
    const bool vec = a16(vx) && a16(vy) && a16(vz);
    if (mode == kModeF64) {
        auto *x = static_cast<const double *>(vx), *y = static_cast<const double *>(vy),
             *z = static_cast<const double *>(vz);
        if (vec)
            hipLaunchKernelGGL((histogram_kernel<double, true>), dim3(grid), dim3(kHistBlock), lds, stream, x, y, z, n,
                               width, nbins, c);
        else
            hipLaunchKernelGGL((histogram_kernel<double, false>), dim3(grid), dim3(kHistBlock), lds, stream, x, y, z,
                               n, width, nbins, c);
    } else {
        auto *x = static_cast<const float *>(vx), *y = static_cast<const float *>(vy),
             *z = static_cast<const float *>(vz);
        if (vec)
            hipLaunchKernelGGL((histogram_kernel<float, true>), dim3(grid), dim3(kHistBlock), lds, stream, x, y, z, n,
                               width, nbins, c);
        else
            hipLaunchKernelGGL((histogram_kernel<float, false>), dim3(grid), dim3(kHistBlock), lds, stream, x, y, z,
                               n, width, nbins, c);
    }
    return hipGetLastError();
}

}  // namespace kappa
