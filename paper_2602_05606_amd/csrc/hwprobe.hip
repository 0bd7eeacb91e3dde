// hwprobe.hip -- measurement probes of the gfx950 instructions the FP32
// generator rests on: the issue cost of an instruction class under saturation
// (the basis of the VALU-issue roofline) and the accuracy of the hardware
// transcendentals (the basis of the FP32 inversion's error budget).
#include "kappa_internal.hpp"

namespace kappa {

namespace {

constexpr int kIssueIters = 4096;
constexpr int kIssueChains = 8;

// Every lane runs kIssueChains independent chains of one instruction class
// for kIssueIters steps; one round of 8 waves per SIMD (8 workgroups of 4
// waves per CU, all resident at once), so the issue port, not latency, sets
// the pace, and the launch is long against its ramp.  Wave w records its
// core-clock cycles (s_memtime) and constant-rate ticks (s_memrealtime) from
// start to end.  Class 5 mixes kinds: each chain step is one v_log_f32 on one
// register and three dependent v_fma_f32 on another, four instructions, to see
// whether the transcendental unit runs beside full-rate work.  Class 6 is
// v_fma_f32 with two VGPR operands and a literal, class 0 with three VGPRs.
template <int OP>
__global__ void __launch_bounds__(256) issue_kernel(float *sink, uint64_t *stamps)
{
    const uint64_t c0 = __builtin_amdgcn_s_memtime();
    const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    const uint32_t t = threadIdx.x;
    float f[kIssueChains], g[kIssueChains], fa[kIssueChains], fb[kIssueChains];
    double d[kIssueChains], da[kIssueChains];
    uint32_t u[kIssueChains], w[kIssueChains];
#pragma unroll
    for (int c = 0; c < kIssueChains; ++c) {
        f[c] = 1.0f + 0.001f * static_cast<float>((t + c) & 31);
        g[c] = f[c];
        fa[c] = 0.999f - 1e-6f * static_cast<float>(t & 7);
        fb[c] = 1e-4f * static_cast<float>((t >> 3) & 3) + 1e-5f * static_cast<float>(c);
        d[c] = f[c];
        da[c] = fa[c];
        u[c] = t * 2654435761u + static_cast<uint32_t>(c);
        w[c] = t * 40503u + 77u * static_cast<uint32_t>(c) + 0xD2511F53u;
    }
    for (int it = 0; it < kIssueIters; ++it) {
#pragma unroll
        for (int c = 0; c < kIssueChains; ++c) {
            if constexpr (OP == 0) f[c] = __builtin_fmaf(f[c], fa[c], fb[c]);
            if constexpr (OP == 1) f[c] = __builtin_amdgcn_logf(f[c]);
            if constexpr (OP == 2) u[c] = static_cast<uint32_t>((static_cast<uint64_t>(u[c]) * 0xD2511F53u + w[c]) >> 32);
            if constexpr (OP == 3) d[c] = __builtin_fma(d[c], da[c], static_cast<double>(fb[c]));
            if constexpr (OP == 4) u[c] = __builtin_amdgcn_bitop3_b32(u[c], w[c], w[(c + 4) % kIssueChains], 0x96);
            if constexpr (OP == 6) f[c] = __builtin_fmaf(f[c], fa[c], 0x1p-14f);
            if constexpr (OP == 5) {
                f[c] = __builtin_amdgcn_logf(f[c]);
                g[c] = __builtin_fmaf(g[c], fa[c], fb[c]);
                g[c] = __builtin_fmaf(g[c], fa[c], 0.5f * fb[c]);
                g[c] = __builtin_fmaf(g[c], fa[c], 0.25f * fb[c]);
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kIssueChains; ++c) s += f[c] + g[c] + static_cast<float>(d[c]) + static_cast<float>(u[c]);
    sink[static_cast<uint64_t>(blockIdx.x) * blockDim.x + t] = s;
    const uint64_t c1 = __builtin_amdgcn_s_memtime();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    if ((t & 63) == 0) {
        const uint64_t wv = static_cast<uint64_t>(blockIdx.x) * 4 + (t >> 6);
        stamps[2 * wv] = c1 - c0;
        stamps[2 * wv + 1] = r1 - r0;
    }
}

// One hardware transcendental per element.  sin and cos take revolutions.
__global__ void __launch_bounds__(256) transcendental_kernel(int op, const float *in, float *out, uint64_t n)
{
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float x = in[i];
        float y;
        switch (op) {
        case 0: y = __builtin_amdgcn_logf(x); break;
        case 1: y = __builtin_amdgcn_exp2f(x); break;
        case 2: y = __builtin_amdgcn_sinf(x); break;
        case 3: y = __builtin_amdgcn_cosf(x); break;
        case 4: y = __builtin_amdgcn_sqrtf(x); break;
        case 5: y = __builtin_amdgcn_rsqf(x); break;
        default: y = __builtin_amdgcn_rcpf(x); break;
        }
        out[i] = y;
    }
}

}  // namespace

int issue_probe_steps(int op) { return kIssueIters * kIssueChains * (op == 5 ? 4 : 1); }

uint32_t issue_probe_blocks() { return static_cast<uint32_t>(device_cu_count()) * 8u; }

hipError_t launch_issue_probe(int op, float *sink, uint64_t *stamps, hipStream_t stream)
{
    const dim3 grid(issue_probe_blocks()), block(256);
    switch (op) {
    case 0: hipLaunchKernelGGL(issue_kernel<0>, grid, block, 0, stream, sink, stamps); break;
    case 1: hipLaunchKernelGGL(issue_kernel<1>, grid, block, 0, stream, sink, stamps); break;
    case 2: hipLaunchKernelGGL(issue_kernel<2>, grid, block, 0, stream, sink, stamps); break;
    case 3: hipLaunchKernelGGL(issue_kernel<3>, grid, block, 0, stream, sink, stamps); break;
    case 4: hipLaunchKernelGGL(issue_kernel<4>, grid, block, 0, stream, sink, stamps); break;
    case 5: hipLaunchKernelGGL(issue_kernel<5>, grid, block, 0, stream, sink, stamps); break;
    case 6: hipLaunchKernelGGL(issue_kernel<6>, grid, block, 0, stream, sink, stamps); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_transcendental_probe(int op, const float *in, float *out, uint64_t n, hipStream_t stream)
{
    const uint64_t need = (n + 255) / 256;
    const uint64_t cap = static_cast<uint64_t>(device_cu_count()) * 16;
    const int grid = static_cast<int>(need < cap ? (need > 0 ? need : 1) : cap);
    hipLaunchKernelGGL(transcendental_kernel, dim3(grid), dim3(256), 0, stream, op, in, out, n);
    return hipGetLastError();
}

}  // namespace kappa
