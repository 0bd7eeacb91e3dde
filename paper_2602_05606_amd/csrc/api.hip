// api.hip -- the C ABI of libkappa (declared in include/kappa.h): argument
// validation, device checks, error mapping and kernel dispatch.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "kappa_internal.hpp"

extern "C" {
kappa_status kappa_plan_create_impl(const kappa_segment *, uint32_t, uint64_t, int, kappa_plan *);
kappa_status kappa_plan_launch_impl(kappa_plan, void *, void *, void *, void *);
kappa_status kappa_plan_graph_launch_impl(kappa_plan, void *, void *, void *, void *);
kappa_status kappa_plan_autotune_impl(kappa_plan, void *, void *, void *, int, void *);
kappa_status kappa_plan_shape_impl(kappa_plan, int *, int *, int *);
kappa_status kappa_plan_set_shape_impl(kappa_plan, int, int, int);
kappa_status kappa_plan_total_impl(kappa_plan, uint64_t *);
kappa_status kappa_plan_destroy_impl(kappa_plan);
kappa_status kappa_plan_set_cells_impl(kappa_plan, const kappa_cell *);
kappa_status kappa_plan_launch_pic_impl(kappa_plan, void *, void *, void *, void *, void *, void *, void *);
kappa_status kappa_plan_graph_launch_pic_impl(kappa_plan, void *, void *, void *, void *, void *, void *, void *);
}

namespace kappa {

namespace {

thread_local char g_last_error[512] = "";

constexpr int kMaxDevices = 64;
std::mutex g_dev_mutex;
int g_dev_state[kMaxDevices] = {0};  // 0 unknown, 1 gfx950, -1 other
int g_dev_cus[kMaxDevices] = {0};

bool kappa_ok(double kappa) { return std::isfinite(kappa) && kappa > 1.5; }
// The sampler also takes kappa = +inf, the Maxwell limit.
bool kappa_or_maxwell_ok(double kappa) { return kappa > 1.5 && !std::isnan(kappa); }
bool theta_ok(double theta) { return std::isfinite(theta) && theta > 0.0; }
bool precision_ok(int p) { return p == KAPPA_FP64 || p == KAPPA_FP32 || p == KAPPA_FP32_NOTAIL; }
size_t elem_size(int p) { return p == KAPPA_FP64 ? 8 : 4; }

// Checks that the current device is gfx950 (cached per device).
kappa_status require_device()
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return check_hip(err, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(KAPPA_EDEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    if (g_dev_state[dev] == 0) {
        hipDeviceProp_t prop;
        err = hipGetDeviceProperties(&prop, dev);
        if (err != hipSuccess) return check_hip(err, "hipGetDeviceProperties");
        g_dev_state[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
        g_dev_cus[dev] = prop.multiProcessorCount;
        if (g_dev_state[dev] < 0)
            return fail(KAPPA_EUNSUPPORTED, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    }
    if (g_dev_state[dev] < 0) return fail(KAPPA_EUNSUPPORTED, "device %d is not gfx950", dev);
    return KAPPA_OK;
}

kappa_status check_outputs(uint64_t n, int precision, void *vx, void *vy, void *vz)
{
    if (n == 0) return KAPPA_OK;
    if (!vx || !vy || !vz) return fail(KAPPA_EINVAL, "null output pointer with n = %llu", (unsigned long long)n);
    const size_t e = elem_size(precision);
    if (reinterpret_cast<uintptr_t>(vx) % e || reinterpret_cast<uintptr_t>(vy) % e ||
        reinterpret_cast<uintptr_t>(vz) % e)
        return fail(KAPPA_EALIGN, "output pointers must be aligned to %zu bytes", e);
    return KAPPA_OK;
}

bool vec_aligned(int precision, const void *vx, const void *vy, const void *vz)
{
    (void)precision;
    return reinterpret_cast<uintptr_t>(vx) % 16 == 0 && reinterpret_cast<uintptr_t>(vy) % 16 == 0 &&
           reinterpret_cast<uintptr_t>(vz) % 16 == 0;
}

// Particles to write one per thread before three views that share one
// misalignment reach a 16-byte boundary together, when the rest is long
// enough to pay for a second launch; 0 otherwise (aligned views, views at
// different misalignments, short calls).
uint64_t peel_head(int precision, uint64_t n, const void *vx, const void *vy, const void *vz)
{
    constexpr uint64_t kPeelMin = 1u << 16;
    const uintptr_t m = reinterpret_cast<uintptr_t>(vx) % 16;
    if (m == 0 || m != reinterpret_cast<uintptr_t>(vy) % 16 || m != reinterpret_cast<uintptr_t>(vz) % 16) return 0;
    const uint64_t head = (16 - m) / (precision == KAPPA_FP64 ? 8 : 4);
    return n >= kPeelMin + head ? head : 0;
}

FwdArgs forward_args(double kappa, double theta, uint64_t n, uint64_t seed, uint64_t counter_offset, uint32_t seg_id,
                     void *vx, void *vy, void *vz)
{
    const Setup s = make_setup(kappa);
    FwdArgs a;
    a.n = n;
    a.counter_offset = counter_offset;
    a.seg = seg_id;
    a.k0 = static_cast<uint32_t>(seed);
    a.k1 = static_cast<uint32_t>(seed >> 32);
    a.vx = vx;
    a.vy = vy;
    a.vz = vz;
    a.s64 = species_f64(s, theta);
    a.s32 = species_f32(s, theta);
    return a;
}

}  // namespace

kappa_status fail(kappa_status status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return status;
}

kappa_status check_hip(hipError_t err, const char *what)
{
    if (err == hipSuccess) return KAPPA_OK;
    return fail(KAPPA_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(err), static_cast<int>(err));
}

int device_cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    if (g_dev_cus[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
        g_dev_cus[dev] = cus;
    }
    return g_dev_cus[dev];
}

}  // namespace kappa

using namespace kappa;

extern "C" {

const char *kappa_version(void) { return "libkappa 0.1.0 (gfx950)"; }

const char *kappa_last_error(void) { return g_last_error; }

const char *kappa_status_string(kappa_status status)
{
    switch (status) {
    case KAPPA_OK: return "KAPPA_OK";
    case KAPPA_EINVAL: return "KAPPA_EINVAL: invalid argument";
    case KAPPA_EALIGN: return "KAPPA_EALIGN: misaligned pointer";
    case KAPPA_EDEVICE: return "KAPPA_EDEVICE: HIP runtime error";
    case KAPPA_ENOMEM: return "KAPPA_ENOMEM: device allocation failed";
    case KAPPA_EUNSUPPORTED: return "KAPPA_EUNSUPPORTED: device is not gfx950";
    case KAPPA_ERANGE: return "KAPPA_ERANGE: size out of range";
    }
    return "unknown kappa_status";
}

kappa_status kappa_params(double kappa, double *out)
{
    if (!kappa_or_maxwell_ok(kappa)) return fail(KAPPA_EINVAL, "kappa must be > 3/2 or +inf (got %g)", kappa);
    if (!out) return fail(KAPPA_EINVAL, "null output array");
    const Setup s = make_setup(kappa);
    out[KAPPA_P_KSTAR] = s.kstar;
    out[KAPPA_P_A] = s.a;
    out[KAPPA_P_B] = s.b;
    out[KAPPA_P_C] = s.c;
    out[KAPPA_P_B_OVER_C] = s.b_over_c;
    out[KAPPA_P_DA] = s.da;
    out[KAPPA_P_DB] = s.db;
    out[KAPPA_P_DC] = s.dc;
    out[KAPPA_P_LNBETA] = s.lnbeta;
    return KAPPA_OK;
}

kappa_status kappa_sample(double kappa, double theta, uint64_t n, uint64_t seed, uint64_t counter_offset,
                          uint32_t seg_id, int precision, void *vx, void *vy, void *vz, void *stream)
{
    if (!kappa_or_maxwell_ok(kappa)) return fail(KAPPA_EINVAL, "kappa must be > 3/2 or +inf (got %g)", kappa);
    if (!theta_ok(theta)) return fail(KAPPA_EINVAL, "theta must be finite and > 0 (got %g)", theta);
    if (!precision_ok(precision)) return fail(KAPPA_EINVAL, "unknown precision %d", precision);
    if (n > 0 && counter_offset > UINT64_MAX - (n - 1))
        return fail(KAPPA_EINVAL, "counter_offset + n exceeds 2^64");
    kappa_status st = check_outputs(n, precision, vx, vy, vz);
    if (st != KAPPA_OK || n == 0) return st;
    st = require_device();
    if (st != KAPPA_OK) return st;
    const FwdArgs a = forward_args(kappa, theta, n, seed, counter_offset, seg_id, vx, vy, vz);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t head = peel_head(precision, n, vx, vy, vz);
    if (head > 0) {
        // a view at a common misalignment (a slice of three aligned arrays):
        // the first particles up to the 16-byte boundary one per thread, the
        // rest with vector stores; the output depends only on the counters
        FwdArgs h = a, b = a;
        h.n = head;
        const size_t esz = precision == KAPPA_FP64 ? 8 : 4;
        b.n = n - head;
        b.counter_offset = counter_offset + head;
        b.vx = static_cast<char *>(vx) + head * esz;
        b.vy = static_cast<char *>(vy) + head * esz;
        b.vz = static_cast<char *>(vz) + head * esz;
        st = check_hip(launch_forward(precision, forward_shape(precision, head, false), false, h, s), "forward kernel launch");
        if (st != KAPPA_OK) return st;
        return check_hip(launch_forward(precision, forward_shape(precision, b.n, true), true, b, s), "forward kernel launch");
    }
    const bool vec = vec_aligned(precision, vx, vy, vz);
    const Shape shape = forward_shape(precision, n, vec);
    return check_hip(launch_forward(precision, shape, vec, a, s), "forward kernel launch");
}

kappa_status kappa_sample_autotune(int precision, uint64_t n, void *vx, void *vy, void *vz, int reps, int *block,
                                   int *unroll, void *stream)
{
    if (!precision_ok(precision)) return fail(KAPPA_EINVAL, "unknown precision %d", precision);
    if (n == 0) return fail(KAPPA_EINVAL, "n must be at least 1");
    if (reps < 1) return fail(KAPPA_EINVAL, "reps must be at least 1 (got %d)", reps);
    kappa_status st = check_outputs(n, precision, vx, vy, vz);
    if (st != KAPPA_OK) return st;
    if (!vec_aligned(precision, vx, vy, vz))
        return fail(KAPPA_EALIGN, "the autotuner times the vector-store kernels: outputs must be 16-byte aligned");
    st = require_device();
    if (st != KAPPA_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the cost per particle barely depends on kappa, theta or the counters
    const FwdArgs a = forward_args(3.0, 1.0, n, 0, 0, 0, vx, vy, vz);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    st = check_hip(hipEventCreate(&e0), "hipEventCreate");
    if (st == KAPPA_OK) st = check_hip(hipEventCreate(&e1), "hipEventCreate");
    Shape best = forward_shape(precision, n, true, false);
    float best_ms = 3.4e38f;
    const int blocks[] = {64, 128, 256};
    const int unrolls[] = {1, 2, 4, 8};
    for (int b : blocks) {
        for (int u : unrolls) {
            if (st != KAPPA_OK) break;
            Shape c{b, u, 1};
            const uint64_t need = ((n + u - 1) / u + b - 1) / b;
            const uint64_t cap = forward_max_grid();
            c.grid = static_cast<int>(need < cap ? need : cap);
            st = check_hip(launch_forward(precision, c, true, a, s), "autotune warm-up launch");
            if (st != KAPPA_OK) break;
            st = check_hip(hipEventRecord(e0, s), "hipEventRecord");
            for (int r = 0; r < reps && st == KAPPA_OK; ++r)
                st = check_hip(launch_forward(precision, c, true, a, s), "autotune launch");
            if (st == KAPPA_OK) st = check_hip(hipEventRecord(e1, s), "hipEventRecord");
            if (st == KAPPA_OK) st = check_hip(hipEventSynchronize(e1), "autotune synchronize");
            float ms = 0.f;
            if (st == KAPPA_OK) st = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            if (st == KAPPA_OK && ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != KAPPA_OK) return st;
    set_forward_tuned(precision, n, best);
    if (block) *block = best.block;
    if (unroll) *unroll = best.unroll;
    return KAPPA_OK;
}

kappa_status kappa_clock_probe(double kappa, double theta, uint64_t n, uint64_t seed, uint64_t counter_offset,
                               uint32_t seg_id, int precision, void *vx, void *vy, void *vz, uint64_t *stamps,
                               uint64_t stamps_len, uint32_t *blocks, double *wall_hz, void *stream)
{
    if (!blocks || !wall_hz) return fail(KAPPA_EINVAL, "null blocks or wall_hz pointer");
    *blocks = 0;
    *wall_hz = 0.0;
    if (!kappa_or_maxwell_ok(kappa)) return fail(KAPPA_EINVAL, "kappa must be > 3/2 or +inf (got %g)", kappa);
    if (!theta_ok(theta)) return fail(KAPPA_EINVAL, "theta must be finite and > 0 (got %g)", theta);
    if (!precision_ok(precision)) return fail(KAPPA_EINVAL, "unknown precision %d", precision);
    if (n > 0 && counter_offset > UINT64_MAX - (n - 1))
        return fail(KAPPA_EINVAL, "counter_offset + n exceeds 2^64");
    kappa_status st = check_outputs(n, precision, vx, vy, vz);
    if (st != KAPPA_OK || n == 0) return st;
    if (!vec_aligned(precision, vx, vy, vz))
        return fail(KAPPA_EALIGN, "the clock probe times the vector-store kernel: outputs must be 16-byte aligned");
    if (!stamps) return fail(KAPPA_EINVAL, "null stamps pointer");
    if (reinterpret_cast<uintptr_t>(stamps) % 8) return fail(KAPPA_EALIGN, "stamps must be 8-byte aligned");
    const Shape shape = forward_shape(precision, n, true, false);
    if (shape.unroll != forward_default_unroll(precision))
        return fail(KAPPA_EINVAL, "the clock probe times the default shape (KAPPA_FORWARD_SHAPE overrides the unroll)");
    if (static_cast<uint64_t>(shape.grid) * shape.block * shape.unroll < n)
        return fail(KAPPA_ERANGE, "the clock probe times one launch: n exceeds what one launch covers");
    *blocks = static_cast<uint32_t>(shape.grid);
    if (stamps_len / 4 < static_cast<uint64_t>(shape.grid))
        return fail(KAPPA_ERANGE, "stamps holds %llu entries, the launch needs 4 x %d",
                    (unsigned long long)stamps_len, shape.grid);
    st = require_device();
    if (st != KAPPA_OK) return st;
    int dev = 0, khz = 0;
    st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st != KAPPA_OK) return st;
    st = check_hip(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
    if (st != KAPPA_OK) return st;
    if (khz <= 0) return fail(KAPPA_EDEVICE, "device reports no constant-rate counter");
    *wall_hz = 1e3 * khz;
    const FwdArgs a = forward_args(kappa, theta, n, seed, counter_offset, seg_id, vx, vy, vz);
    return check_hip(launch_forward_clock(precision, shape, a, stamps, static_cast<hipStream_t>(stream)),
                     "clock probe launch");
}

size_t kappa_backward_workspace_bytes(uint64_t n)
{
    const size_t bytes = static_cast<size_t>(backward_grid(n)) * 2 * sizeof(double);
    return (bytes + 255) & ~static_cast<size_t>(255);
}

namespace {
// Checks shared by the two backward entry points (everything but the
// partial-sum buffer).
kappa_status backward_checks(double kappa, double theta, uint64_t n, uint64_t counter_offset, int precision,
                             const void *gx, const void *gy, const void *gz, const double *grad)
{
    if (!kappa_ok(kappa)) return fail(KAPPA_EINVAL, "kappa must be finite and > 3/2 (got %g)", kappa);
    if (!theta_ok(theta)) return fail(KAPPA_EINVAL, "theta must be finite and > 0 (got %g)", theta);
    if (!precision_ok(precision)) return fail(KAPPA_EINVAL, "unknown precision %d", precision);
    if (!grad) return fail(KAPPA_EINVAL, "null grad pointer");
    if (reinterpret_cast<uintptr_t>(grad) % 8) return fail(KAPPA_EALIGN, "grad must be 8-byte aligned");
    if (n > 0 && counter_offset > UINT64_MAX - (n - 1))
        return fail(KAPPA_EINVAL, "counter_offset + n exceeds 2^64");
    if (n > 0 && (!gx || !gy || !gz)) return fail(KAPPA_EINVAL, "null gradient pointer with n > 0");
    const size_t e = elem_size(precision);
    if (n > 0 && (reinterpret_cast<uintptr_t>(gx) % e || reinterpret_cast<uintptr_t>(gy) % e ||
                  reinterpret_cast<uintptr_t>(gz) % e))
        return fail(KAPPA_EALIGN, "gradient pointers must be aligned to %zu bytes", e);
    return KAPPA_OK;
}

kappa_status backward_launch(double kappa, double theta, uint64_t n, uint64_t seed, uint64_t counter_offset,
                             uint32_t seg_id, int precision, const void *gx, const void *gy, const void *gz,
                             double *grad, double *partials, void *stream)
{
    const Setup s = make_setup(kappa);
    BwdArgs a;
    a.n = n;
    a.counter_offset = counter_offset;
    a.seg = seg_id;
    a.k0 = static_cast<uint32_t>(seed);
    a.k1 = static_cast<uint32_t>(seed >> 32);
    a.gx = gx;
    a.gy = gy;
    a.gz = gz;
    a.partials = partials;
    a.s64 = species_f64(s, theta);
    a.s32 = species_f32(s, theta);
    return check_hip(launch_backward(precision, a, grad, static_cast<hipStream_t>(stream)), "backward kernel launch");
}
}  // namespace

kappa_status kappa_sample_backward(double kappa, double theta, uint64_t n, uint64_t seed, uint64_t counter_offset,
                                   uint32_t seg_id, int precision, const void *gx, const void *gy, const void *gz,
                                   double *grad, void *workspace, size_t workspace_bytes, void *stream)
{
    kappa_status st = backward_checks(kappa, theta, n, counter_offset, precision, gx, gy, gz, grad);
    if (st != KAPPA_OK) return st;
    if (!workspace) return fail(KAPPA_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(KAPPA_EALIGN, "workspace must be 256-byte aligned");
    if (workspace_bytes < kappa_backward_workspace_bytes(n))
        return fail(KAPPA_ERANGE, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes,
                    kappa_backward_workspace_bytes(n));
    st = require_device();
    if (st != KAPPA_OK) return st;
    return backward_launch(kappa, theta, n, seed, counter_offset, seg_id, precision, gx, gy, gz, grad,
                           static_cast<double *>(workspace), stream);
}

kappa_status kappa_sample_backward_noalloc(double kappa, double theta, uint64_t n, uint64_t seed,
                                           uint64_t counter_offset, uint32_t seg_id, int precision, const void *gx,
                                           const void *gy, const void *gz, double *grad, void *stream)
{
    kappa_status st = backward_checks(kappa, theta, n, counter_offset, precision, gx, gy, gz, grad);
    if (st != KAPPA_OK) return st;
    const size_t need = static_cast<size_t>(backward_grid(n)) * 2 * sizeof(double);
    if (need > backward_scratch_bytes())
        return fail(KAPPA_ERANGE, "the backward launch for n = %llu needs %zu bytes of partial sums, more than the "
                                  "%zu of the library's static scratch (KAPPA_BACKWARD_GRID raised the grid)",
                    (unsigned long long)n, need, backward_scratch_bytes());
    st = require_device();
    if (st != KAPPA_OK) return st;
    double *partials = nullptr;
    st = check_hip(backward_scratch(&partials), "hipGetSymbolAddress of the backward scratch");
    if (st != KAPPA_OK) return st;
    return backward_launch(kappa, theta, n, seed, counter_offset, seg_id, precision, gx, gy, gz, grad, partials,
                           stream);
}

kappa_status kappa_philox(uint64_t n, uint64_t seed, uint64_t counter_offset, uint32_t seg_id, uint32_t draw,
                          uint32_t *out, void *stream)
{
    if (n == 0) return KAPPA_OK;
    if (!out) return fail(KAPPA_EINVAL, "null output pointer");
    if (reinterpret_cast<uintptr_t>(out) % 16) return fail(KAPPA_EALIGN, "Philox output must be 16-byte aligned");
    if (counter_offset > UINT64_MAX - (n - 1)) return fail(KAPPA_EINVAL, "counter_offset + n exceeds 2^64");
    kappa_status st = require_device();
    if (st != KAPPA_OK) return st;
    return check_hip(launch_philox(n, counter_offset, seg_id, draw, static_cast<uint32_t>(seed),
                                   static_cast<uint32_t>(seed >> 32), out, static_cast<hipStream_t>(stream)),
                     "Philox kernel launch");
}

static kappa_status exact_common(double kappa, double theta, uint64_t n, int precision, void *vx, void *vy, void *vz,
                                 uint32_t *iters)
{
    if (!kappa_ok(kappa)) return fail(KAPPA_EINVAL, "kappa must be finite and > 3/2 (got %g)", kappa);
    if (!theta_ok(theta)) return fail(KAPPA_EINVAL, "theta must be finite and > 0 (got %g)", theta);
    if (precision != KAPPA_FP64 && precision != KAPPA_FP32)
        return fail(KAPPA_EINVAL, "exact generators take KAPPA_FP64 or KAPPA_FP32 (got %d)", precision);
    kappa_status st = check_outputs(n, precision, vx, vy, vz);
    if (st != KAPPA_OK) return st;
    if (iters && reinterpret_cast<uintptr_t>(iters) % 4) return fail(KAPPA_EALIGN, "iters must be 4-byte aligned");
    return KAPPA_OK;
}

kappa_status kappa_sample_exact_t(double kappa, double theta, uint64_t n, uint64_t seed, int precision, void *vx,
                                  void *vy, void *vz, uint32_t *iters, void *stream)
{
    kappa_status st = exact_common(kappa, theta, n, precision, vx, vy, vz, iters);
    if (st != KAPPA_OK || n == 0) return st;
    st = require_device();
    if (st != KAPPA_OK) return st;
    ExactArgs a{n, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), 0, 0, vx, vy, vz, iters, kappa, theta};
    return check_hip(launch_exact_t(precision, a, static_cast<hipStream_t>(stream)), "exact t kernel launch");
}

kappa_status kappa_sample_exact_pareto(double kappa, double theta, uint64_t n, uint64_t seed, int precision, void *vx,
                                       void *vy, void *vz, uint32_t *iters, void *stream)
{
    kappa_status st = exact_common(kappa, theta, n, precision, vx, vy, vz, iters);
    if (st != KAPPA_OK || n == 0) return st;
    st = require_device();
    if (st != KAPPA_OK) return st;
    ExactArgs a{n, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), 0, 0, vx, vy, vz, iters, kappa, theta};
    return check_hip(launch_exact_pareto(precision, a, static_cast<hipStream_t>(stream)), "exact Pareto kernel launch");
}

kappa_status kappa_speed_histogram(const void *vx, const void *vy, const void *vz, uint64_t n, int precision,
                                   double theta, double bin_width, uint32_t nbins, uint64_t *counts, void *stream)
{
    if (!precision_ok(precision)) return fail(KAPPA_EINVAL, "unknown precision %d", precision);
    if (!theta_ok(theta)) return fail(KAPPA_EINVAL, "theta must be finite and > 0 (got %g)", theta);
    if (!std::isfinite(bin_width) || !(bin_width > 0.0))
        return fail(KAPPA_EINVAL, "bin_width must be finite and > 0 (got %g)", bin_width);
    if (nbins < 1 || nbins > 2047) return fail(KAPPA_ERANGE, "nbins %u outside [1, 2047]", nbins);
    if (n > (1ull << 40)) return fail(KAPPA_ERANGE, "n above 2^40 per call");
    if (!counts) return fail(KAPPA_EINVAL, "null counts");
    if (reinterpret_cast<uintptr_t>(counts) % 8) return fail(KAPPA_EALIGN, "counts must be 8-byte aligned");
    if (n > 0 && (!vx || !vy || !vz)) return fail(KAPPA_EINVAL, "null velocity pointer with n > 0");
    const size_t e = elem_size(precision);
    if (n > 0 && (reinterpret_cast<uintptr_t>(vx) % e || reinterpret_cast<uintptr_t>(vy) % e ||
                  reinterpret_cast<uintptr_t>(vz) % e))
        return fail(KAPPA_EALIGN, "velocity pointers must be aligned to %zu bytes", e);
    if (n == 0) return KAPPA_OK;
    kappa_status st = require_device();
    if (st != KAPPA_OK) return st;
    return check_hip(launch_histogram(precision, vx, vy, vz, n, bin_width * theta, nbins, counts,
                                      static_cast<hipStream_t>(stream)),
                     "histogram kernel launch");
}

kappa_status kappa_divergence_grid(const double *kappa, uint32_t nk, const double *c, uint32_t nc, double *D,
                                   double *dE, uint32_t *argmin, void *stream)
{
    if (nk > 65535u) return fail(KAPPA_ERANGE, "nk %u above 65535", nk);
    if (nc > (1u << 24)) return fail(KAPPA_ERANGE, "nc %u above 2^24", nc);
    if (!c && nc > 1) return fail(KAPPA_EINVAL, "c = NULL (c from eq:c) needs nc = 1 (got %u)", nc);
    if (nk == 0 || nc == 0) return KAPPA_OK;
    if (!kappa || !D) return fail(KAPPA_EINVAL, "null kappa or D");
    auto mis = [](const void *p, uintptr_t a) { return p && reinterpret_cast<uintptr_t>(p) % a != 0; };
    if (mis(kappa, 8) || mis(c, 8) || mis(D, 8) || mis(dE, 8))
        return fail(KAPPA_EALIGN, "kappa, c, D and dE must be 8-byte aligned");
    if (mis(argmin, 4)) return fail(KAPPA_EALIGN, "argmin must be 4-byte aligned");
    kappa_status st = require_device();
    if (st != KAPPA_OK) return st;
    return check_hip(launch_divergence(kappa, nk, c, nc, D, dE, argmin, static_cast<hipStream_t>(stream)),
                     "divergence kernel launch");
}

kappa_status kappa_optimum_c(const double *kappa, uint32_t nk, const double *c_grid, uint32_t nc, uint32_t iters,
                             double *c_opt, double *D_opt, void *stream)
{
    if (nk > (1u << 24)) return fail(KAPPA_ERANGE, "nk %u above 2^24", nk);
    if (nc > (1u << 24)) return fail(KAPPA_ERANGE, "nc %u above 2^24", nc);
    if (iters > 200) return fail(KAPPA_ERANGE, "iters %u above 200", iters);
    if (nk == 0) return KAPPA_OK;
    if (nc == 0) return fail(KAPPA_EINVAL, "empty c grid");
    if (!kappa || !c_grid || !c_opt) return fail(KAPPA_EINVAL, "null kappa, c_grid or c_opt");
    auto mis = [](const void *p) { return p && reinterpret_cast<uintptr_t>(p) % 8 != 0; };
    if (mis(kappa) || mis(c_grid) || mis(c_opt) || mis(D_opt))
        return fail(KAPPA_EALIGN, "kappa, c_grid, c_opt and D_opt must be 8-byte aligned");
    kappa_status st = require_device();
    if (st != KAPPA_OK) return st;
    return check_hip(launch_optimum(kappa, nk, c_grid, nc, iters, c_opt, D_opt, static_cast<hipStream_t>(stream)),
                     "optimum kernel launch");
}

kappa_status kappa_fill_probe(uint64_t n, int precision, void *vx, void *vy, void *vz, void *stream)
{
    if (precision != KAPPA_FP64 && precision != KAPPA_FP32)
        return fail(KAPPA_EINVAL, "fill probe takes KAPPA_FP64 or KAPPA_FP32 (got %d)", precision);
    kappa_status st = check_outputs(n, precision, vx, vy, vz);
    if (st != KAPPA_OK || n == 0) return st;
    if (!vec_aligned(precision, vx, vy, vz)) return fail(KAPPA_EALIGN, "fill probe outputs must be 16-byte aligned");
    st = require_device();
    if (st != KAPPA_OK) return st;
    return check_hip(launch_fill_probe(precision, n, vx, vy, vz, static_cast<hipStream_t>(stream)), "fill probe launch");
}

kappa_status kappa_copy_probe(const void *src, void *dst, uint64_t bytes, void *stream)
{
    if (bytes == 0) return KAPPA_OK;
    if (!src || !dst) return fail(KAPPA_EINVAL, "null pointer");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(KAPPA_EALIGN, "copy probe needs 16-byte aligned pointers and a size multiple of 16");
    kappa_status st = require_device();
    if (st != KAPPA_OK) return st;
    return check_hip(launch_copy_probe(src, dst, bytes, static_cast<hipStream_t>(stream)), "copy probe launch");
}

kappa_status kappa_issue_probe(int op, float *sink, uint64_t sink_len, uint64_t *stamps, uint64_t stamps_len,
                               uint32_t *blocks, uint32_t *steps, double *wall_hz, void *stream)
{
    if (!blocks || !steps || !wall_hz) return fail(KAPPA_EINVAL, "null blocks, steps or wall_hz pointer");
    *blocks = 0;
    *steps = 0;
    *wall_hz = 0.0;
    if (op < 0 || op > 6) return fail(KAPPA_EINVAL, "unknown instruction class %d", op);
    kappa_status st = require_device();
    if (st != KAPPA_OK) return st;
    const uint32_t nb = issue_probe_blocks();
    *blocks = nb;
    *steps = static_cast<uint32_t>(issue_probe_steps(op));
    if (sink_len < static_cast<uint64_t>(nb) * 256 || stamps_len < static_cast<uint64_t>(nb) * 8)
        return fail(KAPPA_ERANGE, "the probe needs %u x 256 sink floats and %u x 8 stamps", nb, nb);
    if (!sink || !stamps) return fail(KAPPA_EINVAL, "null sink or stamps pointer");
    if (reinterpret_cast<uintptr_t>(sink) % 4 || reinterpret_cast<uintptr_t>(stamps) % 8)
        return fail(KAPPA_EALIGN, "sink must be 4-byte and stamps 8-byte aligned");
    int dev = 0, khz = 0;
    st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st != KAPPA_OK) return st;
    st = check_hip(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
    if (st != KAPPA_OK) return st;
    if (khz <= 0) return fail(KAPPA_EDEVICE, "device reports no constant-rate counter");
    *wall_hz = 1e3 * khz;
    return check_hip(launch_issue_probe(op, sink, stamps, static_cast<hipStream_t>(stream)), "issue probe launch");
}

kappa_status kappa_transcendental_probe(int op, const float *in, float *out, uint64_t n, void *stream)
{
    if (op < 0 || op > 6) return fail(KAPPA_EINVAL, "unknown transcendental %d", op);
    if (n == 0) return KAPPA_OK;
    if (!in || !out) return fail(KAPPA_EINVAL, "null pointer with n = %llu", (unsigned long long)n);
    if (reinterpret_cast<uintptr_t>(in) % 4 || reinterpret_cast<uintptr_t>(out) % 4)
        return fail(KAPPA_EALIGN, "in and out must be 4-byte aligned");
    kappa_status st = require_device();
    if (st != KAPPA_OK) return st;
    return check_hip(launch_transcendental_probe(op, in, out, n, static_cast<hipStream_t>(stream)),
                     "transcendental probe launch");
}

// ---- batched --------------------------------------------------------------

static kappa_status validate_segments(const kappa_segment *segs, uint32_t nseg, int precision)
{
    if (!precision_ok(precision)) return fail(KAPPA_EINVAL, "unknown precision %d", precision);
    if (!segs) return fail(KAPPA_EINVAL, "null segment table");
    if (nseg == 0 || nseg > KAPPA_MAX_SEGMENTS)
        return fail(KAPPA_ERANGE, "segment count %u outside [1, %u]", nseg, KAPPA_MAX_SEGMENTS);
    uint64_t total = 0;
    for (uint32_t s = 0; s < nseg; ++s) {
        const kappa_segment &g = segs[s];
        if (!kappa_or_maxwell_ok(g.kappa)) return fail(KAPPA_EINVAL, "segment %u: kappa must be > 3/2 or +inf", s);
        if (!theta_ok(g.theta)) return fail(KAPPA_EINVAL, "segment %u: theta must be finite and > 0", s);
        if (!std::isfinite(g.drift[0]) || !std::isfinite(g.drift[1]) || !std::isfinite(g.drift[2]))
            return fail(KAPPA_EINVAL, "segment %u: drift must be finite", s);
        if (g.reserved != 0) return fail(KAPPA_EINVAL, "segment %u: reserved field must be 0", s);
        if (g.count > UINT64_MAX - total) return fail(KAPPA_ERANGE, "total particle count overflows");
        total += g.count;
    }
    if (total / 1024 >= UINT32_MAX) return fail(KAPPA_ERANGE, "total particle count too large for the tile map");
    // Particle j of a segment draws counter (j, seg_id): two segments with one
    // seg_id would draw the same uniforms.
    std::vector<uint32_t> ids(nseg);
    for (uint32_t s = 0; s < nseg; ++s) ids[s] = segs[s].seg_id;
    std::sort(ids.begin(), ids.end());
    const auto dup = std::adjacent_find(ids.begin(), ids.end());
    if (dup != ids.end()) return fail(KAPPA_EINVAL, "seg_id %u appears in more than one segment", *dup);
    return KAPPA_OK;
}

kappa_status kappa_plan_create(const kappa_segment *segs, uint32_t nseg, uint64_t seed, int precision, kappa_plan *out)
{
    if (!out) return fail(KAPPA_EINVAL, "null plan pointer");
    *out = nullptr;
    kappa_status st = validate_segments(segs, nseg, precision);
    if (st != KAPPA_OK) return st;
    st = require_device();
    if (st != KAPPA_OK) return st;
    return kappa_plan_create_impl(segs, nseg, seed, precision, out);
}

kappa_status kappa_plan_total(kappa_plan plan, uint64_t *total)
{
    if (!plan || !total) return fail(KAPPA_EINVAL, "null argument");
    return kappa_plan_total_impl(plan, total);
}

kappa_status kappa_plan_launch(kappa_plan plan, void *vx, void *vy, void *vz, void *stream)
{
    if (!plan) return fail(KAPPA_EINVAL, "null plan");
    return kappa_plan_launch_impl(plan, vx, vy, vz, stream);
}

kappa_status kappa_plan_graph_launch(kappa_plan plan, void *vx, void *vy, void *vz, void *stream)
{
    if (!plan) return fail(KAPPA_EINVAL, "null plan");
    return kappa_plan_graph_launch_impl(plan, vx, vy, vz, stream);
}

kappa_status kappa_plan_autotune(kappa_plan plan, void *vx, void *vy, void *vz, int reps, void *stream)
{
    if (!plan) return fail(KAPPA_EINVAL, "null plan");
    if (reps < 1) return fail(KAPPA_EINVAL, "reps must be >= 1");
    return kappa_plan_autotune_impl(plan, vx, vy, vz, reps, stream);
}

kappa_status kappa_plan_shape(kappa_plan plan, int *block, int *unroll, int *grid)
{
    if (!plan) return fail(KAPPA_EINVAL, "null plan");
    return kappa_plan_shape_impl(plan, block, unroll, grid);
}

kappa_status kappa_plan_set_shape(kappa_plan plan, int block, int unroll, int grid)
{
    if (!plan) return fail(KAPPA_EINVAL, "null plan");
    return kappa_plan_set_shape_impl(plan, block, unroll, grid);
}

kappa_status kappa_plan_set_cells(kappa_plan plan, const kappa_cell *cells)
{
    if (!plan) return fail(KAPPA_EINVAL, "null plan");
    return kappa_plan_set_cells_impl(plan, cells);
}

kappa_status kappa_plan_launch_pic(kappa_plan plan, void *px, void *py, void *pz, void *vx, void *vy, void *vz,
                                   void *stream)
{
    if (!plan) return fail(KAPPA_EINVAL, "null plan");
    return kappa_plan_launch_pic_impl(plan, px, py, pz, vx, vy, vz, stream);
}

kappa_status kappa_plan_graph_launch_pic(kappa_plan plan, void *px, void *py, void *pz, void *vx, void *vy, void *vz,
                                         void *stream)
{
    if (!plan) return fail(KAPPA_EINVAL, "null plan");
    return kappa_plan_graph_launch_pic_impl(plan, px, py, pz, vx, vy, vz, stream);
}

kappa_status kappa_plan_destroy(kappa_plan plan)
{
    if (!plan) return KAPPA_OK;
    return kappa_plan_destroy_impl(plan);
}

kappa_status kappa_sample_batched(const kappa_segment *segs, uint32_t nseg, uint64_t seed, int precision, void *vx,
                                  void *vy, void *vz, void *stream)
{
    kappa_plan plan = nullptr;
    kappa_status st = kappa_plan_create(segs, nseg, seed, precision, &plan);
    if (st != KAPPA_OK) return st;
    st = kappa_plan_launch_impl(plan, vx, vy, vz, stream);
    if (st == KAPPA_OK) st = check_hip(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "hipStreamSynchronize");
    kappa_plan_destroy_impl(plan);
    return st;
}

kappa_status kappa_load_particles(const kappa_segment *segs, const kappa_cell *cells, uint32_t nseg, uint64_t seed,
                                  int precision, void *px, void *py, void *pz, void *vx, void *vy, void *vz,
                                  void *stream)
{
    if (!cells) return fail(KAPPA_EINVAL, "null cells");
    kappa_plan plan = nullptr;
    kappa_status st = kappa_plan_create(segs, nseg, seed, precision, &plan);
    if (st != KAPPA_OK) return st;
    st = kappa_plan_set_cells_impl(plan, cells);
    if (st == KAPPA_OK) st = kappa_plan_launch_pic_impl(plan, px, py, pz, vx, vy, vz, stream);
    if (st == KAPPA_OK) st = check_hip(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "hipStreamSynchronize");
    kappa_plan_destroy_impl(plan);
    return st;
}

}  // extern "C"
