// kappa_internal.hpp -- host-side declarations shared by the library's
// translation units (launchers, launch shapes, error reporting).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/kappa.h"
#include "kappa_params.hpp"

namespace kappa {

// c of the Maxwell limit kappa = +inf: the minimiser 0.078998 of the relative
// entropy (eq:relative_entropy) against the Maxwell density, to three figures.
// make_setup also takes kappa = +inf and returns that limit.
constexpr double kMaxwellC = 0.079;

enum Mode { kModeF64 = KAPPA_FP64, kModeF32 = KAPPA_FP32, kModeF32NoTail = KAPPA_FP32_NOTAIL };

// Launch shape: threads per block, particles per thread, blocks in the grid
// (the kernels loop over their work with a grid stride, so any grid >= 1 is
// valid and the output never depends on the shape).
struct Shape {
    int block;
    int unroll;
    int grid;
};

// ---- launch-shape tuning and launch logging (tune.cpp) ---------------------
enum TunePolicy { kTuneOff = 0, kTuneUse = 1, kTuneRefresh = 2 };
int autotune_policy();  // KAPPA_AUTOTUNE=off|use|refresh (default use)
// Shape stored under key in the KAPPA_AUTOTUNE_CACHE file (policy use only).
bool cache_lookup(const std::string &key, Shape &shape);
// Records shape under key in the cache file (policies use and refresh).
void cache_store(const std::string &key, const Shape &shape);
int size_bucket(uint64_t n);  // smallest b with 2^b >= n
// Tuned single-species shape for (mode, n's bucket): this process's, else the cache's.
bool forward_tuned(int mode, uint64_t n, Shape &shape);
void set_forward_tuned(int mode, uint64_t n, const Shape &shape);
bool log_enabled();  // KAPPA_LOG set and not "0"
void log_launch(const char *kernel, int mode, uint64_t n, const Shape &shape, const void *stream);

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Records a message for kappa_last_error() and returns status.
kappa_status fail(kappa_status status, const char *fmt, ...);

// Maps a HIP error to KAPPA_EDEVICE with its message (KAPPA_OK on hipSuccess).
kappa_status check_hip(hipError_t err, const char *what);

// ---- forward --------------------------------------------------------------
struct FwdArgs {
    uint64_t n;
    uint64_t counter_offset;
    uint32_t seg, k0, k1;
    void *vx, *vy, *vz;
    SpeciesF64 s64;
    SpeciesF32 s32;
};

// Shape for n particles in a mode; `vec` selects the vector-store path.
// KAPPA_FORWARD_SHAPE overrides it; otherwise, with `tuned`, a shape chosen by
// kappa_sample_autotune for this precision and size bucket replaces the
// default (256 threads, 4 particles per thread in FP32 and 2 in FP64).
Shape forward_shape(int mode, uint64_t n, bool vec, bool tuned = true);
hipError_t launch_forward(int mode, const Shape &shape, bool vec, const FwdArgs &args, hipStream_t stream);
uint64_t forward_max_grid();  // workgroups per forward launch (larger calls run in chunks)
// Unroll (particles per thread) of the default vector-store shape of a mode.
int forward_default_unroll(int mode);
// The forward kernel with per-workgroup clock stamps (4 uint64 per workgroup
// of shape.grid); shape must be the default vector-store shape of the mode.
hipError_t launch_forward_clock(int mode, const Shape &shape, const FwdArgs &args, uint64_t *stamps,
                                hipStream_t stream);
hipError_t launch_philox(uint64_t n, uint64_t counter_offset, uint32_t seg, uint32_t draw, uint32_t k0, uint32_t k1,
                         uint32_t *out, hipStream_t stream);
hipError_t launch_fill_probe(int mode, uint64_t n, void *vx, void *vy, void *vz, hipStream_t stream);
hipError_t launch_copy_probe(const void *src, void *dst, uint64_t bytes, hipStream_t stream);
// Hardware probes (hwprobe.hip): instruction issue cost and transcendental accuracy.
int issue_probe_steps(int op);
uint32_t issue_probe_blocks();
hipError_t launch_issue_probe(int op, float *sink, uint64_t *stamps, hipStream_t stream);
hipError_t launch_transcendental_probe(int op, const float *in, float *out, uint64_t n, hipStream_t stream);

// ---- backward -------------------------------------------------------------
struct BwdArgs {
    uint64_t n;
    uint64_t counter_offset;
    uint32_t seg, k0, k1;
    const void *gx, *gy, *gz;
    double *partials;  // 2 doubles per block
    SpeciesF64 s64;
    SpeciesF32 s32;
};

int backward_grid(uint64_t n);  // number of partial blocks for n particles
// The library's static partial-sum buffer for the allocation-free backward
// entry point: its size, and its device address on the current device (looked
// up once per device with hipGetSymbolAddress, then cached).
size_t backward_scratch_bytes();
hipError_t backward_scratch(double **ptr);
hipError_t launch_backward(int mode, const BwdArgs &args, double *grad, hipStream_t stream);

// ---- exact baselines ------------------------------------------------------
struct ExactArgs {
    uint64_t n;
    uint32_t k0, k1;
    uint32_t hi;     // high word of the launch's particle indices when it is the same for all (launcher)
    uint64_t first;  // particle index of the launch's first output (launcher)
    void *vx, *vy, *vz;
    uint32_t *iters;
    double kappa, theta;
};
hipError_t launch_exact_t(int mode, const ExactArgs &args, hipStream_t stream);
hipError_t launch_exact_pareto(int mode, const ExactArgs &args, hipStream_t stream);

// ---- speed histogram -------------------------------------------------------
size_t histogram_lds_bytes(int mode, uint32_t nbins);
hipError_t launch_histogram(int mode, const void *vx, const void *vy, const void *vz, uint64_t n, double width,
                            uint32_t nbins, uint64_t *counts, hipStream_t stream);

// Speed CDF of the Kappa distribution in x = (v/theta)^2 (eq:CDF; the Maxwell
// limit for kappa = inf) and its complement, each computed directly (entropy.cpp).
void speed_cdf(double kappa, double x, double &F, double &one_minus_F);

// ---- approximation quality over (kappa, c) ---------------------------------
hipError_t launch_optimum(const double *kappa, uint32_t nk, const double *cgrid, uint32_t nc, uint32_t iters,
                          double *c_opt, double *D_opt, hipStream_t stream);
hipError_t launch_divergence(const double *kappa, uint32_t nk, const double *c, uint32_t nc, double *D, double *dE,
                             uint32_t *argmin, hipStream_t stream);

}  // namespace kappa
