/*
 * kappa.h -- C ABI of libkappa, an MI355X (gfx950) implementation of the
 * approximate Kappa velocity generator of Zenitani & Umeda, "An approximate
 * Kappa generator for particle simulations" (arXiv 2602.05606).
 *
 * The generator (Table 1 of the paper) draws three uniforms per particle,
 * inverts the q-exponential approximation G of the Kappa speed CDF in closed
 * form (Sec. 3, eq:G; Sec. 4, eq:GU, eq:qlog, eq:v, eq:L), scatters the speed
 * isotropically and scales it by theta, the most probable speed of the Kappa
 * distribution (Sec. 2, eq:kappa).  It has no loops or rejection steps.
 *
 * Conventions shared by every entry point:
 *
 *   kappa    Kappa index; the distribution needs kappa > 3/2 (Sec. 2).  The
 *            fitted parameter c of eq:c covers kappa in [1.5, 10] (Sec. 3);
 *            larger values are accepted.  +INFINITY is the Maxwell limit
 *            where an entry point says so (see kappa_params).  kappa <= 3/2,
 *            NaN, or +INFINITY elsewhere: KAPPA_EINVAL.
 *   theta    most probable speed, > 0 and finite, else KAPPA_EINVAL.
 *   seed     64-bit Philox4x32-10 key: key = (low 32 bits, high 32 bits).
 *   counters particle i of segment seg draws the Philox4x32-10 block with
 *            counter (low 32 bits of i, high 32 bits of i, seg, draw), draw = 0
 *            for the generator.  i = counter_offset + position in the output.
 *            Output therefore depends only on (kappa, theta, drift, seed, i,
 *            seg, precision): never on grid, block, unroll, stream or device,
 *            and a range can be produced in chunks by advancing counter_offset.
 *   uniforms U1 from the Philox words (r0, r3), U2 from r1, U3 from r2, as
 *            open midpoint dyadics (see KAPPA_FP64 below), in every precision.
 *   outputs  structure-of-arrays vx[n], vy[n], vz[n], device pointers owned by
 *            the caller, written and never read.  double for KAPPA_FP64,
 *            float for KAPPA_FP32 and KAPPA_FP32_NOTAIL.  Each pointer must be
 *            aligned to its element size (else KAPPA_EALIGN); 16-byte aligned
 *            pointers take the vector-store path.  kappa_sample also takes it
 *            for three views at one common misalignment (slices of aligned
 *            arrays) of at least 2^16 particles, after writing the particles
 *            before the 16-byte boundary one per thread in a launch of their
 *            own.
 *   stream   a hipStream_t passed as void*; NULL is the legacy default stream.
 *            Calls are asynchronous on the stream unless stated otherwise.
 *   errors   return codes only; nothing aborts or throws across the ABI.
 *            Arguments are validated before any HIP call.  A HIP failure
 *            returns KAPPA_EDEVICE and kappa_last_error() gives the message.
 *   device   the current HIP device must be gfx950, else KAPPA_EUNSUPPORTED.
 *   threads  entry points that take no plan keep no state between calls but
 *            the calling thread's last-error message and a lock-guarded
 *            per-device cache of the CU count: any number of host threads
 *            may call them at once, on any streams.  A plan is not
 *            thread-safe: calls on one plan must not overlap in time (they
 *            share its captured graph and launch shape).  Its launches may be
 *            in flight on several streams at once, into different outputs.
 *   capture  kappa_sample, kappa_sample_backward and the plan launches
 *            (direct, not graph) allocate, synchronise and memset nothing, so
 *            a caller may capture them into a hipGraph of its own.
 */
#ifndef KAPPA_H
#define KAPPA_H

#include <stddef.h>
#include <stdint.h>

#if defined(KAPPA_BUILDING_LIBRARY)
#define KAPPA_API __attribute__((visibility("default")))
#else
#define KAPPA_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KAPPA_OK = 0,
    KAPPA_EINVAL = 1,      /* invalid argument */
    KAPPA_EALIGN = 2,      /* pointer not aligned to its element size */
    KAPPA_EDEVICE = 3,     /* HIP runtime error */
    KAPPA_ENOMEM = 4,      /* device allocation failed (plans only) */
    KAPPA_EUNSUPPORTED = 5,/* current device is not gfx950 */
    KAPPA_ERANGE = 6       /* size outside a documented limit */
} kappa_status;

typedef enum {
    /* All FP64.  U1 has 53 bits: m = top 53 bits of (r0:r3); U1 = (2m+1) 2^-54
     * if m < 2^52, else 1 - U1 = (2^54 - 2m - 1) 2^-54; U2 = (r1 + 1/2) 2^-32,
     * U3 = (r2 + 1/2) 2^-32.  double outputs. */
    KAPPA_FP64 = 0,
    /* FP32 bulk with an FP64 tail.  The same uniforms as KAPPA_FP64 (each
     * rounded to float inside the FP32 arithmetic), so the two precisions
     * differ only in arithmetic.  When 1 - U1 < 2^-20 (r0 >= 0xFFFFF000,
     * probability 2^-20) the speed is inverted in FP64 and rounded to float.
     * float outputs. */
    KAPPA_FP32 = 1,
    /* KAPPA_FP32 without the FP64 tail (diagnostics only). float outputs. */
    KAPPA_FP32_NOTAIL = 2
} kappa_precision;

/* Per-species parameter block of Table 1 (rows 1-4), with the kappa
 * derivatives the backward pass uses, as returned by kappa_params(). */
enum {
    KAPPA_P_KSTAR = 0,  /* kappa* = kappa - 1/2 (eq:k2) */
    KAPPA_P_A,          /* a (eq:a) */
    KAPPA_P_B,          /* b = (b/c) c (eq:b) */
    KAPPA_P_C,          /* c = c_approx (eq:c) */
    KAPPA_P_B_OVER_C,   /* b/c (eq:b) */
    KAPPA_P_DA,         /* da/dkappa */
    KAPPA_P_DB,         /* db/dkappa */
    KAPPA_P_DC,         /* dc/dkappa */
    KAPPA_P_LNBETA,     /* ln B(3/2, kappa*) */
    KAPPA_NPARAMS
};

/* kappa_params -- the setup rows of Table 1 (once per species), in FP64 on
 * the host: kappa*, a, c, b per eq:k2, eq:a, eq:c, eq:b, with
 * B(3/2, kappa*) = Gamma(3/2) Gamma(kappa*) / Gamma(kappa + 1) (Sec. 6), and
 * their kappa-derivatives.  out: host array of KAPPA_NPARAMS doubles, indexed
 * by KAPPA_P_*.  No HIP call.  KAPPA_EINVAL for a bad kappa or NULL out.
 * kappa = +INFINITY is the Maxwell limit (accepted wherever the sampler takes
 * kappa): exp_q* -> exp and the q-logarithm of eq:L -> ln; a and b/c take
 * the kappa -> inf limits of Sec. 3, (4/(3 sqrt(pi)))^(2/3) and 1; c is 0.079,
 * the three-figure minimiser of the relative entropy of eq:relative_entropy
 * against the Maxwell density (the paper's criterion for c; it gives no
 * Maxwell constants).  kappa* is reported as +inf and the derivatives as 0. */
KAPPA_API kappa_status kappa_params(double kappa, double *out);

/* kappa_sample -- one species: particles counter_offset .. counter_offset+n-1
 * of segment seg_id, Table 1 per particle (Sec. 4).  vx, vy, vz: device arrays
 * of n elements (see conventions).  n = 0 is a no-op returning KAPPA_OK.
 * counter_offset + n must not exceed 2^64 (KAPPA_EINVAL).  kappa > 3/2, or
 * +INFINITY for the Maxwell limit (see kappa_params). */
KAPPA_API kappa_status kappa_sample(double kappa, double theta, uint64_t n, uint64_t seed,
                          uint64_t counter_offset, uint32_t seg_id, int precision,
                          void *vx, void *vy, void *vz, void *stream);

/* kappa_sample_autotune -- time kappa_sample's launch shapes (256, 128 or 64
 * threads per workgroup x 1, 2, 4 or 8 particles per thread) on n particles
 * of the given precision into vx, vy, vz (written; 16-byte aligned, else
 * KAPPA_EALIGN), `reps` timed launches each after one warm-up (HIP events on
 * stream), and keep the fastest for this precision and every n in the same
 * power-of-two bucket: later kappa_sample calls of this process use it, and it
 * is recorded in the autotune cache file (KAPPA_AUTOTUNE_CACHE; see below).
 * block, unroll (host, may be NULL) receive the chosen shape.  The output of
 * kappa_sample never depends on the shape.  Synchronous.
 *
 * Environment of the tuned shapes (single-species and plans):
 *   KAPPA_AUTOTUNE_CACHE=<path>  JSON file of tuned shapes shared by processes;
 *   KAPPA_AUTOTUNE=off|use|refresh  off: the file is neither read nor
 *       written; use (default): launches start from the file's shape and
 *       tuning writes it; refresh: the file is not read, tuning writes it;
 *   KAPPA_FORWARD_SHAPE="block,unroll" overrides kappa_sample's shape;
 *   KAPPA_LOG=1  one line on stderr per kernel launch (kernel, precision,
 *       particles, grid, block, particles per thread, stream). */
KAPPA_API kappa_status kappa_sample_autotune(int precision, uint64_t n, void *vx, void *vy, void *vz, int reps,
                                             int *block, int *unroll, void *stream);

/* One segment of a batched launch: a species (kappa, theta) in one cell
 * (drift) with count particles.  Its particles use counters
 * (0 .. count-1, seg_id, 0), so segment s of a batched call equals
 * kappa_sample(kappa, theta, count, seed, 0, seg_id, ...) plus drift. */
typedef struct {
    double kappa;
    double theta;
    double drift[3]; /* added to (vx, vy, vz) after sampling (Galilean shift) */
    uint64_t count;
    uint32_t seg_id;
    uint32_t reserved; /* must be 0 */
} kappa_segment;

/* A cell box for fused particle loading: positions of a segment's particles
 * are drawn uniformly in [lo, lo + size) per axis.  Not in the paper, which
 * samples velocities only; a PIC code loads both at start-up. */
typedef struct {
    double lo[3];   /* lower corner, finite */
    double size[3]; /* edge lengths, finite and >= 0 */
} kappa_cell;

/* Opaque batched plan: device copies of the segment table and of the tile ->
 * segment map, the chosen launch shape, and a captured hipGraph. */
typedef struct kappa_plan_s *kappa_plan;

/* Limits of a batched plan. */
#define KAPPA_MAX_SEGMENTS (1u << 24)

/* kappa_plan_create -- validate segs (host array of nseg, 1 <= nseg <=
 * KAPPA_MAX_SEGMENTS, each with a valid kappa and theta, finite drift,
 * reserved = 0, and seg_id values distinct: segments sharing a seg_id would
 * draw the same counters, so a repeated seg_id is KAPPA_EINVAL), compute each segment's Table 1 setup in FP64 on the host,
 * lay segments out back to back in the given order (segment s starts at the
 * sum of the earlier counts), and upload the tables.  Allocates device memory
 * (KAPPA_ENOMEM on failure) on the current device; synchronous.  *out owns it
 * until kappa_plan_destroy.  Segments with count 0 are allowed. */
KAPPA_API kappa_status kappa_plan_create(const kappa_segment *segs, uint32_t nseg, uint64_t seed, int precision,
                               kappa_plan *out);

/* Total number of particles of the plan (sum of counts). */
KAPPA_API kappa_status kappa_plan_total(kappa_plan plan, uint64_t *total);

/* kappa_plan_launch -- one persistent-kernel launch writing all segments into
 * vx, vy, vz (device arrays of kappa_plan_total elements).  Asynchronous. */
KAPPA_API kappa_status kappa_plan_launch(kappa_plan plan, void *vx, void *vy, void *vz, void *stream);

/* kappa_plan_graph_launch -- same output as kappa_plan_launch, through a
 * hipGraph holding the one persistent launch.  The graph is captured on the
 * first call (and again if vx, vy, vz or the launch shape change) and then
 * replayed with hipGraphLaunch on stream.  Asynchronous. */
KAPPA_API kappa_status kappa_plan_graph_launch(kappa_plan plan, void *vx, void *vy, void *vz, void *stream);

/* kappa_plan_autotune -- time every launch shape (block size, particles per
 * thread, workgroups per CU) of the persistent kernel on this plan with HIP
 * events, keep the fastest, and record it in the autotune cache file (path in
 * the KAPPA_AUTOTUNE_CACHE environment variable, if set).  Writes vx, vy, vz.
 * Synchronous.  reps: timed launches per shape (>= 1). */
KAPPA_API kappa_status kappa_plan_autotune(kappa_plan plan, void *vx, void *vy, void *vz, int reps, void *stream);

/* The launch shape the plan uses: block size, particles per thread, grid. */
KAPPA_API kappa_status kappa_plan_shape(kappa_plan plan, int *block, int *unroll, int *grid);

/* Set the launch shape explicitly (block in {64,128,256}, unroll in {1,2,4,8},
 * 1 <= grid <= 2^23; KAPPA_EINVAL otherwise).  Output does not depend on the
 * shape. */
KAPPA_API kappa_status kappa_plan_set_shape(kappa_plan plan, int block, int unroll, int grid);

/* kappa_plan_set_cells -- give the plan one cell box per segment (host array
 * of the plan's nseg cells, in segment order; copied to a plan-owned device
 * table, so the host array may be freed).  NULL removes the table.  Replacing
 * a table synchronises the device.  KAPPA_EINVAL for a non-finite lo or a
 * size that is negative or not finite, and, for a plan of an FP32 precision,
 * for lo, size or lo + size that overflow float. */
KAPPA_API kappa_status kappa_plan_set_cells(kappa_plan plan, const kappa_cell *cells);

/* kappa_plan_launch_pic / kappa_plan_graph_launch_pic -- fused particle
 * loading: the plan's launch (direct, or through its captured hipGraph) that
 * also writes positions px, py, pz (device arrays of kappa_plan_total
 * elements, same type as the velocities).  Particle j of a segment is placed
 * at lo + u size, with u from the Philox block of draw 1 of its counter
 * (velocities use draw 0 and are bit-identical to kappa_plan_launch):
 * u = (r + 1/2) 2^-32 in KAPPA_FP64, (floor(r / 2^9) + 1/2) 2^-23 in the
 * FP32 modes, for r = r0, r1, r2 on x, y, z; one fused multiply-add in the
 * output precision, with lo and size rounded to it.  The box is half-open:
 * lo <= p < lo + size in that precision's values (a fused multiply-add that
 * rounds up to lo + size is capped at the largest value below it; a box of
 * size 0 puts every particle at lo).  KAPPA_EINVAL without
 * kappa_plan_set_cells.
 * Asynchronous. */
KAPPA_API kappa_status kappa_plan_launch_pic(kappa_plan plan, void *px, void *py, void *pz, void *vx, void *vy,
                                             void *vz, void *stream);
KAPPA_API kappa_status kappa_plan_graph_launch_pic(kappa_plan plan, void *px, void *py, void *pz, void *vx,
                                                   void *vy, void *vz, void *stream);

/* kappa_plan_destroy -- waits for the plan's device (launches may still be in
 * flight on any stream), then frees the plan's tables, cell table, captured
 * graph and capture stream.  NULL is a no-op. */
KAPPA_API kappa_status kappa_plan_destroy(kappa_plan plan);

/* kappa_sample_batched -- many species and cells in one persistent launch:
 * creates a plan, launches it on stream, waits for it and destroys the plan.
 * Synchronous.  vx, vy, vz hold the sum of the counts. */
KAPPA_API kappa_status kappa_sample_batched(const kappa_segment *segs, uint32_t nseg, uint64_t seed, int precision,
                                  void *vx, void *vy, void *vz, void *stream);

/* Workspace the backward pass needs for n particles, in bytes. */
KAPPA_API size_t kappa_backward_workspace_bytes(uint64_t n);

/* kappa_sample_backward -- reparameterisation gradient of a loss through the
 * samples of kappa_sample (same kappa, theta, n, seed, counter_offset,
 * seg_id, precision), at fixed uniforms; finite kappa only (KAPPA_EINVAL for
 * +INFINITY).  Not in the paper; it differentiates
 * Table 1: dv/dtheta = v/theta, and dv/dkappa = v (dx/dkappa) / (2x), where
 * x = (V/theta)^2 solves b x^2 + (a + cL) x + L = 0 (eq:v, eq:L), so
 * dx/dkappa = -(b' x^2 + (a' + c' L + c L') x + L') / sqrt((a+cL)^2 - 4bL).
 *   gx, gy, gz  device arrays of n upstream gradients dLoss/dv (double for
 *               KAPPA_FP64, float otherwise), read only.
 *   grad        device array of 2 doubles, written: (sum_i g_i . dv_i/dkappa,
 *               sum_i g_i . dv_i/dtheta), accumulated in FP64 in a fixed order.
 *   workspace   device scratch of at least kappa_backward_workspace_bytes(n)
 *               bytes (KAPPA_ERANGE if smaller), 256-byte aligned, owned by
 *               the caller; its contents are overwritten.
 * n = 0 writes zeros.  Asynchronous. */
KAPPA_API kappa_status kappa_sample_backward(double kappa, double theta, uint64_t n, uint64_t seed,
                                   uint64_t counter_offset, uint32_t seg_id, int precision,
                                   const void *gx, const void *gy, const void *gz, double *grad,
                                   void *workspace, size_t workspace_bytes, void *stream);

/* kappa_sample_backward_noalloc -- kappa_sample_backward without a workspace
 * argument, for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels, results (bit for bit) and errors as
 * kappa_sample_backward, except that the partial sums go to a static device
 * array of the library: KAPPA_BACKWARD_SCRATCH_BYTES (64 KiB, one FP64 pair
 * per workgroup of the backward grid) on each device, held from the first
 * call on that device until the process ends.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); its first call on a
 * device looks the array's address up once (hipGetSymbolAddress).  Every
 * call on one device shares that device's array: calls whose launches
 * overlap in time on one device (other streams, other host threads) race on
 * it and may return wrong sums; serialise them.  Each call writes every
 * partial it reads, so nothing needs clearing between calls.  KAPPA_ERANGE
 * when the backward grid for n needs more partials than the array holds
 * (only when the KAPPA_BACKWARD_GRID environment variable raises the grid
 * above its default cap of 4096 workgroups).  Asynchronous. */
#define KAPPA_BACKWARD_SCRATCH_BYTES 65536u
KAPPA_API kappa_status kappa_sample_backward_noalloc(double kappa, double theta, uint64_t n, uint64_t seed,
                                                     uint64_t counter_offset, uint32_t seg_id, int precision,
                                                     const void *gx, const void *gy, const void *gz,
                                                     double *grad, void *stream);

/* kappa_load_particles -- one-shot fused particle loading: kappa_plan_create,
 * kappa_plan_set_cells and kappa_plan_launch_pic, then waits for the stream
 * and frees the plan.  cells: host array of nseg boxes. */
KAPPA_API kappa_status kappa_load_particles(const kappa_segment *segs, const kappa_cell *cells, uint32_t nseg,
                                            uint64_t seed, int precision, void *px, void *py, void *pz, void *vx,
                                            void *vy, void *vz, void *stream);

/* kappa_optimum_c -- the grid search of Sec. 3 that eq:c was fitted to, with
 * a refinement: for each kappa_i, the c of c_grid (device array of nc values,
 * ascending) with the smallest relative entropy D(f||g; kappa_i, c)
 * (eq:relative_entropy, computed as in kappa_divergence_grid; NaN and negative
 * grid entries skipped, lowest index on ties), then `iters` golden-section
 * steps for the minimum of D between that point's grid neighbours (each step
 * shrinks the bracket by 0.618).  c_opt[i] is the midpoint of the final
 * bracket, or the grid point itself if D there is not larger; D_opt[i] (may be
 * NULL) is D at c_opt[i].  D is unimodal in c on the paper's range, so the
 * refinement finds the minimiser to about 1e-8 in c after 40 steps; where the
 * optimum lies at an end of the grid (Fig. fig:map: past c = 1.5 just below
 * kappa 4.1, at 0 just above) the result is that end.  kappa entries that are
 * NaN or not above 3/2 give NaN (+INFINITY is the Maxwell limit).
 * nk, nc <= 2^24, iters <= 200 (else KAPPA_ERANGE); 8-byte aligned arrays.
 * Asynchronous. */
KAPPA_API kappa_status kappa_optimum_c(const double *kappa, uint32_t nk, const double *c_grid, uint32_t nc,
                                       uint32_t iters, double *c_opt, double *D_opt, void *stream);

/* kappa_philox -- raw Philox4x32-10 blocks for particles counter_offset ..
 * counter_offset+n-1 of segment seg_id and draw number draw: out is a device
 * array of 4n uint32 words (r0, r1, r2, r3 per particle).  For bit-exact
 * tests of the generator's counter stream. */
KAPPA_API kappa_status kappa_philox(uint64_t n, uint64_t seed, uint64_t counter_offset, uint32_t seg_id, uint32_t draw,
                          uint32_t *out, void *stream);

/* Same-GPU exact Kappa generators used as performance comparators (Sec. 5,
 * third test; Sec. 6).  Both sample the exact distribution of eq:kappa with
 * rejection loops on the same Philox stream: iteration t of particle i uses
 * the block with counter (i, 0, t).  Finite kappa > 3/2 only.  precision KAPPA_FP64 (double outputs) or
 * KAPPA_FP32 (float outputs, FP32 arithmetic).  iters: optional device array
 * of n uint32 (NULL to skip) receiving the number of rejection-loop
 * iterations each particle took.
 *   kappa_sample_exact_t: the multivariate-t form: three normals (Box-Muller)
 *     times sqrt(kappa / (2 G)), G ~ Gamma(kappa - 1/2) by Marsaglia-Tsang.
 *   kappa_sample_exact_pareto: speed by acceptance-rejection from a Type II
 *     Pareto (Lomax) proposal with index n = kappa/2, isotropic direction. */
KAPPA_API kappa_status kappa_sample_exact_t(double kappa, double theta, uint64_t n, uint64_t seed, int precision,
                                  void *vx, void *vy, void *vz, uint32_t *iters, void *stream);
KAPPA_API kappa_status kappa_sample_exact_pareto(double kappa, double theta, uint64_t n, uint64_t seed, int precision,
                                       void *vx, void *vy, void *vz, uint32_t *iters, void *stream);

/* kappa_speed_histogram -- data of the Monte Carlo relative-entropy test
 * (Sec. 5, second test, eq:KL): adds to counts[k] the number of particles
 * whose speed |v| lies in [k w theta, (k+1) w theta), k < nbins, and to
 * counts[nbins] those at or beyond nbins w theta (w = bin_width).
 * Membership is decided exactly: bin k holds edge2[k] <= s2 < edge2[k+1],
 * with s2 = (vx*vx + vy*vy) + vz*vz evaluated in the data's precision and
 * edge2[k] = (k * (w * theta))^2 computed in FP64 and rounded once to that
 * precision, so any IEEE implementation of this definition gets the same
 * counts.
 *   vx, vy, vz  device arrays of n velocities (double for KAPPA_FP64, float
 *               for KAPPA_FP32 / KAPPA_FP32_NOTAIL), read only.
 *   counts      device array of nbins + 1 uint64, accumulated (not cleared),
 *               8-byte aligned.
 * 1 <= nbins <= 2047 and n <= 2^40 (else KAPPA_ERANGE); theta and bin_width
 * positive and finite (else KAPPA_EINVAL).  Asynchronous. */
KAPPA_API kappa_status kappa_speed_histogram(const void *vx, const void *vy, const void *vz, uint64_t n, int precision,
                                             double theta, double bin_width, uint32_t nbins, uint64_t *counts,
                                             void *stream);

/* kappa_relative_entropy -- the Monte Carlo relative entropy of the second
 * test (Sec. 5, eq:KL) from a speed histogram of kappa_speed_histogram:
 *   D = sum_i (P_i + eps) ln((P_i + eps) / (Q_i + eps)),
 * P_i the exact probability of bin i of the Kappa distribution (the
 * difference of eq:CDF, the regularized incomplete beta function
 * I_{x/(x+kappa)}(3/2, kappa - 1/2) with x = (v/theta)^2, at the bin's edges
 * k w and (k+1) w in units of theta; the last bin, i = nbins, is open-ended;
 * kappa = +INFINITY takes the Maxwell CDF P(3/2, x)), Q_i = counts[i] over the
 * sum of the counts.  The paper uses eps = 1e-10.  Host computation.
 *   counts  host array of nbins + 1 counts (not all zero, else KAPPA_EINVAL)
 *   D       host, written
 *   prob    host array of nbins + 1 doubles receiving P_i, or NULL
 * 1 <= nbins <= 2047 (else KAPPA_ERANGE); bin_width positive and finite,
 * eps finite and >= 0 (else KAPPA_EINVAL).  No HIP call. */
KAPPA_API kappa_status kappa_relative_entropy(double kappa, const uint64_t *counts, uint32_t nbins, double bin_width,
                                              double eps, double *D, double *prob);

/* kappa_divergence_grid -- quality of the approximation G (Sec. 3, eq:G)
 * against the Kappa distribution over a grid of (kappa, c), as in the grid
 * search behind eq:c (Sec. 3, eq:relative_entropy, Fig. fig:map) and the
 * energy comparison of Fig. fig:DE(b).  For each kappa_i and c_j, with a, b/c
 * and kappa* of Table 1 and b = (b/c) c_j:
 *   D[i*nc + j]  = int_0^inf f ln(f/g) dx          (eq:relative_entropy)
 *   dE[i*nc + j] = (E_approx - E_kappa) / E_kappa  (eq:kappaE, Fig. fig:DE)
 * with f of eq:kappax and g of eq:approx_x.  Integrals by an exp-sinh rule of
 * 192 nodes over x in [1e-61, 1e291]; against 30-digit quadrature of the
 * definitions the rule is within 1e-12 relative for D and 1e-14 absolute for
 * dE (for c = 0 the energy tail decays like x^(1/2 - kappa), so dE is only
 * settled for kappa >= 1.6 there).
 *   kappa   device array of nk doubles.  Entries that are NaN or not above
 *           3/2 give NaN rows.  +INFINITY is the Maxwell limit: f is then the
 *           Maxwell density 2/sqrt(pi) x^(1/2) e^-x, exp_q* -> exp, a and b/c
 *           at their limits (see kappa_params), E_kappa = 3/2.
 *   c       device array of nc doubles (c >= 0; other entries give NaN), or
 *           NULL with nc = 1 to take the c the sampler uses: eq:c for each
 *           kappa (the paper's curve of Fig. fig:DE), 0.079 for +INFINITY.
 *   D       device array of nk*nc doubles, written (row i = kappa_i).
 *   dE      device array of nk*nc doubles, written; NULL to skip.
 *   argmin  device array of nk uint32, written with the j of the smallest
 *           D in row i (NaN skipped, lowest j on ties, 0xFFFFFFFF if none);
 *           NULL to skip.
 * nk <= 65535 and nc <= 2^24 (else KAPPA_ERANGE); 8-byte aligned doubles,
 * 4-byte aligned argmin (else KAPPA_EALIGN).  nk = 0 or nc = 0 is a no-op.
 * Nodes where f has underflowed to zero are skipped.
 * Asynchronous. */
KAPPA_API kappa_status kappa_divergence_grid(const double *kappa, uint32_t nk, const double *c, uint32_t nc,
                                             double *D, double *dE, uint32_t *argmin, void *stream);

/* Measurement probes.
 * kappa_fill_probe: store-only kernel writing the constant pattern 1, 2, 3 to
 *   vx, vy, vz (n elements of the precision's type) with the generator's store
 *   path; its rate is the achievable HBM-write ceiling.
 * kappa_copy_probe: plain copy of bytes from src to dst (device pointers,
 *   16-byte aligned, bytes a multiple of 16) to calibrate traffic counters. */
KAPPA_API kappa_status kappa_fill_probe(uint64_t n, int precision, void *vx, void *vy, void *vz, void *stream);
KAPPA_API kappa_status kappa_copy_probe(const void *src, void *dst, uint64_t bytes, void *stream);

/* kappa_clock_probe: kappa_sample (same arguments, same outputs, same kernel
 * and launch shape) with timestamps, to find the core clock the chip holds
 * while it runs the generator.  Thread 0 of workgroup w writes
 *   stamps[4w + 0], stamps[4w + 2]: shader-clock counter (core clock cycles)
 *                                   at entry and exit of its wave;
 *   stamps[4w + 1], stamps[4w + 3]: constant-rate counter at the same points,
 *                                   ticking at *wall_hz (written, host).
 * (stamps[4w+2] - stamps[4w]) / (stamps[4w+3] - stamps[4w+1]) * *wall_hz is
 * that wave's mean core clock in Hz.
 *   stamps      device array of stamps_len uint64, 8-byte aligned; written
 *               for w < *blocks.
 *   blocks      host; written with the number of workgroups of the launch
 *               (also when stamps_len is too small: then KAPPA_ERANGE).
 *               4 * ceil(n / 64) entries always suffice.
 * The outputs must be 16-byte aligned (KAPPA_EALIGN otherwise), the launch
 * shape the default one (KAPPA_EINVAL when KAPPA_FORWARD_SHAPE changes the
 * particles per thread), and n within one launch (2^33 particles in FP32,
 * 2^32 in FP64; KAPPA_ERANGE otherwise).  n = 0 writes *blocks = 0 and launches
 * nothing.  Asynchronous like kappa_sample. */
KAPPA_API kappa_status kappa_clock_probe(double kappa, double theta, uint64_t n, uint64_t seed,
                                         uint64_t counter_offset, uint32_t seg_id, int precision, void *vx, void *vy,
                                         void *vz, uint64_t *stamps, uint64_t stamps_len, uint32_t *blocks,
                                         double *wall_hz, void *stream);

/* kappa_issue_probe: issue cost of one gfx950 instruction class, the basis of
 * the VALU-issue roofline.  One launch in which each wave issues *steps
 * instructions of the class on 8 independent chains per lane, one round of 8
 * waves per SIMD:
 *   op 0 v_fma_f32 (VGPR operands), 1 v_log_f32 (a transcendental),
 *   2 v_mad_u64_u32, 3 v_fma_f64, 4 v_bitop3_b32 (VGPR operands),
 *   5 a mix: per chain step one v_log_f32 and three v_fma_f32 on another
 *     register (4 instructions, all counted in *steps), whose cost against
 *     the sum of classes 0 and 1 shows whether the two kinds overlap,
 *   6 v_fma_f32 with two VGPR operands and a literal constant.
 * Wave w writes stamps[2w] = core-clock cycles (s_memtime) and stamps[2w+1] =
 * constant-rate ticks (s_memrealtime, *wall_hz per second) from its start to
 * its end.  With t the launch's duration, clock = sum(cycles) / sum(ticks) x
 * *wall_hz and SIMDs = 4 x CUs = *blocks / 2: SIMD-cycles per wave
 * instruction = SIMDs x clock x t / (4 x *blocks x *steps).
 *   sink    device floats, at least *blocks x 256, written (keeps the chains live)
 *   stamps  device uint64, at least *blocks x 8, 8-byte aligned, written
 *   blocks, steps, wall_hz  host, written (blocks = 8 x CUs) also when the
 *           buffers are too small (KAPPA_ERANGE), so a first call with zero
 *           lengths sizes them.
 * Asynchronous; needs the device (KAPPA_EDEVICE/KAPPA_EUNSUPPORTED otherwise).
 *
 * kappa_transcendental_probe: out[i] = the hardware instruction applied to
 * in[i] (n floats, device, 4-byte aligned): op 0 v_log_f32 (log2), 1
 * v_exp_f32 (2^x), 2 v_sin_f32 and 3 v_cos_f32 (argument in revolutions), 4
 * v_sqrt_f32, 5 v_rsq_f32, 6 v_rcp_f32.  Asynchronous. */
KAPPA_API kappa_status kappa_issue_probe(int op, float *sink, uint64_t sink_len, uint64_t *stamps,
                                         uint64_t stamps_len, uint32_t *blocks, uint32_t *steps, double *wall_hz,
                                         void *stream);
KAPPA_API kappa_status kappa_transcendental_probe(int op, const float *in, float *out, uint64_t n, void *stream);

/* Human-readable name of a status code (static storage). */
KAPPA_API const char *kappa_status_string(kappa_status status);

/* Message of the last failing call on this thread (static per-thread storage). */
KAPPA_API const char *kappa_last_error(void);

/* Library version string. */
KAPPA_API const char *kappa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KAPPA_H */
