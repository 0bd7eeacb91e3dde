// divergence.hip -- how far the approximation G (Sec. 3, eq:G) is from the
// Kappa distribution, over a grid of (kappa, c): the relative entropy
// D(f||g; kappa, c) of eq:relative_entropy (the quantity the paper's grid
// search over c in [0, 1.5] x kappa in [1.5, 10] minimises, Fig. fig:map) and
// the energy error (E_approx - E_kappa)/E_kappa of Fig. fig:DE(b).
//
// For a free c the other parameters stay as Table 1 sets them: a of eq:a,
// kappa* of eq:k2, b = (b/c) c with b/c of eq:b.  f is eq:kappax and g is
// eq:approx_x, both in x = v^2/theta^2.  kappa = +inf is the Maxwell limit:
// f = 2/sqrt(pi) x^(1/2) e^-x, exp_q* -> exp, a and b/c at their limits.
//
// Quadrature.  x = exp(ell), ell = (pi/2) sinh(t) (the exp-sinh rule for
// [0, inf)), trapezoidal in t with step 1/16 over t in [-83/16, 108/16]: 192
// nodes, x from 1e-61 to 1e291.  With delta = ln g - ln f and since f and g
// both integrate to one,
//     D  = int f (e^delta - 1 - delta) dx,
//     dE = int x f (e^delta - 1) dx / (3 kappa / (2 kappa - 3)),
// where E_kappa = 3 kappa / (2 kappa - 3) in units of m theta^2 / 2 is
// eq:kappaE.  Both integrands are sums of non-cancelling terms.  The first
// form equals the printed definition int f ln(f/g) dx up to the truncation of
// the range; it has no cancellation where f and g nearly agree, which is where
// the paper's D of 1e-9..1e-5 comes from.
//
// Every evaluation stays finite for x up to 1e291: ln g is assembled from
//   y   = (a + b x) * x / (1 + c x)
//   s   = log1p(y / kappa*)             (1 + y/kappa*)^(-kappa*) = exp(-kappa* s)
//   y'  = (a/x + 2b + b c x) * x / (1 + c x)^2,
//   ln g = ln(3/2) + ln(1 - e^(-kappa* s))/2 - (kappa* + 1) s + ln y'.
//
// Work layout: one block per (kappa, group of c values); the block first
// tabulates the c-independent part of every node (ell, x, 1/x, ln f and the
// two quadrature weights) in LDS, then each wave takes one c at a time with
// its 64 lanes over the nodes and reduces with a fixed butterfly, so results
// do not depend on the launch shape.  The bound is FP64 VALU (five FP64
// transcendentals per node); no HBM traffic beyond the outputs.
#include <math.h>

#include "kappa_internal.hpp"

namespace kappa {

namespace {

constexpr int kDivNodes = 192;
constexpr int kDivNeg = 83;  // nodes with t < 0
constexpr double kDivH = 1.0 / 16.0;
constexpr double kHalfPi = 1.5707963267948966;
constexpr int kDivCPerBlock = 16;

struct DivNode {
    double x, q, lnf, w_d, w_e;  // x, 1/x, ln f(x), h (dx/dt) f, h (dx/dt) f x
};

struct KappaConst {
    double kappa, kstar, lnB, a, b_over_c;
    bool ok, maxwell;
};

__device__ KappaConst kappa_const(double k)
{
    KappaConst s;
    s.ok = k > 1.5 && !isnan(k);
    s.maxwell = isinf(k);
    s.kappa = k;
    s.kstar = k - 0.5;                                                 // eq:k2
    if (!s.ok) return s;
    if (s.maxwell) {
        s.lnB = 0.0;
        s.a = 0.82713398786586665;  // (4 / (3 sqrt(pi)))^(2/3)
        s.b_over_c = 1.0;
        return s;
    }
    s.lnB = lgamma(1.5) + lgamma(s.kstar) - lgamma(k + 1.0);           // B(3/2, kappa - 1/2)
    s.a = exp(-log(k) + (2.0 / 3.0) * (log(2.0 / 3.0) - s.lnB));       // eq:a
    s.b_over_c = exp((log(1.5 * s.kstar) + s.lnB) / s.kstar) * s.kstar / k;  // eq:b
    return s;
}

// The c the sampler uses: eq:c, or the Maxwell-limit constant for kappa = inf.
__device__ double c_from_eq_c(double k)
{
    if (isinf(k)) return kMaxwellC;
    return (0.123 * k * k - 1.12 * k + 2.56) / (k * k - 7.89 * k + 15.6);  // eq:c
}

// e^d - 1 - d and e^d - 1 without cancellation for small d (Taylor series to
// d^8, truncation below 1e-19 relative for |d| < 1/32).
__device__ inline void expm1_parts(double d, double &em1_minus_d, double &em1)
{
    if (fabs(d) < 0.03125) {
        const double p = d * d *
                         (0.5 + d * (1.0 / 6 + d * (1.0 / 24 + d * (1.0 / 120 + d * (1.0 / 720 + d * (1.0 / 5040 +
                                                                                               d * (1.0 / 40320)))))));
        em1_minus_d = p;
        em1 = p + d;
    } else {
        em1 = expm1(d);
        em1_minus_d = em1 - d;
    }
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// The c-independent part of every node for one kappa, in LDS.
__device__ void build_nodes(DivNode *nodes, const KappaConst &s)
{
    if (!s.ok) return;
    const double lnk = log(s.kappa);
    for (int n = threadIdx.x; n < kDivNodes; n += blockDim.x) {
        const double t = (n - kDivNeg) * kDivH;
        const double ell = kHalfPi * sinh(t);
        const double x = exp(ell);
        // eq:kappax in logs; Maxwell: ln(2/sqrt(pi)) + ell/2 - x
        const double lnf = s.maxwell ? 0.12078223763524522 + 0.5 * ell - x
                                     : -lnk - s.lnB + 0.5 * (ell - lnk) - (s.kappa + 1.0) * log1p(x / s.kappa);
        const double wf = kDivH * kHalfPi * cosh(t) * x * exp(lnf);  // h dx/dt f(x)
        nodes[n] = DivNode{x, exp(-ell), lnf, wf, wf * x};
    }
}

// D and the energy integral (before the 1/E_kappa factor) at one c, by the
// calling wave: lanes over the nodes, then a butterfly sum, so every lane
// returns the same two numbers.  Requires s.ok and a finite c >= 0.
__device__ void wave_quality(const DivNode *nodes, const KappaConst &s, double c, double &dsum, double &esum)
{
    const int lane = threadIdx.x & 63;
    const double kstar = s.kstar, inv_kstar = 1.0 / s.kstar;
    const double a = s.a, b = s.b_over_c * c;
    dsum = 0.0;
    esum = 0.0;
    for (int n = lane; n < kDivNodes; n += 64) {
        const DivNode nd = nodes[n];
        // f has underflowed (Maxwell: x > 745): the node adds nothing, and delta
        // = ln g - ln f would be the difference of two numbers of order x
        if (nd.w_d == 0.0) continue;
        const double inv = 1.0 / (1.0 + c * nd.x);
        const double t1 = nd.x * inv;                      // x / (1 + c x) <= 1/c
        const double y = (a + b * nd.x) * t1;
        // ln exp_q*(-y) = -kappa* log1p(y / kappa*), and ln of the (kappa*+1) power; -y for Maxwell
        double lq, lq1;
        if (s.maxwell) {
            lq = -y;
            lq1 = -y;
        } else {
            const double sl = log1p(y * inv_kstar);
            lq = -kstar * sl;
            lq1 = -(kstar + 1.0) * sl;
        }
        const double ln1mE = log(-expm1(lq));
        const double yp = (a * nd.q + 2.0 * b + b * c * nd.x) * t1 * inv;
        const double lng = 0.40546510810816438 + 0.5 * ln1mE + lq1 + log(yp);  // ln(3/2) + ...
        double em1_minus_d, em1;
        expm1_parts(lng - nd.lnf, em1_minus_d, em1);
        dsum += nd.w_d * em1_minus_d;
        esum += nd.w_e * em1;
    }
    dsum = wave_sum(dsum);
    esum = wave_sum(esum);
}

__device__ inline double inv_energy(const KappaConst &s)
{
    return s.maxwell ? 2.0 / 3.0 : (2.0 * s.kappa - 3.0) / (3.0 * s.kappa);
}

__global__ void __launch_bounds__(256) divergence_kernel(const double *__restrict__ kappa,
                                                         const double *__restrict__ cvals, uint32_t nc,
                                                         double *__restrict__ D, double *__restrict__ dE)
{
    __shared__ DivNode nodes[kDivNodes];
    const uint32_t i = blockIdx.y;
    const KappaConst s = kappa_const(kappa[i]);
    build_nodes(nodes, s);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    const uint32_t j0 = blockIdx.x * kDivCPerBlock;
    const uint32_t j1 = j0 + kDivCPerBlock < nc ? j0 + kDivCPerBlock : nc;
    for (uint32_t j = j0 + wave; j < j1; j += nwaves) {
        const double c = cvals ? cvals[j] : (s.ok ? c_from_eq_c(s.kappa) : 0.0);
        double dsum = 0.0, esum = 0.0;
        const bool ok = s.ok && isfinite(c) && c >= 0.0;
        if (ok) wave_quality(nodes, s, c, dsum, esum);
        if (lane == 0) {
            const size_t o = static_cast<size_t>(i) * nc + j;
            const double nan = __builtin_nan("");
            D[o] = ok ? dsum : nan;
            if (dE) dE[o] = ok ? esum * inv_energy(s) : nan;
        }
    }
}

// The grid search of Sec. 3 refined: for one kappa per block, the four waves
// evaluate D at every c of the grid and keep the smallest (lowest index on
// ties, NaN skipped); then wave 0 runs a golden-section search for the
// minimum of D between the grid neighbours of that point (D is unimodal there
// on the paper's range), `iters` steps, and writes the midpoint of the final
// bracket and D there.
__global__ void __launch_bounds__(256) optimum_kernel(const double *__restrict__ kappa,
                                                      const double *__restrict__ cgrid, uint32_t nc, uint32_t iters,
                                                      double *__restrict__ c_opt, double *__restrict__ D_opt)
{
    __shared__ DivNode nodes[kDivNodes];
    __shared__ double best_d[4];
    __shared__ uint32_t best_j[4];
    const uint32_t i = blockIdx.x;
    const KappaConst s = kappa_const(kappa[i]);
    build_nodes(nodes, s);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    double bd = __builtin_inf();
    uint32_t bj = 0xFFFFFFFFu;
    if (s.ok) {
        for (uint32_t j = wave; j < nc; j += nwaves) {
            const double c = cgrid[j];
            if (!(isfinite(c) && c >= 0.0)) continue;
            double d, e;
            wave_quality(nodes, s, c, d, e);
            if (d < bd) {  // j increases within a wave: strict keeps the lowest index
                bd = d;
                bj = j;
            }
        }
    }
    if (lane == 0) {
        best_d[wave] = bd;
        best_j[wave] = bj;
    }
    __syncthreads();
    if (wave != 0) return;
    for (int w = 1; w < nwaves; ++w) {
        if (best_d[w] < bd || (best_d[w] == bd && best_j[w] < bj)) {
            bd = best_d[w];
            bj = best_j[w];
        }
    }
    const double nan = __builtin_nan("");
    if (bj == 0xFFFFFFFFu) {
        if (lane == 0) {
            c_opt[i] = nan;
            if (D_opt) D_opt[i] = nan;
        }
        return;
    }
    // bracket: the grid neighbours (clamped to the grid, and to valid c)
    double lo = cgrid[bj > 0 ? bj - 1 : 0], hi = cgrid[bj + 1 < nc ? bj + 1 : nc - 1];
    if (!(isfinite(lo) && lo >= 0.0)) lo = cgrid[bj];
    if (!(isfinite(hi) && hi >= 0.0)) hi = cgrid[bj];
    constexpr double kInvPhi = 0.6180339887498949;  // (sqrt(5) - 1) / 2
    double x1 = hi - kInvPhi * (hi - lo), x2 = lo + kInvPhi * (hi - lo), f1, f2, e;
    wave_quality(nodes, s, x1, f1, e);
    wave_quality(nodes, s, x2, f2, e);
    for (uint32_t it = 0; it < iters; ++it) {
        if (f1 < f2) {
            hi = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi - kInvPhi * (hi - lo);
            wave_quality(nodes, s, x1, f1, e);
        } else {
            lo = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo + kInvPhi * (hi - lo);
            wave_quality(nodes, s, x2, f2, e);
        }
    }
    const double cm = 0.5 * (lo + hi);
    double dm;
    wave_quality(nodes, s, cm, dm, e);
    // the grid point itself if the refinement did not beat it (a minimum at the end of the range)
    const bool keep_grid = !(dm <= bd);
    if (lane == 0) {
        c_opt[i] = keep_grid ? cgrid[bj] : cm;
        if (D_opt) D_opt[i] = keep_grid ? bd : dm;
    }
}

// One wave per kappa row: the index of the smallest D (NaN skipped, lowest
// index on ties; 0xFFFFFFFF when the row has no number).
__global__ void __launch_bounds__(64) argmin_kernel(const double *__restrict__ D, uint32_t nc,
                                                    uint32_t *__restrict__ argmin)
{
    const uint32_t i = blockIdx.x;
    const double *row = D + static_cast<size_t>(i) * nc;
    double best = __builtin_inf();
    uint32_t bj = 0xFFFFFFFFu;
    for (uint32_t j = threadIdx.x; j < nc; j += 64) {
        const double v = row[j];
        if (v < best) {  // false for NaN; strict, so the lowest j of this lane wins ties
            best = v;
            bj = j;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(best, off, 64);
        const uint32_t oj = __shfl_xor(bj, off, 64);
        if (ov < best || (ov == best && oj < bj)) {
            best = ov;
            bj = oj;
        }
    }
    if (threadIdx.x == 0) argmin[i] = bj;
}

}  // namespace

hipError_t launch_optimum(const double *kappa, uint32_t nk, const double *cgrid, uint32_t nc, uint32_t iters,
                          double *c_opt, double *D_opt, hipStream_t stream)
{
    hipLaunchKernelGGL(optimum_kernel, dim3(nk), dim3(256), 0, stream, kappa, cgrid, nc, iters, c_opt, D_opt);
    return hipGetLastError();
}

hipError_t launch_divergence(const double *kappa, uint32_t nk, const double *c, uint32_t nc, double *D, double *dE,
                             uint32_t *argmin, hipStream_t stream)
{
    const uint32_t per_block = nc < kDivCPerBlock ? nc : kDivCPerBlock;
    const int waves = per_block < 4 ? static_cast<int>(per_block) : 4;
    const dim3 grid((nc + kDivCPerBlock - 1) / kDivCPerBlock, nk);
    hipLaunchKernelGGL(divergence_kernel, grid, dim3(64 * waves), 0, stream, kappa, c, nc, D, dE);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || !argmin) return err;
    hipLaunchKernelGGL(argmin_kernel, dim3(nk), dim3(64), 0, stream, D, nc, argmin);
    return hipGetLastError();
}

}  // namespace kappa
