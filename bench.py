"""Benchmark of the approximate Kappa velocity generator on one MI355X.

One step = one pass of the generator over the C2 workload: 1e8 particles for
each kappa in {1.6, 2, 3, 4, 6, 10}, theta 1, FP32 with the FP64 tail
inversion, seed 1 (the paper's third test generates 1e8 particles over a
range of kappa, Sec. 5).  Outputs stay resident in HBM; nothing is copied to
the host inside the timed region.

Prints one JSON line: the headline throughput (particles/s), the roofline of
the dominant kernel (HBM write bytes per launch over its event-timed duration,
against the 8 TB/s peak), the same GPU's exact generators and FP64 path, the
backward and batched forms, and the CPU oracle as a baseline.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-extras]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
METRIC = "particles/sec (3D velocities) and % HBM-write roofline vs same-GPU exact generator"
# Per hot-path kernel: the sources it is built from (a committed counter
# profile is used only while they are unchanged), the rocprofv3 name of its
# product instantiation, the algorithmic HBM bytes per unit (particle), the
# direction of that traffic, and the file stem of its profiles under profiles/.
_FWD = ["paper_2602_05606_amd/csrc/kappa_device.hpp", "paper_2602_05606_amd/csrc/forward.hip",
        "paper_2602_05606_amd/csrc/kappa_params.hpp", "paper_2602_05606_amd/csrc/kappa_store.hpp"]
_BWD = ["paper_2602_05606_amd/csrc/kappa_device.hpp", "paper_2602_05606_amd/csrc/backward.hip",
        "paper_2602_05606_amd/csrc/kappa_params.hpp"]
_BAT = ["paper_2602_05606_amd/csrc/kappa_device.hpp", "paper_2602_05606_amd/csrc/batched.hip",
        "paper_2602_05606_amd/csrc/kappa_params.hpp", "paper_2602_05606_amd/csrc/kappa_store.hpp"]
KERNELS = {
    "c2-fp32": dict(stem="forward_fp32_c2", match="forward_kernel<1, 4, true, false>", sources=_FWD, unit_bytes=12,
                    traffic="write", label="forward_kernel<FP32 tail, 4 particles/thread>"),
    "c2-fp64": dict(stem="forward_fp64_c2", match="forward_kernel<0, 2, true, false>", sources=_FWD, unit_bytes=24,
                    traffic="write", label="forward_kernel<FP64, 2 particles/thread>"),
    "c3-fp32": dict(stem="backward_fp32_c3", match="backward_kernel<1, 4, true, true>", sources=_BWD, unit_bytes=12,
                    traffic="read", label="backward_kernel<FP32 tail, 4 particles/thread>"),
    "c3-fp64": dict(stem="backward_fp64_c3", match="backward_kernel<0, 2, true, true>", sources=_BWD, unit_bytes=24,
                    traffic="read", label="backward_kernel<FP64, 2 particles/thread>"),
    "c4-direct": dict(stem="batched_fp32_c4", match="batched_kernel<1, 4, false, unsigned int>", sources=_BAT, unit_bytes=12,
                      traffic="write", label="batched_kernel<FP32 tail, 4 particles/thread>"),
    "c4-pic": dict(stem="batched_pic_fp32_c4", match="batched_kernel<1, 4, true, unsigned int>", sources=_BAT, unit_bytes=24,
                   traffic="write", label="batched_kernel<FP32 tail, positions, 4 particles/thread>"),
}
_EXACT = ["paper_2602_05606_amd/csrc/baselines.hip", "paper_2602_05606_amd/csrc/kappa_device.hpp",
          "paper_2602_05606_amd/csrc/kappa_store.hpp"]
KERNELS["exact-t"] = dict(stem="exact_t_fp32_c2", match="exact_t_kernel<float, 4, true>", sources=_EXACT, unit_bytes=12,
                          traffic="write", label="exact_t_kernel<float, 4 particles/thread> (t/gamma rejection)")
KERNELS["exact-pareto"] = dict(stem="exact_pareto_fp32_c2", match="exact_pareto_kernel<float, 4, true>", sources=_EXACT,
                               unit_bytes=12, traffic="write",
                               label="exact_pareto_kernel<float, 4 particles/thread> (Pareto rejection)")
KERNELS["hist-fp32"] = dict(stem="histogram_fp32_test2", match="histogram_kernel<float, true>",
                           sources=["paper_2602_05606_amd/csrc/histogram.hip"], unit_bytes=12, traffic="read",
                           label="histogram_kernel<float, 16-byte loads>")
KERNELS["c4-graph"] = dict(KERNELS["c4-direct"])
KERNELS["c4-caller-graph"] = dict(KERNELS["c4-direct"])
# VALU issue capacity: 256 CUs x 4 SIMDs, 2.4 GHz at most.  Issue floor of one
# wave64 instruction in SIMD-cycles, from the chip's published vector rates:
# full-rate 32-bit operations 2 (64 lanes at 32 per cycle: the 157.3 TFLOP/s
# FP32 vector peak), FP64 arithmetic 4 (78.6 TFLOP/s), 64-bit integer
# operations such as v_mad_u64_u32 4 (two passes), transcendentals 8 (quarter
# rate).  Priced at these floors an instruction mix cannot exceed the chip's
# capacity: the fraction is a lower bound on the share of issue time the
# kernel needs.  The issue probe's measured costs (all a little above the
# floors) are reported beside it.
SIMD_COUNT = 256 * 4
SIMD_CYCLES_PER_S = SIMD_COUNT * 2.4e9
ISSUE_FLOOR = {"full_rate": 2.0, "f64": 4.0, "int64": 4.0, "transcendental_f32": 8.0, "transcendental_f64": 8.0}
# rocprofv3 instruction classes (SQ_INSTS_VALU_*) of each priced class
VALU_CLASSES = {"transcendental_f32": ["SQ_INSTS_VALU_TRANS_F32"], "transcendental_f64": ["SQ_INSTS_VALU_TRANS_F64"],
                "f64": ["SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64"],
                "int64": ["SQ_INSTS_VALU_INT64"]}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(path="c2-fp32"):
    h = hashlib.sha256()
    for p in KERNELS[path]["sources"]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_profile(kind, path):
    """A committed profile summary (kind 'valu' or 'traffic') of a path's
    kernel, or None when it is missing or was taken on other kernel sources."""
    try:
        with open(os.path.join(ROOT, "profiles", f"{kind}_{KERNELS[path]['stem']}.json")) as f:
            t = json.load(f)
    except (OSError, ValueError, KeyError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash(path):
        return None
    return t


def measured_traffic(launch_bytes, path="c2-fp32"):
    """HBM bytes per launch from the committed rocprofv3 counter runs (each
    counter scaled by what it reads for a plain copy of known size in the same
    run), or None when they are missing or stale."""
    t = load_profile("traffic", path)
    if t is None:
        return None
    return {"write_bytes": t["write_bytes_per_launch"], "fetch_bytes": t["fetch_bytes_per_launch"],
            "algorithmic_bytes": launch_bytes, "calibration": t.get("calibration")}


def measure_issue_costs(kp):
    """SIMD-cycles per wave64 instruction of the classes the kernels issue,
    measured on this chip (kappa_issue_probe: saturated issue, in-kernel
    clock, so independent of the clock the chip holds)."""
    return {name: kp.issue_cost(name)["cycles"]
            for name in ("fma_f32", "transcendental_f32", "mad_u64_u32", "fma_f64", "fma_f32_literal")}


def alu_roofline(units_per_s, clock=None, costs=None, path="c2-fp32", profile=None):
    """VALU-issue roofline of a path's kernel: its committed rocprofv3
    instruction counts per unit (SQ_INSTS_VALU and the transcendental and FP64
    classes; v_mad_u64_u32 from the kernel's ISA) priced at the issue floors,
    against 1024 SIMDs at 2.4 GHz and, with `clock` (the core clock measured
    during the same workload), at that clock.  None when the counts are
    missing or were taken on other kernel sources."""
    v = profile if profile is not None else load_profile("valu", path)
    if v is None:
        return None
    pu = v["per_unit"]
    mix = {k: pu.get(k, 0.0) for k in VALU_CLASSES}
    mix["full_rate"] = pu["valu"] - sum(mix.values())
    cycles = sum(ISSUE_FLOOR[k] * n for k, n in mix.items()) / 64.0
    achieved = units_per_s * cycles
    out = {"bound": "alu", "achieved": achieved, "peak": SIMD_CYCLES_PER_S, "unit": "SIMD-cycles/s",
           "frac": achieved / SIMD_CYCLES_PER_S, "kernel": KERNELS[path]["label"],
           "valu_per_unit": pu["valu"], "per_unit": mix, "issue_floor_simd_cycles": ISSUE_FLOOR,
           "simd_cycles_per_unit_at_floor": cycles, "counts_from": f"profiles/valu_{KERNELS[path]['stem']}.json"}
    if costs:
        out["measured_issue_costs"] = costs
    if clock:
        at_clock = SIMD_COUNT * clock["core_clock_ghz"] * 1e9
        out.update({"measured_clock": clock, "peak_at_measured_clock": at_clock,
                    "frac_at_measured_clock": achieved / at_clock})
    return out


def hbm_roofline(path, units, ms, clock=None, costs=None):
    """HBM roofline object of one launch of a path's kernel (algorithmic bytes
    over the event-timed launch duration against 8 TB/s), with its measured
    traffic and its VALU-issue fraction where committed counters cover it."""
    k = KERNELS[path]
    launch_bytes = k["unit_bytes"] * units
    achieved = launch_bytes / (ms * 1e-3) / 1e9
    alu = alu_roofline(units / (ms * 1e-3), clock, costs, path)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(launch_bytes, path), "direction": k["traffic"], "kernel": k["label"],
            "algorithmic_bytes_per_launch": launch_bytes, "avg_launch_ms": ms,
            "valu_issue_frac": alu["frac_at_measured_clock" if clock else "frac"] if alu else None}


def launch_clock_probe(kp, torch, kappas, theta, n, seed, out):
    """Core clock during the timed workload, part 1: one clock-probe launch per
    kappa right after the timed steps (the same kernel with per-workgroup
    stamps of the core-clock and constant-rate counters), back to back like
    the timed launches, into stamp buffers allocated beforehand.  Nothing is
    read back here, so the GPU does not idle (and clock down) before the
    extras that follow."""
    bufs = [torch.empty(kp.clock_probe_stamps(n), dtype=torch.int64, device=out[0].device) for _ in kappas]
    kp.clock_probe(kappas[0], theta, n, seed, precision=kp.FP32, out=out, stamps=bufs[0])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    runs = [kp.clock_probe(k, theta, n, seed, precision=kp.FP32, out=out, stamps=b) for k, b in zip(kappas, bufs)]
    e1.record()
    return runs, (e0, e1)


def finish_clock_probe(probe, torch, avg_kernel_ms):
    """Part 2: reads the stamps back; the clock is weighted by wave lifetime."""
    runs, (e0, e1) = probe
    torch.cuda.synchronize()
    cycles = ticks = 0
    hz = None
    for _, stamps, hz in runs:
        s = stamps.cpu()
        cycles += int((s[:, 2] - s[:, 0]).sum())
        ticks += int((s[:, 3] - s[:, 1]).sum())
    ghz = cycles / ticks * hz / 1e9
    return {"core_clock_ghz": ghz, "max_clock_ghz": 2.4, "constant_rate_counter_hz": hz,
            "probe_launch_ms": e0.elapsed_time(e1) / len(runs), "timed_launch_ms": avg_kernel_ms,
            "how": "kappa_clock_probe: the forward kernel with core-clock (s_memtime) and constant-rate "
                   "(s_memrealtime) stamps per workgroup, one launch per kappa after the timed steps"}


def step_protocol(step_ms, particles_per_step):
    """Per-step times of the timed region (HIP events between steps): their
    median, and the paper's protocol of four runs with the mean of the last
    three (Sec. 5) taken on the first four timed steps."""
    srt = sorted(step_ms)
    med = 0.5 * (srt[(len(srt) - 1) // 2] + srt[len(srt) // 2])
    out = {"steps": len(step_ms), "step_ms_median": med, "step_ms_min": srt[0], "step_ms_max": srt[-1],
           "particles_per_s_at_median": particles_per_step / (med * 1e-3)}
    if len(step_ms) >= 4:
        paper = sum(step_ms[1:4]) / 3.0
        out.update({"paper_protocol_step_ms": paper, "paper_protocol_particles_per_s": particles_per_step / (paper * 1e-3),
                    "paper_protocol": "four runs (the first four timed steps), mean of the last three"})
    return out


def time_launches(fn, reps, torch, warm=2, warm_ms=50.0):
    """Average duration (ms) of fn() over reps back-to-back calls after `warm`
    untimed ones, and more untimed ones until at least warm_ms of GPU time has
    passed (the core clock ramps up over tens of ms of load after the GPU
    idles, which it does between the extras): HIP events on the current stream
    (the one the library launches on) before the first timed call and after
    the last, so host-side call overhead overlaps the GPU work instead of being
    counted as idle time."""
    w0 = torch.cuda.Event(enable_timing=True)
    w0.record()
    for _ in range(warm):
        fn()
    while warm_ms > 0:
        w1 = torch.cuda.Event(enable_timing=True)
        w1.record()
        w1.synchronize()
        if w0.elapsed_time(w1) >= warm_ms:
            break
        for _ in range(max(warm, 1)):
            fn()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps


def exact_cdf_table(kappa, points=1 << 20):
    """The exact Kappa speed CDF (eq:CDF) tabulated in y = x / (x + kappa) on
    [0, 1], for interpolation on the GPU (scipy's regularized incomplete beta)."""
    import numpy as np
    from scipy import special
    y = np.linspace(0.0, 1.0, points + 1)
    return special.betainc(1.5, kappa - 0.5, y)


def ks_distance(torch, vx, vy, vz, theta, kappa, table):
    """Kolmogorov-Smirnov distance of the speeds against the exact CDF, on the GPU."""
    x = ((vx.double() ** 2 + vy.double() ** 2 + vz.double() ** 2) / theta ** 2)
    x, _ = torch.sort(x)
    y = x / (x + kappa)
    tab = torch.as_tensor(table, device=x.device)
    pos = y * (tab.numel() - 1)
    i0 = torch.clamp(pos.floor().long(), 0, tab.numel() - 2)
    w = pos - i0.double()
    f = tab[i0] * (1 - w) + tab[i0 + 1] * w
    n = x.numel()
    hi = torch.arange(1, n + 1, device=x.device, dtype=torch.float64) / n
    return float(torch.maximum((hi - f).max(), (f - (hi - 1.0 / n)).max()))


def sup_G_minus_F(kp, kappa):
    """sup_x |G(x) - F(x)| on a dense log grid: G of eq:G with the library's
    Table 1 setup, F the exact CDF of eq:CDF (scipy's regularized incomplete
    beta).  The approximate generator's KS accuracy equals an exact
    generator's until 1.36 / sqrt(N) falls to about this value."""
    import numpy as np
    from scipy import special
    p = kp.params(kappa)
    x = np.logspace(-6, 4, 200_001)
    u = (p["a"] * x + p["b"] * x * x) / (1 + p["c"] * x)
    G = (-np.expm1(-p["kstar"] * np.log1p(u / p["kstar"]))) ** 1.5
    F = special.betainc(1.5, kappa - 0.5, x / (x + kappa))
    return float(np.max(np.abs(G - F)))


def ks_table(kp, torch, kappas, theta, seed, out32, n_ks=10 ** 7):
    """KS distance against the exact CDF at n_ks particles for the approximate
    generator and the two exact ones, with the 1.36/sqrt(n) 5% critical value;
    and per kappa sup|G - F| with the sample size N* = (1.36 / sup|G - F|)^2
    below which the approximate generator's KS accuracy equals the exact ones'
    (the speedups of the rates extra hold at equal KS accuracy up to N*)."""
    res = {"n": n_ks, "critical_5pct": 1.36 / n_ks ** 0.5}
    sub = tuple(t[:n_ks] for t in out32)
    for k in kappas:
        table = exact_cdf_table(k)
        row = {}
        kp.sample(k, theta, n_ks, seed, precision=kp.FP32, out=sub)
        row["approx"] = ks_distance(torch, *sub, theta, k, table)
        kp.sample_exact_t(k, theta, n_ks, seed, precision=kp.FP32, out=sub)
        row["t_gamma"] = ks_distance(torch, *sub, theta, k, table)
        kp.sample_exact_pareto(k, theta, n_ks, seed, precision=kp.FP32, out=sub)
        row["pareto"] = ks_distance(torch, *sub, theta, k, table)
        sup = sup_G_minus_F(kp, k)
        row["sup_G_minus_F"] = sup
        row["equal_ks_accuracy_up_to_N"] = (1.36 / sup) ** 2
        res[str(k)] = row
    return res


def relative_entropy_test2(kp, torch, dev, kappas=(3.0, 4.1, 7.5), n_max=10 ** 10, chunk=10 ** 8, seed=3):
    """The paper's second test (Sec. 5, eq:KL, Fig. fig:KL) at N = 1e6 .. n_max:
    D(P||Q) between the exact Kappa speed bins (width theta/5) and the Monte
    Carlo histogram, for the approximate generator (one counter stream,
    accumulated) and the exact t generator (one seed per chunk), with the
    time the GPU spent generating and binning."""
    import numpy as np
    checkpoints = [10 ** e for e in range(6, int(round(np.log10(n_max))) + 1)]
    buf = tuple(torch.empty(chunk, dtype=torch.float32, device=dev) for _ in range(3))
    res = {"bin_width": 0.2, "nbins": 100, "eps": 1e-10, "N": checkpoints}
    for k in kappas:
        row = {}
        for name in ("approx", "t_gamma"):
            counts = torch.zeros(101, dtype=torch.int64, device=dev)
            done, ds = 0, []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for target in checkpoints:
                while done < target:
                    m = min(chunk, target - done)
                    sub = tuple(b[:m] for b in buf)
                    if name == "approx":
                        kp.sample(k, 1.0, m, seed, counter_offset=done, precision=kp.FP32, out=sub)
                    else:
                        kp.sample_exact_t(k, 1.0, m, seed + 1000 + done // chunk, precision=kp.FP32, out=sub)
                    kp.speed_histogram(*sub, theta=1.0, bin_width=0.2, nbins=100, counts=counts)
                    done += m
                ds.append(kp.relative_entropy(k, counts, 0.2))
            torch.cuda.synchronize()
            row[name] = ds
            row[name + "_s"] = time.perf_counter() - t0
        res[str(k)] = row
    h_ms = time_launches(lambda: kp.speed_histogram(*buf, theta=1.0, bin_width=0.2, nbins=100), 5, torch)
    res["histogram_GB_per_s_read"] = 12 * chunk / (h_ms * 1e-3) / 1e9
    res["histogram_ms"] = h_ms
    return res


def mt_acceptance(kappa):
    """eq:mt_eff: acceptance of the Marsaglia-Tsang gamma rejection at shape
    k = kappa - 1/2 (the loop inside the t-form exact generator)."""
    k = kappa - 0.5
    return math.exp(k - 1.0 / 3 + math.lgamma(k) - 0.5 * math.log(2 * math.pi) - (k - 0.5) * math.log(k - 1.0 / 3))


def pareto_acceptance(kappa):
    """eq:pareto_eff: acceptance of the Type II Pareto rejection with index kappa/2."""
    ln_b = math.lgamma(1.5) + math.lgamma(kappa - 0.5) - math.lgamma(kappa + 1)
    return math.exp((1 + kappa / 2) * math.log(kappa) - math.log(2) - 0.5 * (kappa - 1) * math.log(kappa - 1) + ln_b)


def ridley_mu1(rho, t):
    """eq:ridley1: typical loop count of t lanes in lock step, rejection rate rho
    below about 2^(1/t) - 1."""
    return 3 - (1 - rho) ** t - (1 - rho * rho) ** t


def ridley_mu2(rho, t):
    """eq:ridley2: the same for rho well above 2^(1/t) - 1."""
    return math.log(2 * (rho - 1) * t / math.log(rho)) / math.log(1 / rho) + 1


def simt_loop_counts(kp, torch, kappas, theta, seed, n=1 << 24):
    """Sec. 6's SIMT cost model against the GPU: for each kappa, the per-particle
    loop counts of the two exact generators (mean ~ 1/p), the mean over groups
    of t consecutive particles of their largest count (the count a t-wide SIMT
    group waits for: t = 64 is the MI355X wave, t = 32 the paper's warp), and
    the model's mu1 (t-gamma) and mu2 (Pareto) with the variates per particle
    it predicts, 3 + 2 mu1 and 2 + 2 mu2."""
    res = {"n": n, "threshold_2^(1/t)-1": {"32": 2 ** (1 / 32) - 1, "64": 2 ** (1 / 64) - 1}}
    for k in kappas:
        row = {}
        for name, fn, p in (("t_gamma", kp.sample_exact_t, mt_acceptance(k)),
                            ("pareto", kp.sample_exact_pareto, pareto_acceptance(k))):
            *_, it = fn(k, theta, n, seed, precision=kp.FP32, with_iters=True)
            it = it.to(torch.float64)
            entry = {"acceptance": p, "mean_loops": it.mean().item(), "cpu_variates_model": (3 + 2 / p)
                     if name == "t_gamma" else (2 + 2 / p)}
            for t in (32, 64):
                rho = 1 - p
                mu = ridley_mu1(rho, t) if name == "t_gamma" else ridley_mu2(rho, t)
                entry[f"group_max_mean_t{t}"] = it.view(-1, t).max(dim=1).values.mean().item()
                entry[f"model_mu_t{t}"] = mu
                entry[f"model_variates_t{t}"] = (3 + 2 * mu) if name == "t_gamma" else (2 + 2 * mu)
            row[name] = entry
        res[str(k)] = row
    return res


def dc_inside(ks):
    """kappa values where eq:c lies inside the survey's c range [0, 1.5]."""
    cap = (0.123 * ks ** 2 - 1.12 * ks + 2.56) / (ks ** 2 - 7.89 * ks + 15.6)
    return cap <= 1.5


def dc_all(kp, kt):
    d, _, _ = kp.divergence_grid(kt, None, energy=False)
    return d.cpu().numpy()[:, 0]


def divergence_survey(kp, torch, dev):
    """The grid search behind eq:c (Sec. 3, Fig. fig:map): D(f||g; kappa, c) on
    c in [0, 1.5] x kappa in (1.5, 10] at steps 0.005 and 0.01, with the
    optimum c per kappa, and D and the energy error along eq:c (Fig. fig:DE)."""
    import numpy as np
    ks = np.round(np.arange(1.51, 10.0001, 0.01), 10)
    cs = np.round(np.arange(0.0, 1.5001, 0.005), 10)
    kt = torch.tensor(ks, dtype=torch.float64, device=dev)
    ct = torch.tensor(cs, dtype=torch.float64, device=dev)
    D = torch.empty((len(ks), len(cs)), dtype=torch.float64, device=dev)
    am = torch.empty(len(ks), dtype=torch.int32, device=dev)
    kp.divergence_grid(kt, ct, energy=False, argmin=True)  # warm-up
    ms = time_launches(lambda: kp._lib.check(kp._lib.load().kappa_divergence_grid(
        kp._ptr(kt), len(ks), kp._ptr(ct), len(cs), kp._ptr(D), None, kp._ptr(am),
        kp._stream(None, dev)), "kappa_divergence_grid"), 3, torch)
    copt = cs[am.cpu().numpy()]
    # golden-section refinement of the grid optimum (kappa_optimum_c), 40 steps per kappa
    c_ref, d_ref = kp.optimum_c(kt, ct, iters=40)
    opt_ms = time_launches(lambda: kp.optimum_c(kt, ct, iters=40), 3, torch)
    c_ref, d_ref = c_ref.cpu().numpy(), d_ref.cpu().numpy()
    dc, ec, _ = kp.divergence_grid(kt, None)
    dc, ec = dc.cpu().numpy()[:, 0], ec.cpu().numpy()[:, 0]
    pick = [1.6, 2.0, 2.6, 3.0, 3.5, 3.9, 4.1, 4.2, 5.0, 7.5, 10.0]
    idx = [int(np.argmin(np.abs(ks - k))) for k in pick]
    points = len(ks) * len(cs)
    return {"kappa_points": len(ks), "c_points": len(cs), "ms": ms, "grid_points_per_s": points / (ms * 1e-3),
            "quadrature_nodes": 192,
            "optimum_c": {str(pick[n]): float(copt[i]) for n, i in enumerate(idx)},
            "optimum_c_refined": {str(pick[n]): float(c_ref[i]) for n, i in enumerate(idx)},
            "refine_ms": opt_ms,
            "refined_optimum_never_above_eq_c": bool(np.all(d_ref[dc_inside(ks)] <= dc_all(kp, kt)[dc_inside(ks)]
                                                           * (1 + 1e-12))),
            "D_along_eq_c": {str(pick[n]): float(dc[i]) for n, i in enumerate(idx)},
            "dE_over_E_along_eq_c": {str(pick[n]): float(ec[i]) for n, i in enumerate(idx)},
            "kappa_where_optimum_c_leaves_the_range": [float(ks[i]) for i in np.nonzero(copt == cs[-1])[0][[0, -1]]]
            if np.any(copt == cs[-1]) else None}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def timing_protocol(fn, reps=10):
    """Runs fn() reps times (reps >= 10) and returns (median s, the paper's
    protocol of four runs with the mean of the last three (Sec. 5), all
    times).  The first four runs serve the paper's protocol."""
    times = []
    for _ in range(max(reps, 10)):
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
    srt = sorted(times)
    median = 0.5 * (srt[(len(srt) - 1) // 2] + srt[len(srt) // 2])
    return median, sum(times[1:4]) / 3.0, times


def cpu_baseline():
    """The oracle (plain C, FP64, OpenMP over particles, not tuned) timed on
    the host, single-threaded and on every core: C1 (1e6 particles, kappa 3,
    FP64, seed 0) in full, and C2 at kappa 3 in FP64 (seed 1) on a bounded
    sample of its 1e8 particles (the first 2e7 on all cores, the first 2e6 on
    one).  Each figure is the median of 10 runs, with the paper's four runs,
    mean of the last three, beside it.  `value` is the all-core C2 rate."""
    sys.path.insert(0, ROOT)
    import oracle
    import workloads
    c1, c2 = workloads.C1, workloads.C2
    all_cores = oracle.num_threads()
    res = {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "omp_threads_all": all_cores}
    runs = {}
    for threads in (all_cores, 1):
        oracle.set_num_threads(threads)
        tag = "all_cores" if threads == all_cores else "single_thread"
        n1 = c1["n"]
        med, paper, _ = timing_protocol(lambda: oracle.sample(c1["kappa"], c1["theta"], n1, c1["seed"],
                                                               mode=oracle.MODE_FP64))
        runs[f"c1_{tag}"] = {"particles": n1, "median_s": med, "paper_mean_of_last_3_of_4_s": paper,
                             "particles_per_s": n1 / med, "threads": threads}
        n2 = 20_000_000 if threads == all_cores else 2_000_000
        med, paper, _ = timing_protocol(lambda: oracle.sample(3.0, c2["theta"], n2, c2["seed"], mode=oracle.MODE_FP64))
        runs[f"c2_kappa3_{tag}"] = {"particles": n2, "median_s": med, "paper_mean_of_last_3_of_4_s": paper,
                                    "particles_per_s": n2 / med, "threads": threads}
        log(f"cpu baseline {tag}: C1 {runs[f'c1_{tag}']['particles_per_s']:.3e}/s, "
            f"C2 kappa 3 {runs[f'c2_kappa3_{tag}']['particles_per_s']:.3e}/s")
    oracle.set_num_threads(all_cores)
    res["runs"] = runs
    main = runs["c2_kappa3_all_cores"]
    res.update({"value": main["particles_per_s"], "unit": "particles/s", "cores": all_cores, "kind": "oracle",
                "sample": f"C2 at kappa 3 in FP64: the first {main['particles']} of its 1e8 particles on "
                          f"{all_cores} threads, median of 10 runs (single-thread and C1 figures in runs)"})
    return res


EXTRAS = ("rates", "simt", "ks", "test2", "survey", "c5", "fp64", "backward", "batched")

# Single paths for profiling runs (--profile-path): each runs only its own
# launches, W untimed then K timed, so a rocprofv3 trace or counter pass of the
# command sees that kernel alone (plus torch's own buffer set-up).
PROFILE_PATHS = ("c1-fp64", "c2-fp32", "c2-fp64", "c3-fp32", "c3-fp64", "c4-direct", "c4-graph", "c4-caller-graph",
                 "c4-pic", "hist-fp32", "copy", "store-fp32", "store-fp64", "exact-t", "exact-pareto")


def _rocprof_rows(directories, suffix):
    """Rows of every rocprofv3 CSV whose name ends in suffix under the
    directories (one path, or several joined by commas: the passes of one
    measurement, e.g. FETCH_SIZE and WRITE_SIZE)."""
    import csv
    rows = []
    for directory in directories.split(","):
        for root, _, files in os.walk(directory):
            for f in sorted(files):
                if f.endswith(suffix):
                    with open(os.path.join(root, f), newline="") as fh:
                        for r in csv.DictReader(fh):
                            r["_pass"] = directory
                            rows.append(r)
    return rows


def _path_units(path):
    sys.path.insert(0, ROOT)
    import workloads
    if path.startswith("c2") or path.startswith("exact"):
        return workloads.C2["n"]
    if path.startswith("c3"):
        return workloads.C3["n"]
    if path.startswith("c4"):
        return int(sum(s["count"] for s in workloads.batched_segments()))
    if path.startswith("hist"):
        return 10 ** 8
    raise SystemExit(f"no unit count for {path}")


def summarise_counters(directory, path, command, mad_per_unit=None, note=None):
    """Reduces a rocprofv3 --pmc run of `bench.py --profile-path <path>` to the
    per-dispatch means of every counter for the path's kernel and, per unit
    (particle): wave instructions x 64 / units of the VALU classes, or HBM bytes
    per launch from FETCH_SIZE / WRITE_SIZE (KiB) scaled by what the same
    counter reads for the plain copy kernel of 1.2e9 bytes each way in the same
    run (--calibrate)."""
    k = KERNELS[path]
    rows = _rocprof_rows(directory, "counter_collection.csv")
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {directory}")
    sums = {}
    for r in rows:
        name = r["Kernel_Name"]
        who = "kernel" if k["match"] in name else "copy" if "copy_kernel" in name else None
        if who is None:
            continue
        key = (who, r["Counter_Name"], r["_pass"], r.get("Dispatch_Id") or r.get("Correlation_Id"))
        sums[key] = sums.get(key, 0.0) + float(r["Counter_Value"])
    per = {}
    for (who, cname, _, _), v in sums.items():
        per.setdefault((who, cname), []).append(v)
    mean = {key: sum(v) / len(v) for key, v in per.items()}
    units = _path_units(path)
    counters = {c: m for (who, c), m in mean.items() if who == "kernel"}
    if not counters:
        raise SystemExit(f"no dispatch of {k['match']} in {directory}")
    out = {"kernel": k["label"], "profile_path": path, "units_per_launch": units,
           "kernel_source_sha": kernel_source_hash(path),
           "dispatches": max(len(v) for (who, _), v in per.items() if who == "kernel"),
           "counters_per_dispatch": counters, "command": command}
    if "FETCH_SIZE" in counters or "WRITE_SIZE" in counters:
        copy_bytes = 1.2e9
        cal = {}
        for c, field in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
            if c in counters:
                ratio = mean[("copy", c)] * 1024.0 / copy_bytes if ("copy", c) in mean else None
                cal[f"{field}_counter_over_true"] = ratio
                out[f"{field}_kib_raw"] = counters[c]
                out[f"{field}_bytes_per_launch"] = counters[c] * 1024.0 / ratio if ratio else None
        cal["copy_bytes_per_launch"] = copy_bytes
        out["calibration"] = cal
        out["algorithmic_bytes_per_launch"] = k["unit_bytes"] * units
        out["algorithmic_direction"] = k["traffic"]
    else:
        # wave instructions x 64 lanes / particles: instructions per particle
        pu = {"valu": counters["SQ_INSTS_VALU"] * 64.0 / units}
        for cls, names in VALU_CLASSES.items():
            if any(c in counters for c in names):
                pu[cls] = sum(counters.get(c, 0.0) for c in names) * 64.0 / units
        if mad_per_unit is not None:
            pu["mad_u64_u32_isa"] = float(mad_per_unit)
        out["per_unit"] = pu
        if "GRBM_GUI_ACTIVE" in counters:
            out["grbm_gui_active_per_dispatch"] = counters["GRBM_GUI_ACTIVE"]
    if note:
        out["notes"] = note
    return out


def summarise_trace(directory, path, command, timed=None, skip=None):
    """Markdown summary of a rocprofv3 --kernel-trace --runtime-trace run of
    `bench.py --profile-path <path>`: the kernel's durations, the idle gaps
    between consecutive dispatches, and the host time of the HIP launch calls."""
    k = KERNELS.get(path, {"match": ""})
    rows = [r for r in _rocprof_rows(directory, "kernel_trace.csv") if k["match"] in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    st = [int(r["Start_Timestamp"]) for r in rows]
    en = [int(r["End_Timestamp"]) for r in rows]
    dur = sorted(e - b for b, e in zip(st, en))
    gaps = sorted(st[i + 1] - en[i] for i in range(len(rows) - 1))
    med = lambda v: v[len(v) // 2] if v else float("nan")  # noqa: E731
    mean = lambda v: sum(v) / len(v) if v else float("nan")  # noqa: E731
    period = (st[-1] - st[0]) / (len(st) - 1) if len(st) > 1 else float("nan")
    api = {r["Name"]: r for r in _rocprof_rows(directory, "hip_api_stats.csv")}
    lines = [f"# Kernel trace of `bench.py --profile-path {path}` on MI355X", "",
             "Command (from the repository root, on the machine with the GPU):", "", f"    {command}", "",
             f"Kernel `{rows[0]['Kernel_Name'] if rows else k['match']}`: {len(rows)} dispatches "
             "(warm-up included).  Times in microseconds.", "",
             "| Quantity | Median | Mean | Min | Max |", "|---|---|---|---|---|",
             f"| kernel duration | {med(dur) / 1e3:.2f} | {mean(dur) / 1e3:.2f} | {dur[0] / 1e3:.2f} | {dur[-1] / 1e3:.2f} |"
             if dur else "| kernel duration | - | - | - | - |",
             f"| idle gap to the next dispatch | {med(gaps) / 1e3:.2f} | {mean(gaps) / 1e3:.2f} | {gaps[0] / 1e3:.2f} | "
             f"{gaps[-1] / 1e3:.2f} |" if gaps else "| idle gap | - | - | - | - |",
             f"| dispatch period (start to start) | | {period / 1e3:.2f} | | |", ""]
    if timed:
        if skip is None:
            sel, where = slice(-timed, None), "the last ones of the kernel"
        else:
            sel, where = slice(skip, skip + timed), f"those after the first {skip}"
        part = [e - b for b, e in zip(st[sel], en[sel])]
        span = (en[sel][-1] - st[sel][0]) / len(part) if part else float("nan")
        lines += [f"The timed region's {timed} dispatches ({where}): mean duration {sum(part) / len(part) / 1e3:.2f} us; "
                  f"first start to last end {span / 1e3:.2f} us per dispatch.", ""]
    stats = _rocprof_rows(directory, "kernel_stats.csv")
    if stats:
        lines += ["All kernels of the run (kernel_stats.csv):", "", "| Kernel | Calls | Average us | Min us | Max us | % of GPU time |",
                  "|---|---|---|---|---|---|"]
        for r in stats:
            lines.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                         f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
        lines.append("")
    calls = [n for n in ("hipGraphLaunch", "hipLaunchKernel", "hipModuleLaunchKernel", "hipExtLaunchKernel") if n in api]
    if calls:
        lines += ["Host time of the launch calls (hip_api_stats.csv):", "", "| Call | Calls | Average us |", "|---|---|---|"]
        lines += [f"| {n} | {api[n]['Calls']} | {float(api[n]['AverageNs']) / 1e3:.2f} |" for n in calls]
        lines.append("")
    return "\n".join(lines)


def profile_path(name, steps, warmup, calibrate=False):
    """Runs one path of the hot path `warmup` times untimed and `steps` times
    timed with HIP events on the launching stream; prints one JSON line with
    the average per launch."""
    import torch
    sys.path.insert(0, ROOT)
    import paper_2602_05606_amd as kp
    import workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    c2 = workloads.C2
    launches, fn, units, unit_bytes = 1, None, 0, 0
    keep = []
    if name in ("c1-fp64",):
        c1 = workloads.C1
        out = kp.sample(c1["kappa"], c1["theta"], c1["n"], c1["seed"], precision=kp.FP64)
        fn = lambda: kp.sample(c1["kappa"], c1["theta"], c1["n"], c1["seed"], precision=kp.FP64, out=out)
        units, unit_bytes = c1["n"], 24
    elif name in ("c2-fp32", "c2-fp64", "store-fp32", "store-fp64", "exact-t", "exact-pareto"):
        prec = kp.FP64 if name.endswith("fp64") else kp.FP32
        out = tuple(torch.empty(c2["n"], dtype=torch.float64 if prec == kp.FP64 else torch.float32, device=dev)
                    for _ in range(3))
        launches = len(c2["kappas"])
        if name.startswith("store"):
            fn = lambda: [kp.fill_probe(c2["n"], prec, out) for _ in c2["kappas"]]
        elif name == "exact-t":
            fn = lambda: [kp.sample_exact_t(k, c2["theta"], c2["n"], c2["seed"], precision=prec, out=out)
                          for k in c2["kappas"]]
        elif name == "exact-pareto":
            fn = lambda: [kp.sample_exact_pareto(k, c2["theta"], c2["n"], c2["seed"], precision=prec, out=out)
                          for k in c2["kappas"]]
        else:
            fn = lambda: [kp.sample(k, c2["theta"], c2["n"], c2["seed"], precision=prec, out=out)
                          for k in c2["kappas"]]
        units, unit_bytes = c2["n"], 24 if prec == kp.FP64 else 12
    elif name in ("c3-fp32", "c3-fp64"):
        c3 = workloads.C3
        prec = kp.FP64 if name.endswith("fp64") else kp.FP32
        gen = torch.Generator(device=dev).manual_seed(c3["grad_seed"])
        g = torch.randn((3, c3["n"]), generator=gen, device=dev,
                        dtype=torch.float64 if prec == kp.FP64 else torch.float32)
        ws = torch.empty(kp.backward_workspace_bytes(c3["n"]), dtype=torch.uint8, device=dev)
        grad = torch.empty(2, dtype=torch.float64, device=dev)
        fn = lambda: kp.sample_backward(c3["kappa"], c3["theta"], c3["n"], c3["seed"], g[0], g[1], g[2],
                                        precision=prec, workspace=ws, out=grad)
        units, unit_bytes = c3["n"], 24 if prec == kp.FP64 else 12
    elif name.startswith("c4"):
        plan = kp.Plan(workloads.batched_segments(), workloads.C4["seed"], kp.FP32)
        keep.append(plan)
        outb = plan.outputs()
        units, unit_bytes = plan.total, 12
        if name == "c4-direct":
            fn = lambda: plan.launch(outb)
        elif name == "c4-graph":
            plan.graph_launch(outb)
            fn = lambda: plan.graph_launch(outb)
        elif name == "c4-pic":
            plan.set_cells(workloads.batched_cells())
            posb = plan.outputs()
            fn = lambda: plan.launch_pic(posb, outb)
            unit_bytes = 24
        else:  # c4-caller-graph: 8 plan launches captured into one graph of the caller's
            bufs = [plan.outputs() for _ in range(8)]
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                for b in bufs:
                    plan.launch(b)
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            cg = torch.cuda.CUDAGraph()
            with torch.cuda.graph(cg):
                for b in bufs:
                    plan.launch(b)
            keep.append((bufs, cg))
            fn, launches = cg.replay, len(bufs)
    elif name == "hist-fp32":
        # Test 2's speed histogram of 1e8 FP32 particles (kappa 3), 100 bins of theta/5 and the overflow bin
        v = kp.sample(3.0, 1.0, 10 ** 8, 1, precision=kp.FP32)
        counts = torch.zeros(101, dtype=torch.int64, device=dev)
        keep.append((v, counts))
        fn = lambda: kp.speed_histogram(*v, theta=1.0, bin_width=0.2, nbins=100, counts=counts)
        units, unit_bytes = 10 ** 8, 12
    elif name == "copy":
        src = torch.empty(300_000_000, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        fn = lambda: kp.copy_probe(src, dst)
        units, unit_bytes = 1, 2 * src.numel() * 4
    else:
        raise SystemExit(f"unknown profile path {name}; choose from {', '.join(PROFILE_PATHS)}")
    log(f"profile path {name}: {warmup} untimed, {steps} timed calls of {launches} launch(es)")
    ms = time_launches(fn, steps, torch, warm=warmup, warm_ms=0) / launches
    if calibrate:
        # plain copies of 1.2e9 bytes each way: the scale of the traffic counters
        src = torch.empty(300_000_000, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            kp.copy_probe(src, dst)
        torch.cuda.synchronize()
        del src, dst
    rec = {"profile_path": name, "calls": steps, "warmup": warmup, "launches_per_call": launches,
           "avg_launch_ms": ms, "units_per_launch": units, "algorithmic_bytes_per_launch": units * unit_bytes,
           "GB_per_s": units * unit_bytes / (ms * 1e-3) / 1e9}
    print(json.dumps(rec), flush=True)
    for k in keep:
        if isinstance(k, kp.Plan):
            k.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50,
                    help="untimed steps first: the GPU clock ramps up over about 20 steps (40 ms) after idle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="same as --extras none")
    ap.add_argument("--extras", default="all",
                    help="comma list of extra measurements to run after the timed steps, 'all' or 'none': "
                         + ",".join(EXTRAS))
    ap.add_argument("--calibrate", action="store_true",
                    help="also run the plain copy probe on 1.2e9 bytes (3 launches) and the store probe, so that "
                         "rocprofv3 counters can be scaled against known traffic")
    ap.add_argument("--profile-path", choices=PROFILE_PATHS,
                    help="run only this path's launches (--warmup untimed, --steps timed) for a profiler, print its "
                         "average launch time and exit")
    ap.add_argument("--summarise", metavar="DIR",
                    help="reduce the rocprofv3 output under DIR of a --profile-path run (counters or kernel trace) "
                         "to the summary committed under profiles/, print it and exit (no GPU)")
    ap.add_argument("--command", default="", help="with --summarise: the command that produced DIR, recorded")
    ap.add_argument("--mad-per-unit", type=float, default=None,
                    help="with --summarise of a VALU pass: v_mad_u64_u32 per particle from the kernel's ISA")
    ap.add_argument("--note", default=None, help="with --summarise: a note recorded with the summary")
    ap.add_argument("--timed-dispatches", type=int, default=None,
                    help="with --summarise of a kernel trace: how many dispatches the timed region holds (the last "
                         "ones, or those after --skip-dispatches)")
    ap.add_argument("--skip-dispatches", type=int, default=None,
                    help="with --timed-dispatches: dispatches of the kernel before the timed region")
    args = ap.parse_args()
    if args.summarise:
        if not args.profile_path:
            ap.error("--summarise needs --profile-path")
        if _rocprof_rows(args.summarise, "counter_collection.csv"):
            print(json.dumps(summarise_counters(args.summarise, args.profile_path, args.command, args.mad_per_unit,
                                                args.note), indent=1))
        else:
            print(summarise_trace(args.summarise, args.profile_path, args.command, args.timed_dispatches,
                                  args.skip_dispatches))
        return
    if args.profile_path:
        if args.gpus != 1:
            ap.error("profile paths run on one GPU")
        profile_path(args.profile_path, args.steps, args.warmup, args.calibrate)
        return
    chosen = set(EXTRAS) if args.extras == "all" else set() if args.extras == "none" else set(args.extras.split(","))
    if args.no_extras:
        chosen = set()
    unknown = chosen - set(EXTRAS)
    if unknown:
        ap.error(f"unknown extras {sorted(unknown)}; choose from {','.join(EXTRAS)}")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the generator needs no communication, and a run on N GPUs is "
              "N independent counter ranges. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    sys.path.insert(0, ROOT)
    import paper_2602_05606_amd as kp
    import workloads

    c = workloads.C2
    n, kappas, theta, seed = c["n"], c["kappas"], c["theta"], c["seed"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"{torch.cuda.get_device_name(dev)}; library {kp.version()}")
    out32 = tuple(torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3))

    def step(out=out32, prec=kp.FP32, events=None):
        for k in kappas:
            if events is not None:
                events[0].append(torch.cuda.Event(enable_timing=True))
                events[1].append(torch.cuda.Event(enable_timing=True))
                events[0][-1].record()
            kp.sample(k, theta, n, seed, precision=prec, out=out)
            if events is not None:
                events[1][-1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done; timing {args.steps} steps")
    # The timed region holds the K steps and one HIP event on each side, on the
    # stream the library launches on: events recorded between launches cost
    # about 1.5% of a step, so the per-step and per-launch times of the timing
    # object come from a second run of steps after the timed one.
    region = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    region[0].record()
    for _ in range(args.steps):
        step()
    region[1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # average launch over the timed region (it includes the short idle gaps between launches)
    avg_kernel_ms = region[0].elapsed_time(region[1]) / (args.steps * len(kappas))
    particles = args.steps * len(kappas) * n
    value = particles / elapsed
    events = ([], [])
    step_ev = []
    for _ in range(max(args.steps, 10)):
        step_ev.append(torch.cuda.Event(enable_timing=True))
        step_ev[-1].record()
        step(events=events)
    step_ev.append(torch.cuda.Event(enable_timing=True))
    step_ev[-1].record()
    torch.cuda.synchronize()
    kernel_ms = [s.elapsed_time(e) for s, e in zip(*events)]
    step_ms = [a.elapsed_time(b) for a, b in zip(step_ev[:-1], step_ev[1:])]
    launch_bytes = 12 * n
    achieved = launch_bytes / (avg_kernel_ms * 1e-3) / 1e9
    log(f"timed: {elapsed * 1e3 / args.steps:.3f} ms/step, {value:.4e} particles/s, kernel {avg_kernel_ms:.4f} ms "
        f"= {achieved:.1f} GB/s")

    result = {
        "metric": METRIC, "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "C2 single-species sweep: 1e8 particles per kappa in {1.6,2,3,4,6,10}, theta 1, "
                               "FP32 bulk + FP64 tail (1-U1 < 2^-20), Philox4x32-10 seed 1, SoA outputs resident in HBM",
                   "particles_per_step": len(kappas) * n, "kappas": list(kappas), "precision": "FP32+FP64tail"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(launch_bytes),
                     "kernel": KERNELS["c2-fp32"]["label"],
                     "algorithmic_bytes_per_launch": launch_bytes, "avg_launch_ms": avg_kernel_ms},
        "timing": dict(step_protocol(step_ms, len(kappas) * n), launch_ms_mean=sum(kernel_ms) / len(kernel_ms),
                       how="a second run of steps after the timed one, with HIP events between steps and around "
                           "each launch"),
    }
    probe = launch_clock_probe(kp, torch, kappas, theta, n, seed, out32)
    result["roofline_alu"] = None  # filled in after the extras, when the stamps are read back

    if args.calibrate:
        src = torch.empty(300_000_000, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            kp.copy_probe(src, dst)
        for _ in range(3):
            kp.fill_probe(n, kp.FP32, out32)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copies done (copy_kernel: 1.2e9 bytes read and written per launch; "
            "fill_kernel: 1.2e9 bytes written per launch)")

    extras = {}
    path_ms = {}  # path -> (units per launch, average launch ms), for the roofline objects
    if "rates" in chosen:
        per_kappa = {}
        for k in kappas:
            ms = time_launches(lambda: kp.sample(k, theta, n, seed, precision=kp.FP32, out=out32), 20, torch, warm=10)
            per_kappa[str(k)] = n / (ms * 1e-3)
        extras["fp32_per_kappa_particles_per_s"] = per_kappa
        ms = time_launches(lambda: kp.sample(math.inf, theta, n, seed, precision=kp.FP32, out=out32), 20, torch,
                           warm=10)
        extras["maxwell_limit_fp32_particles_per_s"] = n / (ms * 1e-3)
        fill_ms = time_launches(lambda: kp.fill_probe(n, kp.FP32, out32), 20, torch, warm=10)
        extras["store_probe_fp32"] = {"GB_per_s": 12 * n / (fill_ms * 1e-3) / 1e9,
                                      "particles_per_s": n / (fill_ms * 1e-3)}
        result["roofline"]["frac_of_store_probe"] = achieved / extras["store_probe_fp32"]["GB_per_s"]
        log("store probe done")
        exact = {}
        for k in kappas:
            t_ms = time_launches(lambda: kp.sample_exact_t(k, theta, n, seed, precision=kp.FP32, out=out32), 3, torch)
            p_ms = time_launches(lambda: kp.sample_exact_pareto(k, theta, n, seed, precision=kp.FP32, out=out32), 3,
                                 torch)
            rate_t, rate_p = n / (t_ms * 1e-3), n / (p_ms * 1e-3)
            exact[str(k)] = {"t_gamma": rate_t, "pareto": rate_p,
                             "approx_speedup_vs_t": per_kappa[str(k)] / rate_t,
                             "approx_speedup_vs_pareto": per_kappa[str(k)] / rate_p}
        extras["exact_generators_fp32_particles_per_s"] = exact
        log("exact generators done")
    if "simt" in chosen:
        extras["simt_rejection_loops"] = simt_loop_counts(kp, torch, kappas, theta, seed)
        log("SIMT loop counts done")
    if "ks" in chosen:
        extras["ks_vs_exact_cdf"] = ks_table(kp, torch, kappas, theta, seed, out32)
        log("KS distances done")
    if "test2" in chosen:
        extras["relative_entropy_test2"] = relative_entropy_test2(kp, torch, dev)
        path_ms["hist-fp32"] = (10 ** 8, extras["relative_entropy_test2"]["histogram_ms"])
        log("relative-entropy test done")
    if "survey" in chosen:
        extras["divergence_survey"] = divergence_survey(kp, torch, dev)
        log("divergence survey done")
    if "c5" in chosen:
        c5 = workloads.C5
        chunk_out = tuple(t[:c5["chunk"]] for t in out32) if c5["chunk"] <= n else None
        if chunk_out is None:
            chunk_out = tuple(torch.empty(c5["chunk"], dtype=torch.float32, device=dev) for _ in range(3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for off, cnt in workloads.c5_chunks():
            kp.sample(c5["kappa"], c5["theta"], cnt, c5["seed"], counter_offset=off, precision=kp.FP32,
                      out=tuple(t[:cnt] for t in chunk_out))
        torch.cuda.synchronize()
        dt5 = time.perf_counter() - t0
        extras["c5_stream_fp32"] = {"particles": c5["n"], "chunks": len(workloads.c5_chunks()), "s": dt5,
                                    "particles_per_s": c5["n"] / dt5}
        del chunk_out
    del out32
    if "fp64" in chosen:
        out64 = tuple(torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
        fp64 = {}
        for k in kappas:
            ms = time_launches(lambda: kp.sample(k, theta, n, seed, precision=kp.FP64, out=out64), 10, torch, warm=5)
            fp64[str(k)] = {"particles_per_s": n / (ms * 1e-3), "GB_per_s": 24 * n / (ms * 1e-3) / 1e9}
        extras["fp64_per_kappa"] = fp64
        path_ms["c2-fp64"] = (n, n / (sum(v["particles_per_s"] for v in fp64.values()) / len(fp64)) * 1e3)
        fill64 = time_launches(lambda: kp.fill_probe(n, kp.FP64, out64), 3, torch)
        extras["store_probe_fp64_GB_per_s"] = 24 * n / (fill64 * 1e-3) / 1e9
        del out64
        log("FP64 sweep done")
    if "backward" in chosen:
        c3 = workloads.C3
        gen = torch.Generator(device=dev).manual_seed(c3["grad_seed"])
        g = torch.randn((3, c3["n"]), generator=gen, device=dev, dtype=torch.float32)
        ws = torch.empty(kp.backward_workspace_bytes(c3["n"]), dtype=torch.uint8, device=dev)
        bw_ms = time_launches(lambda: kp.sample_backward(c3["kappa"], c3["theta"], c3["n"], c3["seed"], g[0], g[1],
                                                         g[2], precision=kp.FP32, workspace=ws), 30, torch, warm=10)
        extras["backward_c3"] = {"particles_per_s": c3["n"] / (bw_ms * 1e-3), "ms": bw_ms,
                                 "GB_per_s_read": 12 * c3["n"] / (bw_ms * 1e-3) / 1e9}
        path_ms["c3-fp32"] = (c3["n"], bw_ms)
        # the same backward in FP64 (FP64 upstream gradient, FP64 inversion throughout)
        g64 = g.double()
        del g
        bw64_ms = time_launches(lambda: kp.sample_backward(c3["kappa"], c3["theta"], c3["n"], c3["seed"], g64[0],
                                                           g64[1], g64[2], precision=kp.FP64, workspace=ws), 20, torch,
                                 warm=5)
        extras["backward_c3"]["fp64"] = {"particles_per_s": c3["n"] / (bw64_ms * 1e-3), "ms": bw64_ms,
                                         "GB_per_s_read": 24 * c3["n"] / (bw64_ms * 1e-3) / 1e9}
        path_ms["c3-fp64"] = (c3["n"], bw64_ms)
        del g64
        log("backward done")
    if "batched" in chosen:
        segs = workloads.batched_segments()
        with kp.Plan(segs, workloads.C4["seed"], kp.FP32) as plan:
            outb = plan.outputs()
            default_shape = plan.shape
            plan.launch(outb)
            tuned = plan.autotune(outb, reps=5)
            # launches of 20-50 us: 200 back to back, after 20 untimed
            direct_ms = time_launches(lambda: plan.launch(outb), 200, torch, warm=20)
            plan.graph_launch(outb)
            graph_ms = time_launches(lambda: plan.graph_launch(outb), 200, torch, warm=20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(50):
                plan.graph_launch(outb)
            torch.cuda.synchronize()
            wall_ms = (time.perf_counter() - t0) * 1e3 / 50
            # the plan's launch as nodes of a caller's graph (a PIC step captures its whole
            # step): 8 launches into 8 output sets per replay, so hipGraphLaunch's host
            # cost is paid once per 8 kernels
            caller_bufs = [plan.outputs() for _ in range(8)]
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                for b in caller_bufs:
                    plan.launch(b)
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            caller_graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(caller_graph):
                for b in caller_bufs:
                    plan.launch(b)
            caller_ms = time_launches(caller_graph.replay, 50, torch, warm=5) / len(caller_bufs)
            del caller_graph, caller_bufs
            # the single-species kernel on the same number of particles, for comparison
            single_ms = time_launches(lambda: kp.sample(3.0, 1.0, plan.total, 4, precision=kp.FP32, out=outb), 200,
                                      torch, warm=20)
            # fused particle loading: positions in each cell's box with the velocities
            plan.set_cells(workloads.batched_cells())
            posb = plan.outputs()
            plan.launch_pic(posb, outb)
            pic_ms = time_launches(lambda: plan.launch_pic(posb, outb), 200, torch, warm=20)
            plan.graph_launch_pic(posb, outb)
            pic_graph_ms = time_launches(lambda: plan.graph_launch_pic(posb, outb), 200, torch, warm=20)
            extras["batched_c4"] = {"particles": plan.total, "segments": len(segs), "default_shape": default_shape,
                                    "tuned_shape": tuned, "direct_launch_ms": direct_ms, "graph_launch_ms": graph_ms,
                                    "graph_wall_ms": wall_ms, "particles_per_s": plan.total / (graph_ms * 1e-3),
                                    "direct_launch_particles_per_s": plan.total / (direct_ms * 1e-3),
                                    "in_caller_graph_ms_per_launch": caller_ms,
                                    "in_caller_graph_particles_per_s": plan.total / (caller_ms * 1e-3),
                                    "single_species_same_size_ms": single_ms,
                                    "pic_positions_and_velocities": {
                                        "direct_launch_ms": pic_ms, "graph_launch_ms": pic_graph_ms,
                                        "particles_per_s": plan.total / (pic_ms * 1e-3),
                                        "GB_per_s_written": 24 * plan.total / (pic_ms * 1e-3) / 1e9}}
            path_ms["c4-direct"] = (plan.total, direct_ms)
            path_ms["c4-graph"] = (plan.total, graph_ms)
            path_ms["c4-pic"] = (plan.total, pic_ms)
        log("batched done")
    if extras:
        result["extras"] = extras
    clock = finish_clock_probe(probe, torch, avg_kernel_ms)
    log(f"core clock during the workload: {clock['core_clock_ghz']:.3f} GHz "
        f"(probe launch {clock['probe_launch_ms']:.4f} ms against {avg_kernel_ms:.4f} ms timed)")
    costs = measure_issue_costs(kp)
    log("issue costs (SIMD-cycles per wave64 instruction): " + ", ".join(f"{k} {v:.2f}" for k, v in costs.items()))
    result["roofline_alu"] = alu_roofline(n / (avg_kernel_ms * 1e-3), clock, costs)
    # the other paths' kernels: HBM fraction of their timed launches, VALU-issue
    # fraction at 2.4 GHz (the core clock above was measured on C2 FP32 only)
    result["rooflines"] = {p: hbm_roofline(p, u, ms, None, costs) for p, (u, ms) in path_ms.items()}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline()
        log("cpu baseline done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
