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
KERNEL_SOURCES = ["paper_2602_05606_amd/csrc/kappa_device.hpp", "paper_2602_05606_amd/csrc/forward.hip",
                  "paper_2602_05606_amd/csrc/kappa_params.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_forward_fp32_c2.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_forward_fp32_c2.json")
# VALU issue capacity: 256 CUs x 4 SIMDs x 2.4 GHz.  Nominal costs: a wave64
# full-rate FP32 instruction occupies a SIMD for 2 cycles (the 157.3 TFLOP/s
# FP32 vector peak), a quarter-rate one 8.  The bench prices the kernel with the
# costs the issue probe measures instead (v_mad_u64_u32 takes about 4).
SIMD_COUNT = 256 * 4
SIMD_CYCLES_PER_S = SIMD_COUNT * 2.4e9
CYCLES_FULL, CYCLES_QUARTER = 2, 8


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(launch_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when they are missing or were taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return {"write_bytes": t["write_bytes_per_launch"], "fetch_bytes": t["fetch_bytes_per_launch"],
            "algorithmic_bytes": launch_bytes, "calibration": t.get("calibration")}


def measure_issue_costs(kp):
    """SIMD-cycles per wave64 instruction of the classes the forward kernel
    issues, measured on this chip (kappa_issue_probe: saturated issue, in-kernel
    clock, so independent of the clock the chip holds)."""
    return {name: kp.issue_cost(name)["cycles"]
            for name in ("fma_f32", "transcendental_f32", "mad_u64_u32", "fma_f32_literal")}


def alu_roofline(particles_per_s, clock=None, costs=None):
    """VALU-issue roofline of the dominant kernel from its measured instruction
    counts (rocprofv3 SQ_INSTS_VALU, SQ_INSTS_VALU_TRANS_F32 and the static
    v_mad_u64_u32 count), priced with the issue costs measured by the issue
    probe (`costs`; without them the nominal 2, 8 and 8 SIMD-cycles), or None
    when the counts were taken on other kernel sources.  Full-rate
    instructions are priced as v_fma_f32 with three VGPR operands; with the
    probe's literal-operand v_fma_f32 as well, the range between the two
    prices is reported too.  The peak is the
    2.4 GHz one; with `clock` (the core clock measured by the clock probe
    during the same workload) the fraction of the issue capacity at that
    clock is added."""
    try:
        with open(VALU_FILE) as f:
            v = json.load(f)
    except (OSError, ValueError):
        return None
    if v.get("kernel_source_sha") != kernel_source_hash():
        return None
    c = costs or {"fma_f32": CYCLES_FULL, "transcendental_f32": CYCLES_QUARTER, "mad_u64_u32": CYCLES_QUARTER}
    trans, mad = v["trans_per_particle"], v["mad_u64_per_particle"]
    full = v["valu_per_particle"] - trans - mad
    cycles_per_particle = (c["fma_f32"] * full + c["transcendental_f32"] * trans + c["mad_u64_u32"] * mad) / 64.0
    achieved = particles_per_s * cycles_per_particle
    out = {"bound": "alu", "achieved": achieved, "peak": SIMD_CYCLES_PER_S, "unit": "SIMD-cycles/s",
           "frac": achieved / SIMD_CYCLES_PER_S, "valu_per_particle": v["valu_per_particle"],
           "per_particle": {"full_rate": full, "transcendental": trans, "mad_u64_u32": mad},
           "simd_cycles_per_instruction": c,
           "costs_from": "kappa_issue_probe on this chip" if costs else "nominal rates",
           "simd_cycles_per_particle": cycles_per_particle}
    low = None
    if "fma_f32_literal" in c:
        # the full-rate price with a literal operand (no three-VGPR operand reads): the low end
        low = (c["fma_f32_literal"] * full + c["transcendental_f32"] * trans + c["mad_u64_u32"] * mad) / 64.0
        out["simd_cycles_per_particle_range"] = [low, cycles_per_particle]
    if clock:
        at_clock = SIMD_COUNT * clock["core_clock_ghz"] * 1e9
        out.update({"measured_clock": clock, "peak_at_measured_clock": at_clock,
                    "frac_at_measured_clock": achieved / at_clock})
        if low is not None:
            out["frac_at_measured_clock_range"] = [particles_per_s * low / at_clock, achieved / at_clock]
    return out


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


def time_launches(fn, reps, torch, warm=2):
    """Average duration (ms) of fn() over reps back-to-back calls after `warm`
    untimed ones: HIP events on the current stream (the one the library
    launches on) before the first timed call and after the last, so host-side
    call overhead overlaps the GPU work instead of being counted as idle time."""
    for _ in range(warm):
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


def cpu_baseline(seconds_target=15.0):
    """The oracle (FP64 arithmetic at the FP32 mode's uniforms, OpenMP over
    particles) timed on the host over a bounded sample of the C2 workload."""
    import numpy as np  # noqa: F401
    sys.path.insert(0, ROOT)
    import oracle
    import workloads
    c = workloads.C2
    probe_n = 200_000
    t0 = time.perf_counter()
    oracle.sample(c["kappas"][0], c["theta"], probe_n, c["seed"], mode=oracle.MODE_FP32)
    rate = probe_n / max(time.perf_counter() - t0, 1e-6)
    per_kappa = int(min(c["n"], max(1e5, rate * seconds_target / len(c["kappas"]))))
    t0 = time.perf_counter()
    for k in c["kappas"]:
        oracle.sample(k, c["theta"], per_kappa, c["seed"], mode=oracle.MODE_FP32)
    dt = time.perf_counter() - t0
    return {"value": per_kappa * len(c["kappas"]) / dt, "unit": "particles/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {per_kappa} particles of each of the 6 C2 kappa values (FP32-mode uniforms, "
                      f"FP64 arithmetic), {dt:.1f} s on the host"}


EXTRAS = ("rates", "simt", "ks", "test2", "survey", "c5", "fp64", "backward", "batched")


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
    args = ap.parse_args()
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
    events = ([], [])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(events=events)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = [s.elapsed_time(e) for s, e in zip(*events)]
    avg_kernel_ms = sum(kernel_ms) / len(kernel_ms)
    particles = args.steps * len(kappas) * n
    value = particles / elapsed
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
                     "kernel": "forward_kernel<FP32 tail, 4 particles/thread>",
                     "algorithmic_bytes_per_launch": launch_bytes, "avg_launch_ms": avg_kernel_ms},
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
                                                         g[2], precision=kp.FP32, workspace=ws), 20, torch)
        extras["backward_c3"] = {"particles_per_s": c3["n"] / (bw_ms * 1e-3), "ms": bw_ms,
                                 "GB_per_s_read": 12 * c3["n"] / (bw_ms * 1e-3) / 1e9}
        # the same backward in FP64 (FP64 upstream gradient, FP64 inversion throughout)
        g64 = g.double()
        del g
        bw64_ms = time_launches(lambda: kp.sample_backward(c3["kappa"], c3["theta"], c3["n"], c3["seed"], g64[0],
                                                           g64[1], g64[2], precision=kp.FP64, workspace=ws), 10, torch)
        extras["backward_c3"]["fp64"] = {"particles_per_s": c3["n"] / (bw64_ms * 1e-3), "ms": bw64_ms,
                                         "GB_per_s_read": 24 * c3["n"] / (bw64_ms * 1e-3) / 1e9}
        del g64
        log("backward done")
    if "batched" in chosen:
        segs = workloads.batched_segments()
        with kp.Plan(segs, workloads.C4["seed"], kp.FP32) as plan:
            outb = plan.outputs()
            default_shape = plan.shape
            plan.launch(outb)
            tuned = plan.autotune(outb, reps=5)
            direct_ms = time_launches(lambda: plan.launch(outb), 20, torch)
            plan.graph_launch(outb)
            graph_ms = time_launches(lambda: plan.graph_launch(outb), 20, torch)
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
            caller_ms = time_launches(caller_graph.replay, 10, torch) / len(caller_bufs)
            del caller_graph, caller_bufs
            # the single-species kernel on the same number of particles, for comparison
            single_ms = time_launches(lambda: kp.sample(3.0, 1.0, plan.total, 4, precision=kp.FP32, out=outb), 20,
                                      torch)
            # fused particle loading: positions in each cell's box with the velocities
            plan.set_cells(workloads.batched_cells())
            posb = plan.outputs()
            plan.launch_pic(posb, outb)
            pic_ms = time_launches(lambda: plan.launch_pic(posb, outb), 20, torch)
            plan.graph_launch_pic(posb, outb)
            pic_graph_ms = time_launches(lambda: plan.graph_launch_pic(posb, outb), 20, torch)
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
        log("batched done")
    if extras:
        result["extras"] = extras
    clock = finish_clock_probe(probe, torch, avg_kernel_ms)
    log(f"core clock during the workload: {clock['core_clock_ghz']:.3f} GHz "
        f"(probe launch {clock['probe_launch_ms']:.4f} ms against {avg_kernel_ms:.4f} ms timed)")
    costs = measure_issue_costs(kp)
    log("issue costs (SIMD-cycles per wave64 instruction): " + ", ".join(f"{k} {v:.2f}" for k, v in costs.items()))
    result["roofline_alu"] = alu_roofline(n / (avg_kernel_ms * 1e-3), clock, costs)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline()
        log("cpu baseline done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
