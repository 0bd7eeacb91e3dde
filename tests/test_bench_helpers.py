"""Host-side helpers of bench.py that report accuracy next to the timings:
sup|G - F| (equal-KS-accuracy sample size) against the oracle's G."""
import os
import sys

import numpy as np
import pytest
from scipy import special

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import paper_2602_05606_amd as kp  # noqa: E402


@pytest.mark.parametrize("kappa", [1.6, 4.0, 10.0])
def test_sup_G_minus_F_against_the_oracle(orc, kappa):
    x = np.logspace(-6, 4, 20_001)
    G = np.array([orc.G(kappa, xi)[0] for xi in x])
    F = special.betainc(1.5, kappa - 0.5, x / (x + kappa))
    ref = float(np.max(np.abs(G - F)))
    got = bench.sup_G_minus_F(kp, kappa)
    # the bench's grid is 10x denser: it can only find a slightly larger supremum
    assert ref * (1 - 1e-9) <= got <= ref * 1.01


def test_alu_roofline_prices_at_the_issue_floors():
    """The VALU-issue roofline prices each instruction class at its issue
    floor (full rate 2, FP64 and 64-bit integer 4, transcendentals 8
    SIMD-cycles per wave64 instruction), so a kernel issuing at the chip's
    capacity reaches exactly 1."""
    prof = {"per_unit": {"valu": 115.0, "transcendental_f32": 9.0, "int64": 20.0}}
    r = bench.alu_roofline(3.5e11, {"core_clock_ghz": 2.0}, None, profile=prof)
    full = 115.0 - 9.0 - 20.0
    want = (2 * full + 8 * 9.0 + 4 * 20.0) / 64
    assert abs(r["simd_cycles_per_unit_at_floor"] - want) < 1e-12
    assert abs(r["frac"] - 3.5e11 * want / bench.SIMD_CYCLES_PER_S) < 1e-12
    assert abs(r["frac_at_measured_clock"] - 3.5e11 * want / (1024 * 2.0e9)) < 1e-12
    # the rate at which the mix fills every SIMD's issue slots gives 1
    full_rate = 1024 * 2.0e9 / want
    assert abs(bench.alu_roofline(full_rate, {"core_clock_ghz": 2.0}, None, profile=prof)["frac_at_measured_clock"]
               - 1.0) < 1e-12
    # an FP64 mix
    prof64 = {"per_unit": {"valu": 300.0, "f64": 150.0, "transcendental_f64": 5.0, "int64": 23.5}}
    r64 = bench.alu_roofline(1e11, None, None, profile=prof64)
    want64 = (2 * (300 - 150 - 5 - 23.5) + 4 * 150 + 8 * 5 + 4 * 23.5) / 64
    assert abs(r64["simd_cycles_per_unit_at_floor"] - want64) < 1e-12


def test_summarise_counters_and_trace(tmp_path):
    """The reductions of rocprofv3 CSVs behind the committed profiles: per
    unit instruction counts, traffic scaled by the copy kernel's reading, and
    the kernel trace's durations and gaps."""
    import csv
    d = tmp_path / "pmc" / "host" / "1"
    d.mkdir(parents=True)
    units = 10 ** 8
    rows = []
    for disp in range(3):
        rows.append({"Dispatch_Id": disp, "Kernel_Name": "void kappa::forward_kernel<1, 4, true, false>(...)",
                     "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 110.0 * units / 64})
        rows.append({"Dispatch_Id": disp, "Kernel_Name": "void kappa::forward_kernel<1, 4, true, false>(...)",
                     "Counter_Name": "SQ_INSTS_VALU_TRANS_F32", "Counter_Value": 9.0 * units / 64})
        rows.append({"Dispatch_Id": disp, "Kernel_Name": "void kappa::forward_kernel<1, 4, true, false>(...)",
                     "Counter_Name": "SQ_INSTS_VALU_INT64", "Counter_Value": 20.0 * units / 64})
    with open(d / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    out = bench.summarise_counters(str(tmp_path / "pmc"), "c2-fp32", "cmd")
    assert abs(out["per_unit"]["valu"] - 110.0) < 1e-9 and abs(out["per_unit"]["transcendental_f32"] - 9.0) < 1e-9
    assert abs(out["per_unit"]["int64"] - 20.0) < 1e-9 and out["dispatches"] == 3
    assert out["kernel_source_sha"] == bench.kernel_source_hash("c2-fp32")
    # traffic: WRITE_SIZE of the kernel against the copy kernel's reading (KiB)
    t = tmp_path / "traffic" / "h" / "2"
    t.mkdir(parents=True)
    rows = [{"Dispatch_Id": 0, "Kernel_Name": "forward_kernel<1, 4, true, false>", "Counter_Name": "WRITE_SIZE",
             "Counter_Value": 1.2e9 / 1024 * 0.5},
            {"Dispatch_Id": 1, "Kernel_Name": "copy_kernel(...)", "Counter_Name": "WRITE_SIZE",
             "Counter_Value": 1.2e9 / 1024 * 0.5}]
    with open(t / "y_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    tr = bench.summarise_counters(str(tmp_path / "traffic"), "c2-fp32", "cmd")
    assert abs(tr["write_bytes_per_launch"] - 1.2e9) < 1e-3
    assert abs(tr["calibration"]["write_counter_over_true"] - 0.5) < 1e-12
    # kernel trace: two dispatches 10 us long, 5 us apart
    k = tmp_path / "trace" / "h" / "3"
    k.mkdir(parents=True)
    rows = [{"Kernel_Name": "batched_kernel<1, 4, false, unsigned int>(...)", "Start_Timestamp": s, "End_Timestamp": s + 10_000}
            for s in (0, 15_000, 30_000)]
    with open(k / "z_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    md = bench.summarise_trace(str(tmp_path / "trace"), "c4-graph", "cmd")
    assert "| kernel duration | 10.00 |" in md and "| idle gap to the next dispatch | 5.00 |" in md
    md = bench.summarise_trace(str(tmp_path / "trace"), "c4-graph", "cmd", timed=2, skip=1)
    assert "2 dispatches (those after the first 1): mean duration 10.00 us; first start to last end 12.50 us" in md


def test_more_than_one_gpu_is_refused():
    import subprocess
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""
