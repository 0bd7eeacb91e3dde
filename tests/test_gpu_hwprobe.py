"""GPU hardware probes: the facts about gfx950 that the FP32 design and the
VALU-issue roofline rest on.

* issue costs (kappa_issue_probe, SIMD-cycles per wave64 instruction at
  saturation, clock-independent): v_fma_f32 about 2 (with three VGPR operands
  or with a literal), a transcendental about
  8, v_mad_u64_u32 about 4, v_fma_f64 about 4, v_bitop3_b32 about 2;
* a stream mixing one transcendental with three v_fma_f32 costs at least the
  sum of the two classes' separate costs: the transcendental unit does not
  run beside full-rate work, so a transcendental taken off the path saves
  its whole cost;
* accuracy of the hardware transcendentals the FP32 inversion uses
  (kappa_transcendental_probe) against float64 references: v_log_f32 within
  2 ulp of its result, also next to 1 where log2 x is small; v_exp_f32,
  v_sqrt_f32, v_rsq_f32 and v_rcp_f32 within 2 ulp; v_sin_f32 / v_cos_f32 in
  revolutions within 2e-7 absolute.
"""
import numpy as np
import pytest
import torch

import paper_2602_05606_amd as kp

pytestmark = pytest.mark.gpu

ULP = 2.0 ** -23  # float ulp relative to the value, at most


@pytest.mark.parametrize("op,lo,hi", [("fma_f32", 1.8, 2.8), ("transcendental_f32", 6.5, 10.0),
                                      ("mad_u64_u32", 3.5, 6.5), ("fma_f64", 3.5, 5.5), ("bitop3_b32", 1.8, 3.0),
                                      ("fma_f32_literal", 1.8, 2.8)])
def test_issue_costs(op, lo, hi):
    r = kp.issue_cost(op)
    print(f"{op}: {r['cycles']:.3f} SIMD-cycles per wave64 instruction at {r['clock_ghz']:.3f} GHz")
    assert lo < r["cycles"] < hi
    assert 0.3 < r["clock_ghz"] < 2.45


def test_transcendental_does_not_overlap_full_rate_work():
    fma, log = kp.issue_cost("fma_f32")["cycles"], kp.issue_cost("transcendental_f32")["cycles"]
    mixed = 4 * kp.issue_cost("log_plus_3fma_f32")["cycles"]  # per step of 1 log + 3 fma
    print(f"1 log + 3 fma: {mixed:.2f} SIMD-cycles against {log:.2f} + 3 x {fma:.2f} = {log + 3 * fma:.2f} apart")
    assert mixed > 0.95 * (log + 3 * fma)


def _run(op, x):
    return kp.transcendental_probe(op, torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)


def test_log2_relative_to_its_result_even_near_one():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(2.0 ** -30, 1.0, 1 << 20), rng.uniform(0.5, 2.0, 1 << 20),
                        1.0 + rng.uniform(-2.0 ** -10, 2.0 ** -10, 1 << 16)]).astype(np.float32)
    x = x[x != 1.0]
    ref = np.log2(x.astype(np.float64))
    rel = np.abs(_run("log2", x) - ref) / np.abs(ref)
    print(f"v_log_f32: max relative error {rel.max():.3e}")
    assert rel.max() < 2 * ULP


@pytest.mark.parametrize("op,lo,hi,ref", [("exp2", -40.0, 1.0, np.exp2), ("sqrt", 2.0 ** -40, 4.0, np.sqrt),
                                          ("rsq", 2.0 ** -40, 4.0, lambda v: 1.0 / np.sqrt(v)),
                                          ("rcp", 2.0 ** -20, 4.0, lambda v: 1.0 / v)])
def test_within_two_ulp(op, lo, hi, ref):
    x = np.random.default_rng(6).uniform(lo, hi, 1 << 20).astype(np.float32)
    want = ref(x.astype(np.float64))
    rel = np.abs(_run(op, x) - want) / np.abs(want)
    print(f"{op}: max relative error {rel.max():.3e}")
    assert rel.max() < 2 * ULP


@pytest.mark.parametrize("op,fn", [("sin_rev", np.sin), ("cos_rev", np.cos)])
def test_sin_cos_in_revolutions(op, fn):
    # the generator's argument: U3 in (0, 1) (2 pi U3 radians)
    x = np.random.default_rng(7).uniform(0.0, 1.0, 1 << 20).astype(np.float32)
    err = np.abs(_run(op, x) - fn(2.0 * np.pi * x.astype(np.float64)))
    print(f"{op}: max absolute error {err.max():.3e}")
    assert err.max() < 2e-7
