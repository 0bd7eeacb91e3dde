"""GPU clock probe (kappa_clock_probe): the forward kernel with clock stamps.

* its outputs are bit-identical to kappa_sample's (same kernel body, same
  shape) in every precision, on ragged sizes and a counter range that
  crosses a 2^32 boundary;
* it reports the launch's workgroup count and stamps every workgroup with
  exit after entry on both counters;
* the core clock it derives lies in a physical range (a few hundred MHz to
  the 2.4 GHz maximum of the MI355X, with a small allowance for counter
  granularity) and the constant-rate counter runs at the device's stated
  rate: its span over a launch matches the launch's event time;
* too few stamps give KAPPA_ERANGE with the workgroup count filled in.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2602_05606_amd as kp
from paper_2602_05606_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [kp.FP32, kp.FP64, kp.FP32_NOTAIL])
@pytest.mark.parametrize("n,offset", [(1, 0), (1_000_003, 5), (3000, (1 << 32) - 1000)])
def test_outputs_equal_sample(prec, n, offset):
    ref = kp.sample(2.7, 1.1, n, 99, counter_offset=offset, seg_id=3, precision=prec)
    got, stamps, hz = kp.clock_probe(2.7, 1.1, n, 99, counter_offset=offset, seg_id=3, precision=prec)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    unroll = 2 if prec == kp.FP64 else 4
    groups = -(-n // unroll)  # threads of 256-thread workgroups, one group of particles each
    assert stamps.shape == (-(-groups // 256), 4)
    s = stamps.cpu().numpy()
    assert np.all(s[:, 2] >= s[:, 0]) and np.all(s[:, 3] >= s[:, 1])
    assert hz > 0


def test_core_clock_and_constant_rate_counter():
    n = 100_000_000
    out = tuple(torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3))
    buf = torch.empty(kp.clock_probe_stamps(n), dtype=torch.int64, device="cuda")
    for _ in range(20):  # bring the clock up from idle
        kp.sample(3.0, 1.0, n, 1, precision=kp.FP32, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, stamps, hz = kp.clock_probe(3.0, 1.0, n, 1, precision=kp.FP32, out=out, stamps=buf)
    e1.record()
    torch.cuda.synchronize()
    ghz = kp.core_clock_hz(stamps, hz) / 1e9
    print(f"core clock during the C2 kappa-3 launch: {ghz:.3f} GHz (constant-rate counter {hz / 1e6:.1f} MHz)")
    assert 0.3 < ghz < 2.45
    s = stamps.cpu().numpy()
    span_ms = float(s[:, 3].max() - s[:, 1].min()) / hz * 1e3
    event_ms = e0.elapsed_time(e1)
    # the stamps sit inside the launch: the span is the launch minus its ramp
    assert 0.8 * event_ms < span_ms <= event_ms * 1.02 + 0.01


def test_too_few_stamps():
    n = 1 << 20
    out = tuple(torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3))
    stamps = torch.empty(8, dtype=torch.int64, device="cuda")
    blocks, hz = ctypes.c_uint32(0), ctypes.c_double(0.0)
    st = _lib.load().kappa_clock_probe(3.0, 1.0, n, 0, 0, 0, kp.FP32, out[0].data_ptr(), out[1].data_ptr(),
                                       out[2].data_ptr(), stamps.data_ptr(), stamps.numel(), ctypes.byref(blocks),
                                       ctypes.byref(hz), None)
    assert st == _lib.ERANGE and blocks.value == n // 1024
    with pytest.raises(kp.KappaError):
        kp.clock_probe(3.0, 1.0, n, 0, out=tuple(torch.empty(n + 1, device="cuda")[1:] for _ in range(3)))
    with pytest.raises(ValueError):
        kp.clock_probe(3.0, 1.0, n, 0, out=out, stamps=torch.empty(4096, dtype=torch.int32, device="cuda"))
