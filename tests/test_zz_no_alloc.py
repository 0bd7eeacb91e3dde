"""kappa_sample_backward_noalloc against kappa_sample_backward, through the C
ABI: the allocation-free entry point runs the same kernels with the library's
static partial-sum array in place of the caller's workspace, so its gradient
must equal the workspace entry point's bit for bit.  Two calls in a row, the
second on fewer particles (fewer partial blocks), show that nothing left in
the shared array from the first call leaks into the second; a third call at
the first size shows the reverse.  Each result is also checked against the
FP64 oracle adjoint at the tolerance of the backward parity tests.
"""
import ctypes

import numpy as np
import pytest

from paper_2602_05606_amd import _lib

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("precision", [_lib.FP32, _lib.FP64])
def test_noalloc_backward_equals_workspace_backward(orc, precision):
    import torch
    import workloads

    dev = torch.device("cuda", 0)
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    kappa, theta, seed = 2.5, 1.3, 2
    dt = torch.float64 if precision == _lib.FP64 else torch.float32
    # 2^21 + 5 particles fill 2049 partial blocks of the default grid; 300_007 fill 293
    for n in (2_097_157, 300_007, 2_097_157):
        print(f"noalloc backward precision {precision} n {n}", flush=True)
        gv = workloads.upstream_gradient(n, seed=7)
        g = [torch.from_numpy(gv[i].astype(np.float64 if precision == _lib.FP64 else np.float32)).to(dev)
             for i in range(3)]
        ws = torch.empty(lib.kappa_backward_workspace_bytes(n), dtype=torch.uint8, device=dev)
        ref = torch.full((2,), float("nan"), dtype=torch.float64, device=dev)
        got = torch.full((2,), float("nan"), dtype=torch.float64, device=dev)
        assert lib.kappa_sample_backward(kappa, theta, n, seed, 0, 0, precision, _ptr(g[0]), _ptr(g[1]), _ptr(g[2]),
                                         _ptr(ref), _ptr(ws), ws.numel(), stream) == _lib.OK
        assert lib.kappa_sample_backward_noalloc(kappa, theta, n, seed, 0, 0, precision, _ptr(g[0]), _ptr(g[1]),
                                                 _ptr(g[2]), _ptr(got), stream) == _lib.OK
        torch.cuda.synchronize()
        r, o = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(r.view(np.uint64), o.view(np.uint64)), (r, o)
        mode = orc.MODE_FP64 if precision == _lib.FP64 else orc.MODE_FP32
        adj = orc.backward(kappa, theta, n, seed, *[t.cpu().numpy() for t in g], mode=mode)
        # the backward parity tests' bound: sums of n terms of either sign
        tol = 1e-10 if precision == _lib.FP64 else 1e-4
        for a, b in zip(o, adj):
            assert abs(a - b) <= tol * (abs(b) + np.sqrt(n) * 1e-3), (n, precision, o, adj)


def test_noalloc_backward_zero_particles():
    import torch

    dev = torch.device("cuda", 0)
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    got = torch.full((2,), float("nan"), dtype=torch.float64, device=dev)
    assert lib.kappa_sample_backward_noalloc(3.0, 1.0, 0, 0, 0, 0, _lib.FP32, None, None, None, _ptr(got),
                                             stream) == _lib.OK
    torch.cuda.synchronize()
    assert got.cpu().tolist() == [0.0, 0.0]
