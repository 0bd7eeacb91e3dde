"""Several host threads and streams at once (the threads rule of kappa.h):
stateless entry points called from four Python threads (ctypes releases the
GIL during each call), each on a stream of its own, give the bits of the same
calls made one after another; one plan's launches in flight on two streams
into different outputs give the bits of a single launch.
"""
import threading

import numpy as np
import pytest
import torch

import paper_2602_05606_amd as kp
import workloads
from gpu_helpers import bits_equal, to_host

pytestmark = pytest.mark.gpu

N = (1 << 20) + 11
JOBS = [(3.0, 1.0, 11, kp.FP32), (1.6, 0.5, 12, kp.FP64), (7.5, 2.0, 13, kp.FP32), (float("inf"), 1.0, 14, kp.FP32)]


def test_threads_on_their_own_streams_give_the_same_bits():
    dev = torch.device("cuda")
    refs = [to_host(*kp.sample(k, t, N, s, precision=p)) for k, t, s, p in JOBS]
    g = workloads.upstream_gradient(N, seed=5)
    gdev = [torch.from_numpy(a).to(dev) for a in g]
    ref_grad = kp.sample_backward(2.5, 1.3, N, 2, *gdev, precision=kp.FP32).cpu().numpy()
    outs = [tuple(torch.empty(N, dtype=torch.float64 if p == kp.FP64 else torch.float32, device=dev)
                  for _ in range(3)) for _, _, _, p in JOBS]
    grads = [None] * len(JOBS)
    streams = [torch.cuda.Stream() for _ in JOBS]
    torch.cuda.synchronize()
    errors = []

    def work(i):
        try:
            k, t, s, p = JOBS[i]
            ws = None
            for _ in range(5):
                kp.sample(k, t, N, s, precision=p, out=outs[i], stream=streams[i])
                with torch.cuda.stream(streams[i]):
                    if ws is None:
                        ws = torch.empty(kp.backward_workspace_bytes(N), dtype=torch.uint8, device=dev)
                    grads[i] = kp.sample_backward(2.5, 1.3, N, 2, *gdev, precision=kp.FP32, workspace=ws,
                                                  stream=streams[i])
            streams[i].synchronize()
        except Exception as e:  # reported below, in the main thread
            errors.append((i, repr(e)))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(JOBS))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i in range(len(JOBS)):
        assert bits_equal(to_host(*outs[i]), refs[i]), f"job {i}"
        assert np.array_equal(grads[i].cpu().numpy(), ref_grad), f"backward in job {i}"


def test_one_plan_in_flight_on_two_streams():
    segs = workloads.batched_segments()[:3000]
    with kp.Plan(segs, 4, kp.FP32) as plan:
        ref = plan.outputs()
        plan.launch(ref)
        torch.cuda.synchronize()
        want = to_host(*ref)
        a, b = plan.outputs(), plan.outputs()
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        torch.cuda.synchronize()
        for _ in range(4):
            plan.launch(a, stream=sa)
            plan.launch(b, stream=sb)
        torch.cuda.synchronize()
        assert bits_equal(to_host(*a), want) and bits_equal(to_host(*b), want)
