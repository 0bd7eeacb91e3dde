"""The library's launches inside a caller's hipGraph (torch.cuda.CUDAGraph).

A PIC code captures a whole time step, so the sampler's launches must be
capture-safe: no allocation, synchronisation or memset node on the path of
kappa_sample, kappa_plan_launch (velocities and fused positions) or
kappa_sample_backward.  One graph holds all of them next to a torch
elementwise op; it is replayed several times with eager work (NaN fills)
between replays, and every replay must equal the eager launches bit for bit.
"""
import numpy as np
import pytest
import torch

import paper_2602_05606_amd as kp
import workloads
from gpu_helpers import bits_equal, to_host

pytestmark = pytest.mark.gpu

N = (1 << 18) + 37  # ragged: several launches' worth of tiles and a partial vector tail


def _capture(work):
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        work()  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        result = work()
    return g, result


def test_sampler_plan_and_backward_in_a_caller_graph():
    segs = workloads.batched_segments()[:900]
    cells = workloads.batched_cells()[:900]
    dev = torch.device("cuda")
    with kp.Plan(segs, 4, kp.FP32) as plan:
        plan.set_cells(cells)
        # eager references
        ref_f32 = kp.sample(3.0, 1.0, N, 7, counter_offset=5, seg_id=2, precision=kp.FP32)
        ref_f64 = kp.sample(6.0, 0.5, N, 8, precision=kp.FP64)
        ref_vel = plan.outputs()
        plan.launch(ref_vel)
        ref_pos, ref_pv = plan.outputs(), plan.outputs()
        plan.launch_pic(ref_pos, ref_pv)
        gen = torch.Generator(device=dev).manual_seed(3)
        grad_in = torch.randn((3, N), generator=gen, device=dev, dtype=torch.float32)
        ref_grad = kp.sample_backward(2.5, 1.3, N, 2, grad_in[0], grad_in[1], grad_in[2], precision=kp.FP32)
        ref_shift = torch.add(ref_f32[0], 1.5)
        torch.cuda.synchronize()
        want = [to_host(*ref_f32), to_host(*ref_f64), to_host(*ref_vel), to_host(*ref_pos), to_host(*ref_pv)]
        want_grad = ref_grad.cpu().numpy()
        want_shift = to_host(ref_shift)[0]

        # static buffers of the captured step
        f32 = tuple(torch.empty(N, dtype=torch.float32, device=dev) for _ in range(3))
        f64 = tuple(torch.empty(N, dtype=torch.float64, device=dev) for _ in range(3))
        vel, pos, pv = plan.outputs(), plan.outputs(), plan.outputs()
        shifted = torch.empty(N, dtype=torch.float32, device=dev)
        ws = torch.empty(kp.backward_workspace_bytes(N), dtype=torch.uint8, device=dev)

        def step():
            kp.sample(3.0, 1.0, N, 7, counter_offset=5, seg_id=2, precision=kp.FP32, out=f32)
            torch.add(f32[0], 1.5, out=shifted)  # caller work between library launches
            kp.sample(6.0, 0.5, N, 8, precision=kp.FP64, out=f64)
            plan.launch(vel)
            plan.launch_pic(pos, pv)
            return kp.sample_backward(2.5, 1.3, N, 2, grad_in[0], grad_in[1], grad_in[2], precision=kp.FP32,
                                      workspace=ws)

        g, grad = _capture(step)
        for rep in range(3):
            for t in (*f32, *f64, *vel, *pos, *pv, shifted, grad):
                t.fill_(float("nan"))  # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = [to_host(*f32), to_host(*f64), to_host(*vel), to_host(*pos), to_host(*pv)]
            for name, a, b in zip(("fp32", "fp64", "plan", "positions", "pic velocities"), got, want):
                assert bits_equal(a, b), f"replay {rep}: {name}"
            assert np.array_equal(to_host(shifted)[0], want_shift), f"replay {rep}: caller op"
            assert np.array_equal(grad.cpu().numpy(), want_grad), f"replay {rep}: backward"
        del g
