"""GPU fused particle loading (positions with velocities) on the C4 workload.

* velocities of the fused launch are bit-identical to the velocity-only
  launch (positions use draw 1 of the counter, velocities draw 0);
* positions match the oracle (oracle.positions) per segment: FP64 to a few
  ulps of |lo| + |size| (one fused multiply-add against the oracle's two
  roundings), FP32 to 2^-22 (|lo| + |size|) (float lo and size, one fmaf);
* positions lie in their cell's half-open box, also for the largest Philox
  words, whose fused multiply-add rounds up to the box's upper edge;
* graph replays, the one-shot entry point, ragged and misaligned outputs give
  the same bits; a launch without cells is refused.
"""
import numpy as np
import pytest
import torch

import paper_2602_05606_amd as kp
import workloads
from gpu_helpers import to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c4():
    segs = workloads.batched_segments()
    cells = workloads.batched_cells()
    counts = np.array([s["count"] for s in segs], dtype=np.int64)
    start = np.concatenate([[0], np.cumsum(counts)])
    return segs, cells, start


def _dtype(prec):
    return torch.float64 if prec == kp.FP64 else torch.float32


@pytest.mark.parametrize("prec", [kp.FP32, kp.FP64, kp.FP32_NOTAIL])
def test_positions_against_oracle_and_velocities_unchanged(orc, c4, prec):
    segs, cells, start = c4
    seed = workloads.C4["seed"]
    with kp.Plan(segs, seed, prec) as plan:
        vel_only = plan.outputs()
        plan.launch(vel_only)
        plan.set_cells(cells)
        pos, vel = plan.outputs(), plan.outputs()
        plan.launch_pic(pos, vel)
        torch.cuda.synchronize()
        for a, b in zip(vel, vel_only):
            assert torch.equal(a, b)
        host = to_host(*pos)
    rng = np.random.default_rng(3)
    mode = 0 if prec == kp.FP64 else 1
    worst = 0.0
    for s in list(rng.choice(len(segs), size=300, replace=False)) + [0, len(segs) - 1]:
        seg = segs[s]
        n = seg["count"]
        lo, size = cells[s]
        ref = orc.positions(lo, size, n, seed, seg=seg["seg_id"], mode=mode)
        scale = np.abs(lo) + np.abs(size)
        tol = (4 * 2.0 ** -53 if prec == kp.FP64 else 2.0 ** -22) * scale
        for k in range(3):
            got = host[k][start[s]:start[s + 1]]
            err = np.abs(got - ref[k])
            worst = max(worst, float(np.max(err / scale[k])) if n else 0.0)
            assert np.all(err <= tol[k]), (s, k)
            if prec == kp.FP64:
                assert np.all(got >= lo[k]) and np.all(got < lo[k] + size[k])
            else:
                # the FP32 box: lo and size rounded to float, half-open
                lo32, size32 = np.float64(np.float32(lo[k])), np.float64(np.float32(size[k]))
                assert np.all(got >= lo32) and np.all(got < lo32 + size32)
    print(f"prec {prec}: worst position error {worst:.2e} of |lo| + |size|")


def test_graph_and_one_shot_equal_direct(c4):
    segs, cells, _ = c4
    seed = 77
    with kp.Plan(segs, seed, kp.FP32) as plan:
        plan.set_cells(cells)
        pos, vel = plan.outputs(), plan.outputs()
        plan.launch_pic(pos, vel)
        torch.cuda.synchronize()
        ref = [t.clone() for t in pos + vel]
        gpos, gvel = plan.outputs(), plan.outputs()
        for rep in range(3):
            for t in gpos + gvel:
                t.fill_(float("nan"))
            plan.graph_launch_pic(gpos, gvel)
            torch.cuda.synchronize()
            for a, b in zip(gpos + gvel, ref):
                assert torch.equal(a, b), rep
            _ = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
        # the velocity-only graph of the same plan is a different capture and still right
        vo = plan.outputs()
        plan.graph_launch(vo)
        torch.cuda.synchronize()
        for a, b in zip(vo, ref[3:]):
            assert torch.equal(a, b)
    p1, v1 = kp.load_particles(segs, cells, seed, kp.FP32)
    torch.cuda.synchronize()
    for a, b in zip(p1 + v1, ref):
        assert torch.equal(a, b)


def test_ragged_and_misaligned_outputs():
    segs = [dict(kappa=2.5, theta=1.0, drift=(0, 0, 0), count=c, seg_id=i)
            for i, c in enumerate([1, 7, 0, 130, 3, 64, 5])]
    cells = np.array([[[i, -i, 0.5 * i], [1.0, 2.0, 0.25]] for i in range(len(segs))], dtype=np.float64)
    for prec in (kp.FP32, kp.FP64):
        with kp.Plan(segs, 5, prec) as plan:
            plan.set_cells(cells)
            total = plan.total
            pos, vel = plan.outputs(), plan.outputs()
            plan.launch_pic(pos, vel)
            big = [torch.empty(total + 1, dtype=_dtype(prec), device="cuda") for _ in range(6)]
            views = [b[1:] for b in big]  # 4- or 8-byte offset: not 16-byte aligned
            plan.launch_pic(views[:3], views[3:])
            torch.cuda.synchronize()
            for a, b in zip(pos + vel, views):
                assert torch.equal(a, b)
        # a cell of zero size pins its particles to lo (segment 3: 130 particles from offset 8)
        flat = cells.copy()
        flat[3, 1] = 0.0
        with kp.Plan(segs, 5, prec) as plan:
            plan.set_cells(flat)
            pos, vel = plan.outputs(), plan.outputs()
            plan.launch_pic(pos, vel)
            torch.cuda.synchronize()
            for k in range(3):
                assert torch.all(pos[k][8:138] == float(np.asarray(flat[3, 0, k], dtype=np.float32 if prec != kp.FP64
                                                                     else np.float64)))


def test_refused_without_cells(c4):
    segs, cells, _ = c4
    with kp.Plan(segs[:10], 1, kp.FP32) as plan:
        pos, vel = plan.outputs(), plan.outputs()
        with pytest.raises(kp.KappaError):
            plan.launch_pic(pos, vel)
        plan.set_cells(cells[:10])
        plan.launch_pic(pos, vel)
        plan.set_cells(None)
        with pytest.raises(kp.KappaError):
            plan.launch_pic(pos, vel)
        with pytest.raises(ValueError):
            plan.set_cells(cells[:9])
        bad = cells[:10].copy()
        bad[3, 1, 0] = -1.0
        with pytest.raises(kp.KappaError):
            plan.set_cells(bad)


def test_largest_words_stay_below_the_upper_edge(orc):
    """In FP32 with lo = 3.5 and size = 0.5 the top 2^10 words (u within
    2^-22 of 1) give fmaf(u, 0.5, 3.5) = 4.0, the next cell's lower corner;
    the kernel caps them at the largest float below 4.  2^24 particles hold
    some such words on every axis; all positions are checked against the
    oracle (which caps in FP64) and against the box."""
    n, seed, seg = 1 << 24, 21, 5
    lo, size = np.array([3.5, 3.5, -4.0]), np.array([0.5, 0.5, 0.5])
    segs = [dict(kappa=3.0, theta=1.0, drift=(0, 0, 0), count=n, seg_id=seg)]
    with kp.Plan(segs, seed, kp.FP32) as plan:
        plan.set_cells(np.array([[lo, size]]))
        pos, vel = plan.outputs(), plan.outputs()
        plan.launch_pic(pos, vel)
        words = kp.philox(n, seed, seg_id=seg, draw=1)
        torch.cuda.synchronize()
        host = to_host(*pos)
        words = words.cpu().numpy().view(np.uint32).reshape(n, 4)
    del pos, vel
    ref = orc.positions(lo, size, n, seed, seg=seg, mode=1)
    capped = 0
    for k in range(3):
        got = host[k]
        assert np.all(got >= lo[k]) and np.all(got < lo[k] + size[k])
        assert np.all(np.abs(got - ref[k]) <= 2.0 ** -22 * (abs(lo[k]) + size[k]))
        top = np.nonzero(words[:, k] >= 0xFFFFFC00)[0]
        assert top.size > 0, k
        edge = np.float32(lo[k] + size[k])
        assert np.all(got[top] == np.float64(np.nextafter(edge, np.float32(-np.inf)))), k
        capped += top.size
    print(f"{capped} coordinates at the cap")
