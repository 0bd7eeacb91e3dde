"""GPU parity of the batched persistent launch (C4 workload).

Each segment of a batched launch must equal a single-species call with the
same seed and seg_id plus its drift, bit for bit; hipGraph replays must equal
a direct launch; every launch shape (including the autotuner's pick) must
give the same bits; and sampled particles must match the oracle.
"""
import numpy as np
import pytest
import torch

import paper_2602_05606_amd as kp
import workloads
from gpu_helpers import TOL_FP32, TOL_FP64, bits_equal, norm_rel_err, to_host

pytestmark = pytest.mark.gpu


def segment_bounds(segs):
    counts = np.array([s["count"] for s in segs], dtype=np.int64)
    start = np.concatenate([[0], np.cumsum(counts)])
    return start


@pytest.fixture(scope="module")
def c4():
    segs = workloads.batched_segments()
    return segs, segment_bounds(segs)


def test_c4_segments_equal_single_species_calls(c4):
    segs, start = c4
    seed = workloads.C4["seed"]
    with kp.Plan(segs, seed, kp.FP32) as plan:
        out = plan.outputs()
        plan.launch(out)
        torch.cuda.synchronize()
        assert plan.total == start[-1]
        host = to_host(*out)
    bad = []
    for s, seg in enumerate(segs):
        n = seg["count"]
        v = kp.sample(seg["kappa"], seg["theta"], n, seed, seg_id=seg["seg_id"], precision=kp.FP32)
        ref = tuple((t + torch.tensor(d, dtype=torch.float32, device="cuda")).cpu().numpy().astype(np.float64)
                    for t, d in zip(v, seg["drift"]))
        got = tuple(h[start[s]:start[s + 1]] for h in host)
        if not bits_equal(got, ref):
            bad.append(s)
    assert not bad, f"{len(bad)} segments differ, first {bad[:5]}"


def test_c4_against_oracle(orc, c4):
    """Every particle of every C4 segment against the oracle (FP32 mode)."""
    segs, start = c4
    seed = workloads.C4["seed"]
    out = kp.sample_batched(segs, seed, kp.FP32)
    host = to_host(*out)
    worst = 0.0
    for s, seg in enumerate(segs):
        n = seg["count"]
        r = orc.sample(seg["kappa"], seg["theta"], n, seed, seg=seg["seg_id"], mode=1, drift=seg["drift"])[:3]
        g = tuple(h[start[s]:start[s + 1]] for h in host)
        # drift can make a velocity small: compare against the drift-free norm scale
        d = np.sqrt(sum((a - b) ** 2 for a, b in zip(g, r)))
        scale = np.sqrt(sum((b - dr) ** 2 for b, dr in zip(r, seg["drift"]))) + np.linalg.norm(seg["drift"])
        worst = max(worst, float(np.max(d / scale)))
    print(f"C4 all {int(start[-1])} particles of {len(segs)} segments: max error {worst:.3e}")
    assert worst <= TOL_FP32


def test_c4_fp64_against_oracle(orc, c4):
    """The C4 table in FP64: every particle of every segment against the oracle."""
    segs, start = c4
    seed = workloads.C4["seed"]
    host = to_host(*kp.sample_batched(segs, seed, kp.FP64))
    worst = 0.0
    for s, seg in enumerate(segs):
        n = seg["count"]
        r = orc.sample(seg["kappa"], seg["theta"], n, seed, seg=seg["seg_id"], mode=0, drift=seg["drift"])[:3]
        g = tuple(h[start[s]:start[s + 1]] for h in host)
        d = np.sqrt(sum((a - b) ** 2 for a, b in zip(g, r)))
        scale = np.sqrt(sum((b - dr) ** 2 for b, dr in zip(r, seg["drift"]))) + np.linalg.norm(seg["drift"])
        worst = max(worst, float(np.max(d / scale)))
    print(f"C4 FP64 all {int(start[-1])} particles of {len(segs)} segments: max error {worst:.3e}")
    assert worst <= TOL_FP64


def test_graph_replay_matches_direct_launch(c4):
    segs, _ = c4
    with kp.Plan(segs, 4, kp.FP32) as plan:
        ref = plan.outputs()
        plan.launch(ref)
        torch.cuda.synchronize()
        ref_h = to_host(*ref)
        out = plan.outputs()
        for rep in range(4):
            for t in out:
                t.fill_(float("nan"))  # eager work between replays
            plan.graph_launch(out)
            torch.cuda.synchronize()
            assert bits_equal(to_host(*out), ref_h), f"replay {rep}"
        # new output buffers force a re-capture
        out2 = plan.outputs()
        plan.graph_launch(out2)
        torch.cuda.synchronize()
        assert bits_equal(to_host(*out2), ref_h)


def test_every_shape_gives_the_same_bits(c4):
    segs, _ = c4
    segs = segs[:600]
    with kp.Plan(segs, 4, kp.FP32) as plan:
        ref = plan.outputs()
        plan.launch(ref)
        torch.cuda.synchronize()
        ref_h = to_host(*ref)
        for block in (64, 128, 256):
            for unroll in (1, 2, 4, 8):
                for grid in (1, 7, 256, 2048):
                    plan.set_shape(block, unroll, grid)
                    out = plan.outputs()
                    plan.launch(out)
                    torch.cuda.synchronize()
                    assert bits_equal(to_host(*out), ref_h), (block, unroll, grid)
        shape = plan.autotune(ref, reps=2)
        out = plan.outputs()
        plan.launch(out)
        torch.cuda.synchronize()
        assert bits_equal(to_host(*out), ref_h), shape


def test_autotune_cache_round_trip(tmp_path, monkeypatch, c4):
    segs, _ = c4
    cache = tmp_path / "autotune.json"
    monkeypatch.setenv("KAPPA_AUTOTUNE_CACHE", str(cache))
    with kp.Plan(segs[:3000], 4, kp.FP32) as plan:
        out = plan.outputs()
        shape = plan.autotune(out, reps=1)
    assert cache.exists() and "batched|mode1" in cache.read_text()
    with kp.Plan(segs[:3000], 4, kp.FP32) as plan2:
        assert plan2.shape == shape


def test_uneven_and_empty_segments_fp64(orc):
    segs = [dict(kappa=3.0, theta=1.0, drift=(0.1, -0.2, 0.3), count=1, seg_id=0),
            dict(kappa=1.6, theta=2.0, drift=(0, 0, 0), count=0, seg_id=1),
            dict(kappa=9.0, theta=0.5, drift=(0, 0, 1), count=8192, seg_id=2),
            dict(kappa=2.0, theta=1.0, drift=(0, 0, 0), count=0, seg_id=3),
            dict(kappa=2.0, theta=1.0, drift=(-1, 0, 0), count=3, seg_id=7),
            dict(kappa=4.1, theta=1.5, drift=(0, 0, 0), count=2047, seg_id=9)]
    start = segment_bounds(segs)
    for precision, mode, tol in ((kp.FP64, 0, TOL_FP64), (kp.FP32, 1, TOL_FP32)):
        host = to_host(*kp.sample_batched(segs, 21, precision))
        for s, seg in enumerate(segs):
            n = seg["count"]
            if n == 0:
                continue
            r = orc.sample(seg["kappa"], seg["theta"], n, 21, seg=seg["seg_id"], mode=mode, drift=seg["drift"])[:3]
            g = tuple(h[start[s]:start[s + 1]] for h in host)
            rd = tuple(a - d for a, d in zip(r, seg["drift"]))
            gd = tuple(a - d for a, d in zip(g, seg["drift"]))
            assert norm_rel_err(gd, rd) <= tol * 4 + 1e-7 * (precision != kp.FP64), (precision, s)


def test_single_segment_plan_equals_sample(c4):
    seg = dict(kappa=2.5, theta=1.0, drift=(0, 0, 0), count=1_000_003, seg_id=0)
    a = to_host(*kp.sample_batched([seg], 9, kp.FP32))
    b = to_host(*kp.sample(2.5, 1.0, 1_000_003, 9, precision=kp.FP32))
    assert bits_equal(a, b)


def test_maximum_segment_count():
    """KAPPA_MAX_SEGMENTS = 2^24 segments of one particle each, with six kappa
    values and random theta, from a numpy segment table: sampled segments
    (both ends and 300 random ones) equal single-species calls bit for bit."""
    n = 1 << 24
    rng = np.random.default_rng(24)
    kappas = np.array([1.6, 2.0, 3.0, 4.1, 7.5, 10.0])
    table = kp.segment_table(kappas[rng.integers(0, kappas.size, n)], rng.uniform(0.5, 2.0, n), 1)
    print("segment table built", flush=True)
    with kp.Plan(table, 6, kp.FP32) as plan:
        assert plan.total == n
        out = plan.outputs()
        plan.launch(out)
        torch.cuda.synchronize()
        host = to_host(*out)
    for s in np.concatenate([[0, 1, n - 2, n - 1], rng.integers(0, n, 300)]):
        s = int(s)
        v = kp.sample(table["kappa"][s], table["theta"][s], 1, 6, seg_id=s, precision=kp.FP32)
        assert bits_equal(tuple(h[s:s + 1] for h in host), to_host(*v)), s


def test_segment_longer_than_2_to_32_particles(orc):
    """A segment of 2^32 + 777 particles between two short ones: the plan splits
    it into pieces at the counter's 2^32 boundary.  Around that boundary (and at
    the segment's ends) the plan's output must equal a single-species call over
    the same counters bit for bit, and the oracle at sampled particles.  The
    FP32 outputs take 3 x 17.2 GB."""
    big = (1 << 32) + 777
    segs = [dict(kappa=2.5, theta=1.1, drift=(0.0, 0.0, 0.0), count=1000, seg_id=7),
            dict(kappa=3.5, theta=0.9, drift=(0.0, 0.0, 0.0), count=big, seg_id=8),
            dict(kappa=6.0, theta=1.3, drift=(0.0, 0.0, 0.0), count=5, seg_id=9)]
    seed = 21
    with kp.Plan(segs, seed, kp.FP32) as plan:
        assert plan.total == 1000 + big + 5
        out = plan.outputs()
        plan.launch(out)
        torch.cuda.synchronize()
        first = 1000  # output position of the big segment's particle 0
        for lo in (0, (1 << 32) - 40, big - 40):
            n = 80 if lo + 80 <= big else big - lo
            ref = kp.sample(3.5, 0.9, n, seed, counter_offset=lo, seg_id=8, precision=kp.FP32)
            got = tuple(t[first + lo:first + lo + n] for t in out)
            assert bits_equal(to_host(*got), to_host(*ref)), lo
        idx = np.array([0, 1, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, big - 1], dtype=np.uint64)
        r = orc.sample_indices(3.5, 0.9, idx, seed, seg=8, mode=1)
        it = torch.from_numpy(idx.astype(np.int64) + first).cuda()
        g = to_host(*(t[it] for t in out))
        assert norm_rel_err(g, r) <= TOL_FP32
        # the neighbours are intact
        for s, pos in ((segs[0], 0), (segs[2], first + big)):
            ref = kp.sample(s["kappa"], s["theta"], s["count"], seed, seg_id=s["seg_id"], precision=kp.FP32)
            got = tuple(t[pos:pos + s["count"]] for t in out)
            assert bits_equal(to_host(*got), to_host(*ref))
        del out
    torch.cuda.empty_cache()
