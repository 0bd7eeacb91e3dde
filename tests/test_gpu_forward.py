"""GPU parity of the forward generator (Table 1) against the FP64 oracle.

Every call goes through the C ABI of libkappa.  Bars:
  * Philox words: bit-exact;
  * velocities: per-particle norm-relative error <= 1e-13 (FP64) and 4e-6
    (FP32, against the oracle evaluated at the FP32 mode's uniforms);
  * determinism, chunking and store-path invariance: bit-exact.
"""
import numpy as np
import pytest
import torch

import paper_2602_05606_amd as kp
import workloads
from gpu_helpers import TOL_FP32, TOL_FP64, bits_equal, norm_rel_err, to_host

pytestmark = pytest.mark.gpu

MODE = {kp.FP64: 0, kp.FP32: 1, kp.FP32_NOTAIL: 2}


def gpu_sample(kappa, theta, n, seed, precision, counter_offset=0, seg_id=0):
    v = kp.sample(kappa, theta, n, seed, counter_offset=counter_offset, seg_id=seg_id, precision=precision)
    torch.cuda.synchronize()
    return v


@pytest.mark.parametrize("seed,offset,seg,draw,n", [
    (0, 0, 0, 0, 100_003),
    (1, (1 << 32) - 1000, 0, 0, 5000),
    (0x0123456789ABCDEF, 1 << 40, 12287, 3, 777),
    ((1 << 64) - 1, 17, (1 << 32) - 1, (1 << 32) - 1, 64),
])
def test_philox_bit_exact(orc, seed, offset, seg, draw, n):
    got = kp.philox(n, seed, counter_offset=offset, seg_id=seg, draw=draw).cpu().numpy().view(np.uint32)
    ref = orc.philox_blocks(n, seed, counter_offset=offset, seg=seg, draw=draw)
    np.testing.assert_array_equal(got, ref)


def test_c1_plain_fp64_full(orc):
    """C1 at its full size: 1e6 particles, kappa 3, theta 1, FP64, seed 0."""
    c = workloads.C1
    g = to_host(*gpu_sample(c["kappa"], c["theta"], c["n"], c["seed"], kp.FP64))
    r = orc.sample(c["kappa"], c["theta"], c["n"], c["seed"], mode=0)[:3]
    err = norm_rel_err(g, r)
    print(f"C1 FP64 max norm-relative error {err:.3e}")
    assert err <= TOL_FP64


@pytest.mark.parametrize("kappa", [1.6, 2.5, 4.1, 10.0, 25.0])
@pytest.mark.parametrize("precision", [kp.FP64, kp.FP32, kp.FP32_NOTAIL])
def test_forward_parity_ragged(orc, kappa, precision):
    n = 1_000_003  # several tiles and a ragged tail
    g = to_host(*gpu_sample(kappa, 1.7, n, 11, precision, counter_offset=123))
    r = orc.sample(kappa, 1.7, n, 11, counter_offset=123, mode=MODE[precision])[:3]
    err = norm_rel_err(g, r)
    print(f"kappa {kappa} precision {precision}: max norm-relative error {err:.3e}")
    # FP32_NOTAIL (diagnostics) keeps FP32 arithmetic where 1 - U1 < 2^-20, where
    # the error of z = -ln(1 - U1^{2/3})/kappa* is amplified by z (up to ~30)
    tol = {kp.FP64: TOL_FP64, kp.FP32: TOL_FP32, kp.FP32_NOTAIL: 1e-5}[precision]
    assert err <= tol


@pytest.mark.parametrize("kappa,theta", [(1.5 + 1e-9, 1e-3), (1.5 + 1e-6, 1.0), (1e4, 1e3), (1e8, 0.5),
                                         (1e12, 1.0), (3.0, 1e-30), (3.0, 1e30)])
@pytest.mark.parametrize("precision", [kp.FP64, kp.FP32])
def test_degenerate_kappa_and_theta(orc, kappa, theta, precision):
    """kappa just above 3/2 (kappa* -> 1, the heaviest tail eq:kappa allows),
    very large kappa (kappa* huge: z = -lT/kappa* tiny), and theta far from 1."""
    n = 200_003
    g = to_host(*gpu_sample(kappa, theta, n, 29, precision))
    r = orc.sample(kappa, theta, n, 29, mode=MODE[precision])[:3]
    err = norm_rel_err(g, r)
    print(f"kappa {kappa} theta {theta} precision {precision}: max error {err:.3e}")
    assert err <= (TOL_FP64 if precision == kp.FP64 else TOL_FP32)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 63, 64, 65, 1023, 4097])
def test_small_and_ragged_sizes(orc, n):
    for precision in (kp.FP64, kp.FP32):
        g = to_host(*gpu_sample(3.0, 1.0, n, 5, precision, counter_offset=9))
        r = orc.sample(3.0, 1.0, n, 5, counter_offset=9, mode=MODE[precision])[:3]
        assert norm_rel_err(g, r) <= (TOL_FP64 if precision == kp.FP64 else TOL_FP32)


def test_fp32_tail_particles(orc):
    """Particles whose 1 - U1 < 2^-20 take the FP64 inversion in FP32 mode."""
    n, seed = 1 << 24, 12
    tails = orc.find_tails(n, seed)
    assert len(tails) >= 5
    rng = np.random.default_rng(0)
    idx = np.concatenate([tails, rng.integers(0, n, size=20000).astype(np.uint64)])
    for kappa in (1.6, 3.0, 10.0):
        v = gpu_sample(kappa, 1.0, n, seed, kp.FP32)
        it = torch.from_numpy(idx.astype(np.int64)).cuda()
        g = to_host(*(t[it] for t in v))
        r = orc.sample_indices(kappa, 1.0, idx, seed, mode=1)
        err_tail = norm_rel_err(tuple(a[:len(tails)] for a in g), tuple(a[:len(tails)] for a in r))
        err_all = norm_rel_err(g, r)
        print(f"kappa {kappa}: tail particles {len(tails)}, max error tail {err_tail:.3e}, sample {err_all:.3e}")
        assert err_tail <= TOL_FP32 and err_all <= TOL_FP32
        # the tail speeds are the largest of the run
        speed = torch.sqrt(v[0].double() ** 2 + v[1].double() ** 2 + v[2].double() ** 2)
        assert float(speed[torch.from_numpy(tails.astype(np.int64)).cuda()].min()) > float(torch.quantile(speed[:1 << 20], 0.999))


@pytest.mark.parametrize("kappa", workloads.C2["kappas"])
@pytest.mark.parametrize("precision", [kp.FP32, kp.FP64])
def test_c2_full_size_every_particle(orc, kappa, precision):
    """C2 at full size (1e8 particles, seed 1) in the benchmark's launch
    configuration: every particle against the oracle, in chunks of 1e7
    (the oracle evaluates each chunk at its counter offset).  The FP32 mode's
    tail particles are among them."""
    c = workloads.C2
    n, chunk = c["n"], 10 ** 7
    v = gpu_sample(kappa, c["theta"], n, c["seed"], precision)
    assert all(bool(torch.isfinite(t).all()) for t in v)
    worst = 0.0
    for off in range(0, n, chunk):
        m = min(chunk, n - off)
        g = to_host(*(t[off:off + m] for t in v))
        r = orc.sample(kappa, c["theta"], m, c["seed"], counter_offset=off, mode=MODE[precision])[:3]
        worst = max(worst, norm_rel_err(g, r))
    tails = len(orc.find_tails(n, c["seed"])) if precision == kp.FP32 else 0
    print(f"C2 kappa {kappa} precision {precision}: all {n} particles ({tails} FP64-tail), max error {worst:.3e}")
    assert worst <= (TOL_FP64 if precision == kp.FP64 else TOL_FP32)


def test_beyond_2_to_31_particles_in_one_call(orc):
    """One FP32 call of 2^31 + 1029 particles (25.8 GB of outputs): indices past
    2^31 and the last group (ragged) must match the oracle, and the launch must
    cover every particle (no 32-bit index wrap)."""
    n = (1 << 31) + 1029
    vx, vy, vz = (torch.full((n,), float("nan"), dtype=torch.float32, device="cuda") for _ in range(3))
    kp.sample(2.5, 1.1, n, 13, precision=kp.FP32, out=(vx, vy, vz))
    torch.cuda.synchronize()
    try:
        assert bool(torch.isfinite(vx).all()) and bool(torch.isfinite(vz).all())
        rng = np.random.default_rng(31)
        idx = np.concatenate([rng.integers(0, n, 4000), np.arange((1 << 31) - 8, (1 << 31) + 8),
                              np.arange(n - 12, n)]).astype(np.uint64)
        it = torch.from_numpy(idx.astype(np.int64)).cuda()
        g = to_host(vx[it], vy[it], vz[it])
        r = orc.sample_indices(2.5, 1.1, idx, 13, mode=1)
        assert norm_rel_err(g, r) <= TOL_FP32
    finally:
        del vx, vy, vz
        torch.cuda.empty_cache()


def test_determinism_and_chunking():
    n = 3_000_001
    for precision in (kp.FP64, kp.FP32):
        a = to_host(*gpu_sample(2.0, 1.0, n, 7, precision))
        b = to_host(*gpu_sample(2.0, 1.0, n, 7, precision))
        assert bits_equal(a, b)
        cut = 1_234_567
        c1 = to_host(*gpu_sample(2.0, 1.0, cut, 7, precision))
        c2 = to_host(*gpu_sample(2.0, 1.0, n - cut, 7, precision, counter_offset=cut))
        assert bits_equal(a, tuple(np.concatenate([x, y]) for x, y in zip(c1, c2)))


@pytest.mark.parametrize("precision", [kp.FP64, kp.FP32])
@pytest.mark.parametrize("n", [1000, 65_539, 100_000, 1_000_003])
def test_store_path_invariance(precision, n):
    """Outputs at any element offset give the bits of 16-byte aligned ones:
    views sharing one misalignment write the particles up to the 16-byte
    boundary one per thread and the rest with vector stores (from 2^16 + head
    particles on; one-per-thread below), and views at different
    misalignments take the one-per-thread path throughout."""
    dt = torch.float64 if precision == kp.FP64 else torch.float32
    ref = to_host(*kp.sample(4.0, 1.0, n, 3, counter_offset=9, precision=precision))
    per16 = 16 // (8 if precision == kp.FP64 else 4)
    offsets = [(o, o, o) for o in range(1, per16)] + [(1, 0, per16 - 1)]
    for offs in offsets:
        views = tuple(torch.empty(n + per16, dtype=dt, device="cuda")[o:o + n] for o in offs)
        assert [v.data_ptr() % 16 for v in views] == [o * (16 // per16) for o in offs]
        kp.sample(4.0, 1.0, n, 3, counter_offset=9, precision=precision, out=views)
        torch.cuda.synchronize()
        assert bits_equal(to_host(*views), ref), offs


def test_seg_id_selects_independent_stream(orc):
    n = 10_000
    a = to_host(*gpu_sample(3.0, 1.0, n, 1, kp.FP64, seg_id=5))
    r = orc.sample(3.0, 1.0, n, 1, seg=5, mode=0)[:3]
    assert norm_rel_err(a, r) <= TOL_FP64
    b = to_host(*gpu_sample(3.0, 1.0, n, 1, kp.FP64, seg_id=6))
    assert not np.allclose(a[0], b[0])


def test_device_errors_are_reported():
    """A 1-byte misaligned float pointer is rejected with KAPPA_EALIGN."""
    buf = torch.empty(64, dtype=torch.uint8, device="cuda")
    import ctypes
    from paper_2602_05606_amd import _lib
    p = ctypes.c_void_p(buf.data_ptr() + 1)
    st = _lib.load().kappa_sample(3.0, 1.0, 4, 0, 0, 0, kp.FP32, p, p, p, None)
    assert st == _lib.EALIGN


@pytest.mark.parametrize("prec", [kp.FP32, kp.FP64])
def test_chunked_and_reshaped_launches_give_the_same_bits(prec, monkeypatch):
    """A call larger than one launch runs as consecutive chunks; the launch
    shape can be overridden for tuning.  Neither changes a bit of the output,
    here over a counter range that crosses a 2^32 boundary (so chunks of both
    kernel forms run)."""
    n, off = 1_000_003, (1 << 32) - 5000
    ref = [t.clone() for t in kp.sample(3.0, 1.0, n, 7, counter_offset=off, precision=prec)]
    for env in ({"KAPPA_FORWARD_MAX_GRID": "3"}, {"KAPPA_FORWARD_MAX_GRID": "1000"},
                {"KAPPA_FORWARD_SHAPE": "64,1"}, {"KAPPA_FORWARD_SHAPE": "128,8"},
                {"KAPPA_FORWARD_SHAPE": "256,2", "KAPPA_FORWARD_MAX_GRID": "7"}):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        got = kp.sample(3.0, 1.0, n, 7, counter_offset=off, precision=prec)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), env
        for k in env:
            monkeypatch.delenv(k)
