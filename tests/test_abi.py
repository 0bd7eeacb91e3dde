"""The C ABI on the CPU: the library loads, exports every entry point the
header declares, computes the Table 1 setup like the oracle, and rejects bad
arguments with the documented codes before any HIP call (so no GPU is needed).
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2602_05606_amd as kp
from paper_2602_05606_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kappa.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"KAPPA_API\s+[\w\s\*]*?\b(kappa_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("kappa_sample", "kappa_sample_batched", "kappa_sample_backward"):
        assert required in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    # and the binding's table covers the header exactly
    assert set(_lib.SIGNATURES) == set(declared_symbols())


def test_version_and_status_strings():
    assert "gfx950" in kp.version()
    lib = _lib.load()
    for code in range(7):
        assert lib.kappa_status_string(code).decode().startswith("KAPPA_")


@pytest.mark.parametrize("kappa", [1.5000001, 1.6, 2.0, 2.5, 3.0, 4.1, 7.5, 10.0, 15.0, 1e4])
def test_setup_matches_oracle(orc, kappa):
    got, ref = kp.params(kappa), orc.params(kappa)
    # c (eq:c) is a ratio of two quadratics whose denominator nearly cancels
    # near kappa = 4: its rounding error scales with the condition number of
    # the two sums, which the tolerance of c and b = (b/c) c carries.
    k = kappa
    cond_c = ((0.123 * k * k + 1.12 * k + 2.56) / abs(0.123 * k * k - 1.12 * k + 2.56)
              + (k * k + 7.89 * k + 15.6) / abs(k * k - 7.89 * k + 15.6))
    eps = 2.0 ** -52
    for name in ("kstar", "a", "b", "c", "b_over_c", "lnbeta"):
        tol = 8 * eps * (cond_c if name in ("b", "c") else 4.0)
        assert abs(got[name] - ref[name]) <= tol * abs(ref[name]) + 1e-300, name
    for name in ("da", "db", "dc"):
        assert abs(got[name] - ref[name]) <= 1e-12 * max(1.0, abs(ref[name])), name


FAKE = ctypes.c_void_p(0x10000)        # never dereferenced: validation fails first
FAKE_ODD = ctypes.c_void_p(0x10001)


@pytest.mark.parametrize("kappa,theta,prec,code", [
    (1.5, 1.0, 1, _lib.EINVAL), (1.0, 1.0, 1, _lib.EINVAL), (math.nan, 1.0, 1, _lib.EINVAL),
    (-math.inf, 1.0, 1, _lib.EINVAL), (3.0, 0.0, 1, _lib.EINVAL), (3.0, -1.0, 1, _lib.EINVAL),
    (3.0, math.nan, 1, _lib.EINVAL), (3.0, 1.0, 7, _lib.EINVAL), (3.0, 1.0, -1, _lib.EINVAL),
])
def test_sample_rejects_bad_arguments(kappa, theta, prec, code):
    lib = _lib.load()
    assert lib.kappa_sample(kappa, theta, 10, 0, 0, 0, prec, FAKE, FAKE, FAKE, None) == code
    assert lib.kappa_last_error()


def test_maxwell_limit_is_accepted_where_documented(orc):
    lib = _lib.load()
    got, ref = kp.params(math.inf), orc.params(math.inf)
    assert got == ref
    # the sampler takes +inf (fails later only for want of a GPU); backward and exact generators do not
    assert lib.kappa_sample(math.inf, 1.0, 10, 0, 0, 0, 1, FAKE_ODD, FAKE, FAKE, None) == _lib.EALIGN
    g = ctypes.c_void_p(0x10000)
    assert lib.kappa_sample_backward(math.inf, 1.0, 10, 0, 0, 0, 1, FAKE, FAKE, FAKE, g, FAKE, 1 << 20,
                                     None) == _lib.EINVAL
    assert lib.kappa_sample_exact_t(math.inf, 1.0, 10, 0, 1, FAKE, FAKE, FAKE, None, None) == _lib.EINVAL
    assert lib.kappa_sample_exact_pareto(math.inf, 1.0, 10, 0, 1, FAKE, FAKE, FAKE, None, None) == _lib.EINVAL


def test_sample_pointer_checks():
    lib = _lib.load()
    null = ctypes.c_void_p(0)
    assert lib.kappa_sample(3.0, 1.0, 10, 0, 0, 0, 1, null, FAKE, FAKE, None) == _lib.EINVAL
    assert lib.kappa_sample(3.0, 1.0, 10, 0, 0, 0, 1, FAKE_ODD, FAKE, FAKE, None) == _lib.EALIGN
    assert lib.kappa_sample(3.0, 1.0, 10, 0, 0, 0, 0, ctypes.c_void_p(0x10004), FAKE, FAKE, None) == _lib.EALIGN
    # n = 0 is a no-op, even with null pointers
    assert lib.kappa_sample(3.0, 1.0, 0, 0, 0, 0, 1, null, null, null, None) == _lib.OK
    # counter range overflow
    assert lib.kappa_sample(3.0, 1.0, 10, 0, (1 << 64) - 5, 0, 1, FAKE, FAKE, FAKE, None) == _lib.EINVAL


def test_backward_argument_checks():
    lib = _lib.load()
    n = 1000
    need = lib.kappa_backward_workspace_bytes(n)
    assert need >= 16 and need % 256 == 0
    assert lib.kappa_backward_workspace_bytes(0) >= 16
    args = (3.0, 1.0, n, 0, 0, 0, 1, FAKE, FAKE, FAKE, FAKE)
    assert lib.kappa_sample_backward(*args, FAKE, need - 1, None) == _lib.ERANGE
    assert lib.kappa_sample_backward(*args, ctypes.c_void_p(0x10010), need, None) == _lib.EALIGN
    assert lib.kappa_sample_backward(*args, None, need, None) == _lib.EINVAL
    assert lib.kappa_sample_backward(3.0, 1.0, n, 0, 0, 0, 1, FAKE, FAKE, FAKE, None, FAKE, need, None) == _lib.EINVAL
    assert lib.kappa_sample_backward(1.2, 1.0, n, 0, 0, 0, 1, FAKE, FAKE, FAKE, FAKE, FAKE, need, None) == _lib.EINVAL


def test_plan_argument_checks():
    lib = _lib.load()
    good = kp._segments([(3.0, 1.0, (0, 0, 0), 10, 0)])
    h = ctypes.c_void_p()
    assert lib.kappa_plan_create(good, 0, 0, 1, ctypes.byref(h)) == _lib.ERANGE
    assert lib.kappa_plan_create(None, 1, 0, 1, ctypes.byref(h)) == _lib.EINVAL
    assert lib.kappa_plan_create(good, 1, 0, 9, ctypes.byref(h)) == _lib.EINVAL
    for bad in ([(1.4, 1.0, (0, 0, 0), 10, 0)], [(3.0, 0.0, (0, 0, 0), 10, 0)],
                [(3.0, 1.0, (math.nan, 0, 0), 10, 0)]):
        assert lib.kappa_plan_create(kp._segments(bad), 1, 0, 1, ctypes.byref(h)) == _lib.EINVAL
    seg = kp._segments([(3.0, 1.0, (0, 0, 0), 10, 0)])
    seg[0].reserved = 1
    assert lib.kappa_plan_create(seg, 1, 0, 1, ctypes.byref(h)) == _lib.EINVAL
    over = kp._segments([(3.0, 1.0, (0, 0, 0), (1 << 64) - 1, 0), (3.0, 1.0, (0, 0, 0), 5, 1)])
    assert lib.kappa_plan_create(over, 2, 0, 1, ctypes.byref(h)) == _lib.ERANGE
    assert lib.kappa_plan_destroy(None) == _lib.OK
    assert lib.kappa_plan_launch(None, FAKE, FAKE, FAKE, None) == _lib.EINVAL


def test_plan_refuses_a_repeated_seg_id():
    """Particle j of a segment draws counter (j, seg_id): two segments with one
    seg_id (say the species index reused across cells) would repeat the same
    velocities, so the table is refused before any device call."""
    lib = _lib.load()
    h = ctypes.c_void_p()
    dup = kp._segments([(3.0, 1.0, (0, 0, 0), 10, 7), (2.0, 1.0, (0.1, 0, 0), 5, 3), (3.0, 1.0, (1, 0, 0), 10, 7)])
    assert lib.kappa_plan_create(dup, 3, 0, 1, ctypes.byref(h)) == _lib.EINVAL
    assert b"seg_id 7" in lib.kappa_last_error()
    cells = (kp.Cell * 3)()
    assert lib.kappa_load_particles(dup, cells, 3, 0, 1, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.EINVAL
    t = kp.segment_table([3.0] * 4, [1.0] * 4, [1] * 4, seg_id=[0, 1, 2, 1])
    assert lib.kappa_plan_create(t.ctypes.data_as(ctypes.POINTER(kp.Segment)), 4, 0, 1,
                                 ctypes.byref(h)) == _lib.EINVAL


def test_exact_and_probe_argument_checks():
    lib = _lib.load()
    assert lib.kappa_sample_exact_t(1.5, 1.0, 10, 0, 1, FAKE, FAKE, FAKE, None, None) == _lib.EINVAL
    assert lib.kappa_sample_exact_pareto(3.0, 1.0, 10, 0, 2, FAKE, FAKE, FAKE, None, None) == _lib.EINVAL
    assert lib.kappa_sample_exact_t(3.0, 1.0, 10, 0, 1, FAKE, FAKE, FAKE, ctypes.c_void_p(0x10002), None) == _lib.EALIGN
    assert lib.kappa_fill_probe(10, 1, FAKE, FAKE, ctypes.c_void_p(0x10004), None) == _lib.EALIGN
    assert lib.kappa_copy_probe(FAKE, FAKE, 15, None) == _lib.EALIGN
    assert lib.kappa_philox(4, 0, 0, 0, 0, ctypes.c_void_p(0x10004), None) == _lib.EALIGN
    assert lib.kappa_philox(0, 0, 0, 0, 0, None, None) == _lib.OK


def test_clock_probe_argument_checks():
    lib = _lib.load()
    blocks, hz = ctypes.c_uint32(7), ctypes.c_double(1.0)
    args = (3.0, 1.0, 1 << 20, 0, 0, 0, 1, FAKE, FAKE, FAKE)
    assert lib.kappa_clock_probe(*args, FAKE, 1 << 20, None, ctypes.byref(hz), None) == _lib.EINVAL
    # n = 0: nothing launched, no workgroups
    assert lib.kappa_clock_probe(3.0, 1.0, 0, 0, 0, 0, 1, None, None, None, None, 0,
                                 ctypes.byref(blocks), ctypes.byref(hz), None) == _lib.OK
    assert blocks.value == 0
    # outputs must allow the vector stores of the timed kernel
    odd = ctypes.c_void_p(0x10004)
    assert lib.kappa_clock_probe(3.0, 1.0, 1 << 20, 0, 0, 0, 1, FAKE, odd, FAKE, FAKE, 1 << 20,
                                 ctypes.byref(blocks), ctypes.byref(hz), None) == _lib.EALIGN
    assert lib.kappa_clock_probe(*args, None, 1 << 20, ctypes.byref(blocks), ctypes.byref(hz), None) == _lib.EINVAL
    assert lib.kappa_clock_probe(*args, ctypes.c_void_p(0x10004), 1 << 20, ctypes.byref(blocks),
                                 ctypes.byref(hz), None) == _lib.EALIGN
    # too few stamps: the workgroup count is still reported (FP32: 4 particles
    # per thread, 256 threads per workgroup), with no HIP call
    assert lib.kappa_clock_probe(*args, FAKE, 4, ctypes.byref(blocks), ctypes.byref(hz), None) == _lib.ERANGE
    assert blocks.value == (1 << 20) // 1024
    fp64 = (3.0, 1.0, 1 << 20, 0, 0, 0, 0, FAKE, FAKE, FAKE)
    assert lib.kappa_clock_probe(*fp64, FAKE, 4, ctypes.byref(blocks), ctypes.byref(hz), None) == _lib.ERANGE
    assert blocks.value == (1 << 20) // 512
    assert lib.kappa_clock_probe(1.5, *args[1:], FAKE, 1 << 20, ctypes.byref(blocks), ctypes.byref(hz),
                                 None) == _lib.EINVAL


def test_hardware_probe_argument_checks():
    lib = _lib.load()
    blocks, steps, hz = ctypes.c_uint32(7), ctypes.c_uint32(7), ctypes.c_double(1.0)
    assert lib.kappa_issue_probe(7, FAKE, 1 << 20, FAKE, 1 << 20, ctypes.byref(blocks), ctypes.byref(steps),
                                 ctypes.byref(hz), None) == _lib.EINVAL
    assert lib.kappa_issue_probe(-1, FAKE, 1 << 20, FAKE, 1 << 20, ctypes.byref(blocks), ctypes.byref(steps),
                                 ctypes.byref(hz), None) == _lib.EINVAL
    assert blocks.value == 0 and steps.value == 0
    assert lib.kappa_issue_probe(0, FAKE, 1 << 20, FAKE, 1 << 20, None, ctypes.byref(steps), ctypes.byref(hz),
                                 None) == _lib.EINVAL
    assert lib.kappa_transcendental_probe(7, FAKE, FAKE, 16, None) == _lib.EINVAL
    assert lib.kappa_transcendental_probe(0, None, None, 0, None) == _lib.OK
    assert lib.kappa_transcendental_probe(0, None, FAKE, 16, None) == _lib.EINVAL
    assert lib.kappa_transcendental_probe(0, FAKE_ODD, FAKE, 16, None) == _lib.EALIGN


def test_clock_probe_needs_one_launch(monkeypatch):
    # with at most 4 workgroups per launch, 2^20 particles need several launches,
    # which the probe (one launch, one stamp per workgroup) refuses
    monkeypatch.setenv("KAPPA_FORWARD_MAX_GRID", "4")
    lib = _lib.load()
    blocks, hz = ctypes.c_uint32(7), ctypes.c_double(1.0)
    assert lib.kappa_clock_probe(3.0, 1.0, 1 << 20, 0, 0, 0, 1, FAKE, FAKE, FAKE, FAKE, 1 << 20,
                                 ctypes.byref(blocks), ctypes.byref(hz), None) == _lib.ERANGE
    assert lib.kappa_clock_probe(3.0, 1.0, 4096, 0, 0, 0, 1, FAKE, FAKE, FAKE, FAKE, 3,
                                 ctypes.byref(blocks), ctypes.byref(hz), None) == _lib.ERANGE
    assert blocks.value == 4  # 4096 particles fit one launch of 4 workgroups; 3 stamps are too few


def test_histogram_and_divergence_argument_checks():
    lib = _lib.load()
    assert lib.kappa_speed_histogram(FAKE, FAKE, FAKE, 10, 1, 1.0, 0.2, 0, FAKE, None) == _lib.ERANGE
    assert lib.kappa_speed_histogram(FAKE, FAKE, FAKE, 10, 1, 1.0, 0.2, 2048, FAKE, None) == _lib.ERANGE
    assert lib.kappa_speed_histogram(FAKE, FAKE, FAKE, 10, 1, -1.0, 0.2, 10, FAKE, None) == _lib.EINVAL
    assert lib.kappa_speed_histogram(FAKE, FAKE, FAKE, 10, 1, 1.0, 0.2, 10, ctypes.c_void_p(0x10004), None) == _lib.EALIGN
    assert lib.kappa_speed_histogram(None, None, None, 0, 1, 1.0, 0.2, 10, FAKE, None) == _lib.OK
    div = lib.kappa_divergence_grid
    assert div(FAKE, 65536, FAKE, 1, FAKE, None, None, None) == _lib.ERANGE
    assert div(FAKE, 4, FAKE, (1 << 24) + 1, FAKE, None, None, None) == _lib.ERANGE
    assert div(FAKE, 4, None, 2, FAKE, None, None, None) == _lib.EINVAL     # eq:c column needs nc = 1
    assert div(None, 4, FAKE, 2, FAKE, None, None, None) == _lib.EINVAL
    assert div(FAKE, 4, FAKE, 2, ctypes.c_void_p(0x10004), None, None, None) == _lib.EALIGN
    assert div(FAKE, 4, FAKE, 2, FAKE, None, ctypes.c_void_p(0x10002), None) == _lib.EALIGN
    assert div(None, 0, None, 0, None, None, None, None) == _lib.OK


def test_segment_struct_layout():
    assert ctypes.sizeof(_lib.Segment) == 56


def test_workload_tables_shapes():
    import workloads
    segs = workloads.batched_segments()
    assert len(segs) == 4096 * 3
    counts = np.array([s["count"] for s in segs])
    assert counts.min() >= 1 and counts.max() <= 8192
    # mean of the clipped lognormal (mu = ln 256, sigma = 1) is about 256 e^{1/2} = 422
    assert 400 < counts.mean() < 445
    kappas = sorted({s["kappa"] for s in segs})
    assert len(kappas) == 3 and all(1.6 <= k <= 10 for k in kappas)
    assert [s["seg_id"] for s in segs] == list(range(len(segs)))
    chunks = workloads.c5_chunks()
    assert sum(c for _, c in chunks) == 10 ** 9 and len(chunks) == 4


def test_pic_argument_checks():
    lib = _lib.load()
    assert ctypes.sizeof(_lib.Cell) == 48
    assert lib.kappa_plan_set_cells(None, None) == _lib.EINVAL
    assert lib.kappa_plan_launch_pic(None, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.EINVAL
    assert lib.kappa_plan_graph_launch_pic(None, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.EINVAL
    segs = (_lib.Segment * 1)()
    segs[0].kappa, segs[0].theta, segs[0].count = 3.0, 1.0, 10
    assert lib.kappa_load_particles(segs, None, 1, 0, 1, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.EINVAL


def test_optimum_argument_checks():
    lib = _lib.load()
    opt = lib.kappa_optimum_c
    assert opt(FAKE, (1 << 24) + 1, FAKE, 10, 40, FAKE, None, None) == _lib.ERANGE
    assert opt(FAKE, 4, FAKE, 10, 201, FAKE, None, None) == _lib.ERANGE
    assert opt(FAKE, 4, FAKE, 0, 40, FAKE, None, None) == _lib.EINVAL
    assert opt(FAKE, 4, None, 10, 40, FAKE, None, None) == _lib.EINVAL
    assert opt(FAKE, 4, FAKE, 10, 40, ctypes.c_void_p(0x10004), None, None) == _lib.EALIGN
    assert opt(None, 0, None, 0, 40, None, None, None) == _lib.OK


def test_no_fallback_without_the_library(monkeypatch, tmp_path):
    """Every call goes through libkappa.so: without it the binding raises
    instead of computing anything on the host."""
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libkappa.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        kp.params(3.0)
    with pytest.raises(RuntimeError, match="no fallback"):
        kp.version()


def test_segment_table_layout_and_limit():
    """SEGMENT_DTYPE has the kappa_segment layout, a numpy table is passed
    without copying and equals the dict form byte for byte, and a count above
    KAPPA_MAX_SEGMENTS is refused before the table is read."""
    d = kp.SEGMENT_DTYPE
    assert d.itemsize == ctypes.sizeof(_lib.Segment) == 56
    for name in d.names:
        assert d.fields[name][1] == getattr(_lib.Segment, name).offset, name
    t = kp.segment_table([3.0, 4.1, 1.6], [1.0, 0.5, 2.0], [5, 0, 7], seg_id=[9, 3, 4],
                         drift=[[0.1, 0, 0], [0, 0.2, 0.3], [0, 0, -1]])
    view = kp._segments(t)
    ref = kp._segments([(3.0, 1.0, (0.1, 0, 0), 5, 9), (4.1, 0.5, (0, 0.2, 0.3), 0, 3), (1.6, 2.0, (0, 0, -1), 7, 4)])
    assert bytes(view) == bytes(ref)
    t["count"][0] = 11  # a view, not a copy
    assert view[0].count == 11
    with pytest.raises(ValueError):
        kp._segments(t[::2])
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.kappa_plan_create(view, (1 << 24) + 1, 0, 1, ctypes.byref(h)) == _lib.ERANGE


def test_backward_noalloc_argument_checks(monkeypatch):
    """The allocation-free backward validates like kappa_sample_backward and
    refuses a grid whose partials exceed its static array, before any HIP call."""
    lib = _lib.load()
    FAKE = ctypes.c_void_p(0x10000)
    n = 1 << 20
    assert lib.kappa_sample_backward_noalloc(1.2, 1.0, n, 0, 0, 0, 1, FAKE, FAKE, FAKE, FAKE, None) == _lib.EINVAL
    assert lib.kappa_sample_backward_noalloc(3.0, 0.0, n, 0, 0, 0, 1, FAKE, FAKE, FAKE, FAKE, None) == _lib.EINVAL
    assert lib.kappa_sample_backward_noalloc(3.0, 1.0, n, 0, 0, 0, 7, FAKE, FAKE, FAKE, FAKE, None) == _lib.EINVAL
    assert lib.kappa_sample_backward_noalloc(3.0, 1.0, n, 0, 0, 0, 1, FAKE, FAKE, FAKE, None, None) == _lib.EINVAL
    assert lib.kappa_sample_backward_noalloc(3.0, 1.0, n, 0, 0, 0, 1, None, FAKE, FAKE, FAKE, None) == _lib.EINVAL
    assert lib.kappa_sample_backward_noalloc(3.0, 1.0, n, 0, 0, 0, 1, ctypes.c_void_p(0x10002), FAKE, FAKE, FAKE,
                                             None) == _lib.EALIGN
    assert lib.kappa_sample_backward_noalloc(math.inf, 1.0, n, 0, 0, 0, 1, FAKE, FAKE, FAKE, FAKE,
                                             None) == _lib.EINVAL
    # a grid of 8192 partial blocks (2^23 particles at 1024 per block) needs 128 KiB: more than the 64 KiB array
    monkeypatch.setenv("KAPPA_BACKWARD_GRID", "8192")
    assert lib.kappa_sample_backward_noalloc(3.0, 1.0, 1 << 23, 0, 0, 0, 1, FAKE, FAKE, FAKE, FAKE,
                                             None) == _lib.ERANGE
    assert "static scratch" in lib.kappa_last_error().decode()


def test_sample_autotune_argument_checks():
    """kappa_sample_autotune validates before any HIP call."""
    lib = _lib.load()
    FAKE = ctypes.c_void_p(0x10000)
    b, u = ctypes.c_int(), ctypes.c_int()
    assert lib.kappa_sample_autotune(1, 0, FAKE, FAKE, FAKE, 3, ctypes.byref(b), ctypes.byref(u), None) == _lib.EINVAL
    assert lib.kappa_sample_autotune(9, 1000, FAKE, FAKE, FAKE, 3, None, None, None) == _lib.EINVAL
    assert lib.kappa_sample_autotune(1, 1000, FAKE, FAKE, FAKE, 0, None, None, None) == _lib.EINVAL
    assert lib.kappa_sample_autotune(1, 1000, None, FAKE, FAKE, 3, None, None, None) == _lib.EINVAL
    assert lib.kappa_sample_autotune(1, 1000, ctypes.c_void_p(0x10004), FAKE, FAKE, 3, None, None,
                                     None) == _lib.EALIGN
