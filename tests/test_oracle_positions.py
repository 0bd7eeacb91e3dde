"""Pins of the oracle's particle positions for fused particle loading.

Positions are not in the paper, which samples velocities only.  A PIC code
loads particles uniformly in each cell; the oracle places particle i of a
segment at lo + u size with u from the block of draw 1 of the same counter.
Checked here:
* uniform on [lo, lo + size) per axis (KS) and strictly inside the box;
* the axes are independent of each other and of the particle's velocity (a
  position drawn from the velocity's own block, draw 0, would tie y to the
  polar angle exactly);
* the FP32-mode lattice refines to the FP64 one (the same word, top 24 bits).
"""
import numpy as np
import pytest
from scipy import stats


LO = np.array([-3.0, 0.5, 100.0])
SIZE = np.array([0.25, 2.0, 1e-3])


@pytest.mark.parametrize("mode", [0, 1])
def test_uniform_inside_the_box(orc, mode):
    n = 200_000
    p = orc.positions(LO, SIZE, n, 11, counter_offset=5, seg=9, mode=mode)
    for k in range(3):
        u = (p[k] - LO[k]) / SIZE[k]
        assert np.all(p[k] >= LO[k]) and np.all(p[k] < LO[k] + SIZE[k])
        assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_independent_of_each_other_and_of_the_velocity(orc):
    n = 400_000
    px, py, pz = orc.positions(LO, SIZE, n, 3, seg=2)
    vx, vy, vz, _ = orc.sample(3.0, 1.0, n, 3, seg=2)
    speed = np.sqrt(vx * vx + vy * vy + vz * vz)
    cols = [px, py, pz, vx / speed, vy / speed, vz / speed, speed]
    c = np.corrcoef(np.array(cols))
    off = c[np.triu_indices(3, 1)]
    assert np.all(np.abs(off) < 5 / np.sqrt(n))
    assert np.all(np.abs(c[:3, 3:]) < 5 / np.sqrt(n))
    # rank correlation against the speed too (heavy tail)
    for q in (px, py, pz):
        assert abs(stats.spearmanr(q, speed).statistic) < 5 / np.sqrt(n)


def test_fp32_lattice_refines_to_fp64(orc):
    n = 10_000
    p64 = orc.positions([0, 0, 0], [1, 1, 1], n, 8, mode=0)
    p32 = orc.positions([0, 0, 0], [1, 1, 1], n, 8, mode=1)
    for a, b in zip(p64, p32):
        assert np.all(np.abs(a - b) <= 2.0 ** -24)
        # both are open midpoint dyadics of their lattice, and the FP32 one is exact in float
        assert np.all(np.modf(a * 2.0 ** 32)[0] == 0.5)
        assert np.all(np.modf(b * 2.0 ** 23)[0] == 0.5)
        assert np.all(b.astype(np.float32).astype(np.float64) == b)


def test_counter_offset_and_segments(orc):
    a = orc.positions(LO, SIZE, 100, 4, counter_offset=0, seg=1)
    b = orc.positions(LO, SIZE, 60, 4, counter_offset=40, seg=1)
    c = orc.positions(LO, SIZE, 100, 4, counter_offset=0, seg=2)
    for k in range(3):
        np.testing.assert_array_equal(a[k][40:], b[k][:60])
        assert not np.any(a[k] == c[k])


@pytest.mark.parametrize("lo, size, mode", [(3.5, 0.5, 1), (1e8, 1.0, 0), (1e8, 1.0, 1), (-4.0, 0.5, 0),
                                            (-4.0, 0.5, 1), (0.0, 1e-300, 0), (2.0, 1e-17, 0), (5.0, 0.0, 0)])
def test_extreme_words_stay_inside_the_half_open_box(orc, lo, size, mode):
    """The largest words give u = 1 - 2^-33 (FP64 mode) or 1 - 2^-24 (FP32
    modes): lo + u size then rounds to lo + size when |lo| is large against
    size, and the oracle caps it at the largest double below lo + size.
    Checked in exact rational arithmetic."""
    from fractions import Fraction
    for r in (0, 1, 0x7FFFFFFF, 0xFFFFFE00, 0xFFFFFFFF):
        p = orc.position_coord(lo, size, r, mode)
        assert Fraction(p) >= Fraction(lo)
        if size > 0:
            assert Fraction(p) < Fraction(lo) + Fraction(size), (lo, size, r, p)
        else:
            assert p == lo


def test_cap_only_where_rounding_reaches_the_upper_edge(orc):
    """Away from the edge the coordinate is lo + u size in FP64 (two
    roundings); at lo = 1e8, size = 1 the top word would round to 1e8 + 1
    and is capped to the double just below it."""
    rng = np.random.default_rng(5)
    for r in rng.integers(0, 2 ** 32 - 1024, size=2000, dtype=np.uint64):
        u = (float(r) + 0.5) * 2.0 ** -32
        assert orc.position_coord(-3.0, 0.25, int(r), 0) == -3.0 + u * 0.25
        u32 = (float(int(r) >> 9) + 0.5) * 2.0 ** -23
        assert orc.position_coord(100.0, 1e-3, int(r), 1) == 100.0 + u32 * 1e-3
    u = (float(0xFFFFFFFF) + 0.5) * 2.0 ** -32
    assert 1e8 + u * 1.0 == 1e8 + 1.0
    assert orc.position_coord(1e8, 1.0, 0xFFFFFFFF, 0) == np.nextafter(1e8 + 1.0, -np.inf)
