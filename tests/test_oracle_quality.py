"""Pins of the approximation-quality oracle (oracle/quality.py).

Each pin ties the oracle to something other than itself:
* g of eq:approx_x is the derivative of G of eq:G (numerical differentiation
  of G at 30 digits);
* normalisation: int f = int g = 1, and int x f dx = 3k/(2k-3), the closed
  form of eq:kappaE;
* a and b/c agree with the C oracle's setup (a second implementation);
* D along eq:c agrees with an FP64 scipy quadrature over the C oracle's g;
* the energy error agrees with the mean of x over the inverse-transform
  speeds of the C oracle (a route that never evaluates g);
* the grid-search statements of Sec. 3 (Fig. fig:map): the optimum c sits on
  eq:c in the fitted ranges, runs off the top of the c range just below
  kappa 4.1 and drops to zero just above it;
* the tail-energy argument at kappa 4.1 (about 1% of the particles above
  v = 3 theta missing, 19% of the energy there, so 0.19% of it lost), with
  the tails of eq:CDF and eq:CDF_E from scipy's incomplete beta function.
A mutation test plants mistakes in the oracle and checks that a pin fails.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special

from oracle import quality as Q

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_statements.json")))


@pytest.mark.parametrize("k,c", [(1.6, 0.0), (3.0, 0.33), (4.1, None), (10.0, 1.5)])
def test_g_is_the_derivative_of_G(k, c):
    with mp.workdps(Q.DPS):
        p = Q.Params(k, c)
        for x in ("1e-6", "0.3", "1", "7", "400", "1e9"):
            x = mp.mpf(x)
            g = Q.g_pdf(x, p)
            if Q.G_cdf(x, p) < 0.5:
                d = mp.diff(lambda t: Q.G_cdf(t, p), x)
            else:  # differentiate 1 - G where G is close to 1
                d = -mp.diff(lambda t: Q.G_complement(t, p), x)
            assert abs(g / d - 1) < mp.mpf(10) ** -20
            assert abs(Q.G_cdf(x, p) + Q.G_complement(x, p) - 1) < mp.mpf(10) ** -25


@pytest.mark.parametrize("k,c", [(1.6, 0.7), (4.1, 0.0), (7.5, None)])
def test_normalisation_and_energy_closed_form(k, c):
    with mp.workdps(Q.DPS):
        p = Q.Params(k, c)
        tol = mp.mpf(10) ** -20
        assert abs(Q.integrate(lambda x: Q.g_pdf(x, p)) - 1) < tol
        assert abs(Q.integrate(lambda x: Q.f_pdf(x, p)) - 1) < tol
        ex = Q.integrate(lambda x: x * Q.f_pdf(x, p))
        assert abs(ex / (3 * p.kappa / (2 * p.kappa - 3)) - 1) < tol


@pytest.mark.parametrize("k", [1.6, 4.1, 10.0])
def test_setup_matches_the_c_oracle(orc, k):
    p = Q.Params(k)
    ref = orc.params(k)
    assert abs(float(p.a) / ref["a"] - 1) < 1e-14
    assert abs(float(p.b_over_c) / ref["b_over_c"] - 1) < 1e-14
    # eq:c's denominator cancels to about 0.06 near kappa 4.1 (condition ~ 300)
    assert abs(float(p.c) / ref["c"] - 1) < 1e-12


def _scipy_relative_entropy(orc, k):
    lnB = special.betaln(1.5, k - 0.5)

    def integrand(x):
        if x <= 0:
            return 0.0
        fx = math.exp(-math.log(k) - lnB + 0.5 * math.log(x / k) - (k + 1) * math.log1p(x / k))
        return fx * math.log(fx / orc.g_pdf(k, x)) if fx > 0 else 0.0

    edges = [0, 1e-6, 1e-3, 0.1, 1, 3, 10, 30, 100, 1e3, 1e4, 1e5, 1e6, 1e8, 1e10, np.inf]
    return sum(integrate.quad(integrand, lo, hi, limit=400, epsabs=1e-16, epsrel=1e-10)[0]
               for lo, hi in zip(edges[:-1], edges[1:]))


@pytest.mark.parametrize("k", [3.0, 4.1, 7.5])
def test_relative_entropy_matches_an_fp64_quadrature_of_the_c_oracle(orc, k):
    d = float(Q.relative_entropy(k))
    assert abs(d / _scipy_relative_entropy(orc, k) - 1) < 1e-5


@pytest.mark.parametrize("k", [2.3, 4.1])
def test_energy_error_matches_the_sampler_mean(orc, k):
    """<x> under G is int_0^1 x(U) dU over the inverse transform, which never
    evaluates g; split at U = 1/2 with the high side in W = 1 - U."""
    lo = integrate.quad(lambda u: orc.speed(k, orc.SIDE_LOW, u) ** 2, 0, 0.5, limit=200, epsabs=0, epsrel=1e-12)[0]
    hi = integrate.quad(lambda w: orc.speed(k, orc.SIDE_HIGH, w) ** 2, 0, 0.5, limit=400, epsabs=0, epsrel=1e-12)[0]
    ref = (lo + hi) / (3 * k / (2 * k - 3)) - 1
    assert abs(float(Q.energy_error(k)) - ref) < 1e-9


def test_grid_search_statements():
    """Sec. 3, Fig. fig:map: in the fitted ranges the optimum c is close to
    eq:c; just below kappa 4.1 it runs past the top of the c range [0, 1.5];
    just above 4.1 it is zero."""
    D = Q.relative_entropy
    ca = float(Q.c_approx(3.0))
    assert D(3.0, ca) < D(3.0, ca - 0.1) and D(3.0, ca) < D(3.0, ca + 0.1)
    assert D(8.0, float(Q.c_approx(8.0))) < D(8.0, 0.0)
    assert D(3.9, 1.5) < D(3.9, 1.2)
    assert D(4.2, 0.0) < D(4.2, 0.05)
    # the fit anchor (4.1, 0.4) is not the optimum there: c has little effect near 4.1
    assert abs(D(4.1, 0.4) / D(4.1, 0.0) - 1) < 0.5


def test_tail_energy_argument_at_kappa_4p1():
    """Sec. 3, discussion of fig:DE(b): at kappa 4.1 the approximation puts
    about 1% too few particles above v = 3 theta (x = 9); eq:CDF_E says that
    tail carries about 19% of the energy, so about 0.19% of the energy goes
    missing, in line with the 10^-2.5 energy error there.  Each step is
    checked against the exact beta-prime tails, not the oracle's own f."""
    st = GOLD["energy_tail_fraction_v_gt_3theta_kappa_4p1"]
    k, x0 = st["kappa"], st["x"]
    pop_kappa = special.betaincc(1.5, k - 0.5, x0 / (x0 + k))     # eq:CDF
    energy_kappa = special.betaincc(2.5, k - 1.5, x0 / (x0 + k))  # eq:CDF_E
    assert round(energy_kappa, 2) == st["approx"]
    with mp.workdps(Q.DPS):
        p = Q.Params(k)
        pop_approx = float(Q.G_complement(mp.mpf(x0), p))
        e_kappa = 3 * k / (2 * k - 3)  # mean x of the Kappa distribution, eq:kappaE
        tail_approx = float(mp.quad(lambda x: x * Q.g_pdf(x, p), [x0, 30, 100, 1000, mp.inf])) / e_kappa
    lost_population = 1 - pop_approx / pop_kappa
    assert 0.005 < lost_population < 0.02          # "1% of the tail population"
    lost_energy = energy_kappa - tail_approx
    assert 0.0015 < lost_energy < 0.0025           # "0.19% of the energy density"
    assert abs(lost_energy - lost_population * energy_kappa) < 0.0005
    # the whole energy error at 4.1 is of order 10^-2.5 (fig:DE(b))
    de = abs(float(Q.energy_error(k)))
    assert abs(math.log10(de) - GOLD["energy_error_at_transition"]["log10_approx"]) < 0.25


def test_paper_level_along_eq_c():
    """Fig. fig:DE(a): D is about 1e-6 for kappa above about 5."""
    level = GOLD["relative_entropy_high_kappa_level"]["approx"]
    assert level / 3 < Q.relative_entropy(6.0) < 3 * level


# ----------------------------------------------------------------------------- mutations

def _mutant_g_drops_2(x, p):
    y = Q._y(x, p)
    l1p = mp.log1p(y)
    return (3 * (p.a + p.b * x + p.b * p.c * x * x) / (2 * (1 + p.c * x) ** 2)
            * mp.sqrt(-mp.expm1(-p.kstar * l1p)) * mp.exp(-(p.kstar + 1) * l1p))


def _mutant_g_power(x, p):
    y = Q._y(x, p)
    l1p = mp.log1p(y)
    return (3 * (p.a + 2 * p.b * x + p.b * p.c * x * x) / (2 * (1 + p.c * x) ** 2)
            * mp.sqrt(-mp.expm1(-p.kstar * l1p)) * mp.exp(-p.kstar * l1p))


def _mutant_f_exponent(x, p):
    k = p.kappa
    return mp.sqrt(x / k) * mp.exp(-k * mp.log1p(x / k)) / (k * p.B)


@pytest.mark.parametrize("name,target,mutant", [
    ("g drops the 2 of 2bx", "g_pdf", _mutant_g_drops_2),
    ("g with exponent -k* instead of -(k*+1)", "g_pdf", _mutant_g_power),
    ("f with exponent -k instead of -(k+1)", "f_pdf", _mutant_f_exponent),
])
def test_pins_catch_planted_mistakes(monkeypatch, name, target, mutant):
    monkeypatch.setattr(Q, target, mutant)
    caught = False
    try:
        if target == "g_pdf":
            test_g_is_the_derivative_of_G(3.0, 0.33)
        else:
            test_normalisation_and_energy_closed_form(3.0, 0.3)
    except AssertionError:
        caught = True
    assert caught, name
