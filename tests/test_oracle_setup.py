"""Oracle pins for the per-species setup (Table 1, first four rows).

Pins, none of which retypes the setup formulas:
  * limits the paper states for a and b/c at kappa -> 3/2 and kappa -> inf,
    and where the two curves cross (Sec. 3, eq:a and eq:b);
  * the extrema of c_approx the paper states (eq:c);
  * asymptotic matching, which is how the paper derives a, kappa* and b/c:
    G/F -> 1 as x -> 0 and (1-G)/(1-F) -> 1 as x -> inf, with F the exact
    Beta-prime CDF of eq:CDF from scipy's regularized incomplete beta;
  * the next Taylor coefficient of G at x -> 0 printed in eq:G_taylor_0;
  * digamma against scipy, and the kappa-derivatives against central
    differences of the parameters.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import optimize, special

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_statements.json")))
KAPPAS = [1.6, 2.0, 2.5, 3.0, 4.0, 4.1, 6.0, 7.5, 10.0, 15.0]


def exact_cdf(x, k):
    return special.betainc(1.5, k - 0.5, x / (x + k))


def exact_ccdf(x, k):
    # 1 - I_y(3/2, k-1/2) = I_{1-y}(k-1/2, 3/2) with 1-y = k/(x+k) formed directly
    return special.betainc(k - 0.5, 1.5, k / (x + k))


def test_limit_at_three_halves(orc):
    v = GOLD["a_and_b_over_c_at_kappa_three_halves"]["value"]
    p = orc.params(1.5 + 1e-10)
    assert abs(p["a"] - v) < 1e-8
    assert abs(p["b_over_c"] - v) < 1e-8


def test_limit_large_kappa(orc):
    a_inf = (4.0 / (3.0 * math.sqrt(math.pi))) ** (2.0 / 3.0)
    assert abs(a_inf - GOLD["a_limit_large_kappa"]["approx"]) < 5e-4
    p = orc.params(1e7)
    assert abs(p["a"] / a_inf - 1) < 1e-6
    assert abs(p["b_over_c"] - GOLD["b_over_c_limit_large_kappa"]["value"]) < 1e-5


def test_a_and_b_over_c_increase_and_cross(orc):
    ks = np.linspace(1.51, 30, 400)
    a = np.array([orc.params(k)["a"] for k in ks])
    r = np.array([orc.params(k)["b_over_c"] for k in ks])
    assert np.all(np.diff(a) > 0) and np.all(np.diff(r) > 0)
    cross = optimize.brentq(lambda k: orc.params(k)["a"] - orc.params(k)["b_over_c"], 3.0, 6.0)
    assert abs(cross - GOLD["a_b_over_c_crossing_kappa"]["approx"]) < 0.1


def test_c_extrema(orc):
    kmax = optimize.minimize_scalar(lambda k: -orc.params(k)["c"], bounds=(3.0, 4.4), method="bounded").x
    kmin = optimize.minimize_scalar(lambda k: orc.params(k)["c"], bounds=(4.4, 6.0), method="bounded").x
    gmax, gmin = GOLD["c_approx_maximum"], GOLD["c_approx_minimum"]
    assert abs(kmax - gmax["kappa"]) < 0.05 and abs(orc.params(kmax)["c"] - gmax["c"]) < 0.05
    assert abs(kmin - gmin["kappa"]) < 0.05 and abs(orc.params(kmin)["c"] - gmin["c"]) < 0.005
    # c > 0 everywhere (both quadratics of eq:c have no real root), hence b > 0
    for k in np.linspace(1.5001, 50, 2000):
        p = orc.params(k)
        assert p["c"] > 0 and p["b"] > 0


@pytest.mark.parametrize("k", KAPPAS)
def test_small_x_matching(orc, k):
    """G/F -> 1 as x -> 0, with error linear in x (this fixes a, eq:a)."""
    r = [orc.G(k, x)[0] / exact_cdf(x, k) - 1 for x in (1e-6, 1e-7, 1e-8)]
    assert abs(r[2]) < 1e-9
    # error shrinks linearly with x: next term of eq:F_taylor_0 / eq:G_taylor_0
    assert abs(r[0] / r[1] - 10) < 0.05 and abs(r[1] / r[2] - 10) < 0.05


@pytest.mark.parametrize("k", KAPPAS)
def test_large_x_matching(orc, k):
    """(1-G)/(1-F) -> 1 as x -> inf (this fixes kappa* and b/c, eq:k2, eq:b)."""
    for x in (1e9, 1e11, 1e13):
        h = orc.G(k, x)[1]
        assert abs(h / exact_ccdf(x, k) - 1) < 1e-6, (x, h, exact_ccdf(x, k))


@pytest.mark.parametrize("k", KAPPAS)
def test_taylor_coefficient_at_zero(orc, k):
    """eq:G_taylor_0: G = a^{3/2} x^{3/2} {1 + (3/2)((b - ac)/a - (k*+1) a/(2k*)) x + O(x^2)}."""
    p = orc.params(k)
    a, b, c, ks = p["a"], p["b"], p["c"], p["kstar"]
    coef = 1.5 * ((b - a * c) / a - (ks + 1) * a / (2 * ks))
    x = 1e-5
    g = orc.G(k, x)[0]
    est = (g / (a ** 1.5 * x ** 1.5) - 1) / x
    assert abs(est - coef) < 1e-3 * max(1.0, abs(coef))
    # and F's own coefficient (eq:F_taylor_0) differs from G's: the match is only at order x^{3/2}
    f_est = (exact_cdf(x, k) / (a ** 1.5 * x ** 1.5) - 1) / x
    assert abs(f_est + 3 * (k + 1) / (5 * k)) < 1e-3


@pytest.mark.parametrize("x", [1.0001, 1.1, 1.5, 2.0, 2.5, 3.7, 5.5, 11.0, 16.0, 40.0])
def test_digamma(orc, x):
    assert abs(orc.digamma(x) - special.digamma(x)) < 2e-15 * max(1, abs(special.digamma(x)))


@pytest.mark.parametrize("k", KAPPAS)
def test_parameter_derivatives(orc, k):
    h = 1e-5
    up, dn, p = orc.params(k + h), orc.params(k - h), orc.params(k)
    for name, dname in (("a", "da"), ("b", "db"), ("c", "dc")):
        fd = (up[name] - dn[name]) / (2 * h)
        assert abs(p[dname] - fd) < 1e-7 * max(1.0, abs(fd)), (name, p[dname], fd)
