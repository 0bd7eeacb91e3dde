"""Approximation-quality oracle (test infrastructure only, like all of oracle/).

Plain definitions of how far the approximation G is from the Kappa
distribution, evaluated with mpmath at 30 significant digits.  Only tests/,
the golden-file script beside them and the benchmark's CPU leg may use it.

* f(x; kappa)             Sec. 2, eq:kappax (beta-prime form, x = v^2/theta^2)
* G(x; kappa, c)          Sec. 3, eq:G with eq:qexp, q* = 1 + 1/kappa*
* g(x; kappa, c)          Sec. 3, eq:approx_x (the printed derivative of G)
* a, b/c, kappa*          Sec. 3, eq:a, eq:b, eq:k2; for a free c, b = (b/c) c
* c_approx                Sec. 3, eq:c
* D(f||g; kappa, c)       Sec. 3, eq:relative_entropy, the integral over [0, inf)
* (E_approx - E_kappa)/E_kappa
                          Sec. 3, Fig. fig:DE(b); E_kappa from eq:kappaE, both
                          energies in units of m theta^2 / 2 so that
                          E = int x f(x) dx = 3 kappa / (2 kappa - 3)

The integrals use mpmath's tanh-sinh quadrature on [0, inf) split at powers
of ten.  Where the printed formulas contain 1 - (1 + y)^(-k) or (1 + y)^p with
tiny y, they are evaluated as -expm1(-k log1p(y)) and exp(p log1p(y)): the
same numbers, without the loss of every digit near x = 0.
"""
import mpmath as mp

DPS = 30
_SPLIT = [0] + [mp.mpf(10) ** e for e in range(-8, 312, 4)] + [mp.inf]


class Params:
    """kappa, kappa*, B(3/2, kappa - 1/2), a, b/c, c and b = (b/c) c."""

    def __init__(self, kappa, c=None):
        with mp.workdps(DPS):
            k = mp.mpf(kappa)
            self.kappa = k
            self.kstar = k - mp.mpf(1) / 2                                   # eq:k2
            self.B = mp.beta(mp.mpf(3) / 2, k - mp.mpf(1) / 2)
            self.a = (2 / (3 * self.B)) ** (mp.mpf(2) / 3) / k                # eq:a
            self.b_over_c = (self.kstar * mp.mpf(3) / 2 * self.B) ** (1 / self.kstar) * self.kstar / k  # eq:b
            self.c = c_approx(k) if c is None else mp.mpf(c)
            self.b = self.b_over_c * self.c


def c_approx(kappa):
    """eq:c: the fitted c as a function of kappa."""
    with mp.workdps(DPS):
        k = mp.mpf(kappa)
        return (mp.mpf("0.123") * k * k - mp.mpf("1.12") * k + mp.mpf("2.56")) / \
               (k * k - mp.mpf("7.89") * k + mp.mpf("15.6"))


def f_pdf(x, p):
    """eq:kappax: f(x) = (x/k)^(1/2) (1 + x/k)^-(k+1) / (k B(3/2, k - 1/2))."""
    k = p.kappa
    return mp.sqrt(x / k) * mp.exp(-(k + 1) * mp.log1p(x / k)) / (k * p.B)


def _y(x, p):
    """(a x + b x^2) / (kappa* (1 + c x)), the argument shared by eq:G and eq:approx_x."""
    return (p.a * x + p.b * x * x) / (p.kstar * (1 + p.c * x))


def G_cdf(x, p):
    """eq:G: G = {1 - exp_q*(-(a x + b x^2)/(1 + c x))}^(3/2), with
    exp_q*(-u) = (1 + u/kappa*)^(-kappa*) (eq:qexp, 1 - q* = -1/kappa*)."""
    return (-mp.expm1(-p.kstar * mp.log1p(_y(x, p)))) ** (mp.mpf(3) / 2)


def G_complement(x, p):
    """1 - G of eq:G, written so that it keeps its digits when G is near 1."""
    E = mp.exp(-p.kstar * mp.log1p(_y(x, p)))
    return -mp.expm1(mp.mpf(3) / 2 * mp.log1p(-E))


def g_pdf(x, p):
    """eq:approx_x: 3(a + 2bx + bcx^2)/(2(1 + cx)^2) sqrt(1 - (1+y)^-k*) (1+y)^-(k*+1)."""
    y = _y(x, p)
    l1p = mp.log1p(y)
    return (3 * (p.a + 2 * p.b * x + p.b * p.c * x * x) / (2 * (1 + p.c * x) ** 2)
            * mp.sqrt(-mp.expm1(-p.kstar * l1p)) * mp.exp(-(p.kstar + 1) * l1p))


def integrate(fn):
    """int_0^inf fn(x) dx by tanh-sinh quadrature on power-of-ten pieces."""
    with mp.workdps(DPS):
        return mp.quad(fn, _SPLIT)


def relative_entropy(kappa, c=None):
    """eq:relative_entropy: D(f||g; kappa, c) = int f ln(f/g) dx (c=None: eq:c)."""
    with mp.workdps(DPS):
        p = Params(kappa, c)

        def integrand(x):
            if x == 0:
                return mp.mpf(0)
            fx = f_pdf(x, p)
            return fx * mp.log(fx / g_pdf(x, p))
        return integrate(integrand)


def energy_error(kappa, c=None):
    """Fig. fig:DE(b): (E_approx - E_kappa)/E_kappa = int x (g - f) dx / (3k/(2k-3))."""
    with mp.workdps(DPS):
        p = Params(kappa, c)
        diff = integrate(lambda x: x * (g_pdf(x, p) - f_pdf(x, p)))
        return diff / (3 * p.kappa / (2 * p.kappa - 3))


def quality(kappa, c=None):
    """(D, dE/E) as Python floats."""
    return float(relative_entropy(kappa, c)), float(energy_error(kappa, c))
