"""Approximation-quality oracle (test infrastructure only, like all of oracle/).

Plain definitions of how far the approximation G is from the Kappa
distribution, evaluated with mpmath at 30 significant digits.  Only tests/,
the golden-file script beside them and the benchmark's CPU leg may use it.

* f(x; kappa)             Sec. 2, eq:kappax (beta-prime form, x = v^2/theta^2)
* G(x; kappa, c)          Sec. 3, eq:G with eq:qexp, q* = 1 + 1/kappa*
* g(x; kappa, c)          Sec. 3, eq:approx_x (the printed derivative of G)
* a, b/c, kappa*          Sec. 3, eq:a, eq:b, eq:k2; for a free c, b = (b/c) c
* c_approx                Sec. 3, eq:c
* kappa = inf             the Maxwell limit (Sec. 1, Sec. 3): f is the Maxwell
                          density in x, 2/sqrt(pi) x^(1/2) e^-x; exp_q* -> exp
                          in eq:G and eq:approx_x; a -> (4/(3 sqrt(pi)))^(2/3)
                          and b/c -> 1 (the limits Sec. 3 states)
* D(f||g; kappa, c)       Sec. 3, eq:relative_entropy, the integral over [0, inf)
* (E_approx - E_kappa)/E_kappa
                          Sec. 3, Fig. fig:DE(b); E_kappa from eq:kappaE, both
                          energies in units of m theta^2 / 2 so that
                          E = int x f(x) dx = 3 kappa / (2 kappa - 3)

* F(x; kappa)             Sec. 2, eq:CDF, the speed CDF (regularized
                          incomplete beta), and the binned relative entropy
                          D(P||Q) of the second test, Sec. 5, eq:KL

The integrals use mpmath's tanh-sinh quadrature on [0, inf) split at powers
of ten.  Where the printed formulas contain 1 - (1 + y)^(-k) or (1 + y)^p with
tiny y, they are evaluated as -expm1(-k log1p(y)) and exp(p log1p(y)): the
same numbers, without the loss of every digit near x = 0.
"""
import mpmath as mp

DPS = 30
# The Maxwell-limit c of the sampler (three figures of the minimiser of D with
# the Maxwell density, written by tests/golden/make_maxwell_golden.py).
C_MAXWELL = "0.079"
_SPLIT = [0] + [mp.mpf(10) ** e for e in range(-8, 312, 4)] + [mp.inf]


class Params:
    """kappa, kappa*, B(3/2, kappa - 1/2), a, b/c, c and b = (b/c) c."""

    def __init__(self, kappa, c=None):
        with mp.workdps(DPS):
            k = mp.mpf(kappa)
            self.kappa = k
            self.maxwell = mp.isinf(k)
            if self.maxwell:
                if c is None:
                    c = mp.mpf(C_MAXWELL)
                self.kstar = mp.inf
                self.B = None
                self.a = (4 / (3 * mp.sqrt(mp.pi))) ** (mp.mpf(2) / 3)
                self.b_over_c = mp.mpf(1)
            else:
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
    """eq:kappax: f(x) = (x/k)^(1/2) (1 + x/k)^-(k+1) / (k B(3/2, k - 1/2));
    for kappa = inf the Maxwell density 2/sqrt(pi) x^(1/2) e^-x."""
    k = p.kappa
    if p.maxwell:
        return 2 / mp.sqrt(mp.pi) * mp.sqrt(x) * mp.exp(-x)
    return mp.sqrt(x / k) * mp.exp(-(k + 1) * mp.log1p(x / k)) / (k * p.B)


def _u(x, p):
    """(a x + b x^2) / (1 + c x), the argument of exp_q* in eq:G."""
    return (p.a * x + p.b * x * x) / (1 + p.c * x)


def _y(x, p):
    """(a x + b x^2) / (kappa* (1 + c x)), the argument shared by eq:G and eq:approx_x."""
    return _u(x, p) / p.kstar


def _log_exp_q(x, p):
    """ln exp_q*(-u) = -kappa* ln(1 + u/kappa*) (eq:qexp); -u in the Maxwell limit."""
    if p.maxwell:
        return -_u(x, p)
    return -p.kstar * mp.log1p(_y(x, p))


def G_cdf(x, p):
    """eq:G: G = {1 - exp_q*(-(a x + b x^2)/(1 + c x))}^(3/2), with
    exp_q*(-u) = (1 + u/kappa*)^(-kappa*) (eq:qexp, 1 - q* = -1/kappa*)."""
    return (-mp.expm1(_log_exp_q(x, p))) ** (mp.mpf(3) / 2)


def G_complement(x, p):
    """1 - G of eq:G, written so that it keeps its digits when G is near 1."""
    E = mp.exp(_log_exp_q(x, p))
    return -mp.expm1(mp.mpf(3) / 2 * mp.log1p(-E))


def g_pdf(x, p):
    """eq:approx_x: 3(a + 2bx + bcx^2)/(2(1 + cx)^2) sqrt(1 - (1+y)^-k*) (1+y)^-(k*+1);
    in the Maxwell limit (1+y)^-k* -> e^-u and (1+y)^-(k*+1) -> e^-u."""
    lq = _log_exp_q(x, p)
    tail = lq if p.maxwell else lq - mp.log1p(_y(x, p))
    return (3 * (p.a + 2 * p.b * x + p.b * p.c * x * x) / (2 * (1 + p.c * x) ** 2)
            * mp.sqrt(-mp.expm1(lq)) * mp.exp(tail))


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
        e_kappa = mp.mpf(3) / 2 if p.maxwell else 3 * p.kappa / (2 * p.kappa - 3)
        return diff / e_kappa


def optimum_c(kappa, lo, hi, tol=1e-10):
    """The c in [lo, hi] that minimises D(f||g; kappa, c): the criterion of the
    grid search of Sec. 3 (Fig. fig:map), by golden-section search (D is
    unimodal in c on the brackets used here)."""
    with mp.workdps(DPS):
        return _golden(lambda c: relative_entropy(kappa, c), lo, hi, tol)


def _golden(fn, lo, hi, tol):
    invphi = (mp.sqrt(5) - 1) / 2
    a, b = mp.mpf(lo), mp.mpf(hi)
    c, d = b - invphi * (b - a), a + invphi * (b - a)
    fc, fd = fn(c), fn(d)
    while b - a > tol:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - invphi * (b - a)
            fc = fn(c)
        else:
            a, c, fc = c, d, fd
            d = a + invphi * (b - a)
            fd = fn(d)
    return float((a + b) / 2)


def quality(kappa, c=None):
    """(D, dE/E) as Python floats."""
    return float(relative_entropy(kappa, c)), float(energy_error(kappa, c))


def speed_cdf(kappa, x):
    """(F, 1 - F) of the speed in x = (v/theta)^2: eq:CDF, the regularized
    incomplete beta function I_{x/(x+kappa)}(3/2, kappa - 1/2), each side
    evaluated directly; for kappa = inf the Maxwell CDF P(3/2, x)."""
    with mp.workdps(DPS):
        k, x = mp.mpf(kappa), mp.mpf(x)
        if mp.isinf(k):
            F = mp.gammainc(mp.mpf(3) / 2, 0, x, regularized=True)
            R = mp.gammainc(mp.mpf(3) / 2, x, mp.inf, regularized=True)
        else:
            F = mp.betainc(mp.mpf(3) / 2, k - mp.mpf(1) / 2, 0, x / (x + k), regularized=True)
            R = mp.betainc(k - mp.mpf(1) / 2, mp.mpf(3) / 2, 0, k / (x + k), regularized=True)
        return F, R


def binned_relative_entropy(kappa, counts, bin_width, eps):
    """The Monte Carlo relative entropy of the second test (Sec. 5, eq:KL):
    sum_i (P_i + eps) ln((P_i + eps) / (Q_i + eps)), P_i the exact probability
    of speed bin [i w, (i+1) w) in units of theta (the last of len(counts)
    bins open-ended), Q_i = counts_i / sum(counts).  Returns (D, [P_i])."""
    with mp.workdps(DPS):
        n = len(counts)
        total = mp.fsum(mp.mpf(int(c)) for c in counts)
        w = mp.mpf(bin_width)
        P = []
        F0, R0 = mp.mpf(0), mp.mpf(1)
        for i in range(n):
            if i < n - 1:
                F1, R1 = speed_cdf(kappa, ((i + 1) * w) ** 2)
                P.append(F1 - F0 if F1 < mp.mpf(1) / 2 else R0 - R1)
                F0, R0 = F1, R1
            else:
                P.append(R0)
        e = mp.mpf(eps)
        D = mp.fsum((p + e) * mp.log((p + e) / (mp.mpf(int(c)) / total + e)) for p, c in zip(P, counts))
        return D, P
