"""Exact reference distributions and statistical checks used by the tests.

These are written independently of both the oracle and the HIP library: each
CDF is obtained by numerical integration of the density the paper defines.
"""
import numpy as np
from scipy import integrate, stats


def upar_cdf_factory(a, x):
    """CDF of the parallel atom velocity, f(u) ~ exp(-u^2) / (a^2 + (x-u)^2)
    (eq. uparf), by the substitution u = x + a tan(theta), under which
    f du ~ exp(-(x + a tan theta)^2) d theta, integrated on a grid that is
    uniform and log-spaced in theta + pi/2 (to resolve the Gaussian bump)."""
    sgn = -1.0 if x < 0 else 1.0
    X = abs(x)
    phi = np.unique(np.concatenate([np.logspace(-15, np.log10(np.pi), 40001),
                                    np.linspace(0.0, np.pi, 40001)]))
    phi = phi[(phi > 0) & (phi < np.pi)]
    # theta = phi - pi/2, tan(theta) = -1/tan(phi); the density vanishes at both ends
    with np.errstate(divide="ignore", over="ignore"):
        u = X - a / np.tan(phi)
        g = np.exp(-u * u)
    phi = np.concatenate([[0.0], phi, [np.pi]])
    g = np.concatenate([[0.0], g, [0.0]])
    cum = np.concatenate([[0.0], integrate.cumulative_trapezoid(g, phi)])
    cum /= cum[-1]

    def cdf(v):
        v = np.asarray(v, float) * sgn           # f(-x, u) = f(x, -u)
        ph = np.arctan2(a, X - v)                 # phi in (0, pi)
        F = np.interp(ph, phi, cum)
        return F if sgn > 0 else 1.0 - F
    return cdf


def upar_split_numeric(a, x, u0):
    """Probability that the two-part comparison function draws u <= u0
    (Sec. 3.2.3), by direct quadrature in u of g1 below u0 and g2 above."""
    def lor(u):
        return 1.0 / (a * a + (x - u) ** 2)

    def q(lo, hi):
        return integrate.quad(lor, lo, hi, limit=500, epsabs=0.0, epsrel=1e-11)[0]
    w = 200.0 * a
    lo_part = q(-np.inf, u0)
    hi_part = q(u0, x - w) + q(x - w, x) + q(x, x + w) + q(x + w, np.inf)
    return lo_part / (lo_part + np.exp(-u0 * u0) * hi_part)


def mu_cdf_factory(rW):
    """CDF of the scattering-angle cosine for W(mu) ~ 1 + rW mu^2, by quadrature."""
    grid = np.linspace(-1.0, 1.0, 20001)
    dens = 1.0 + rW * grid * grid
    cum = np.concatenate([[0.0], integrate.cumulative_trapezoid(dens, grid)])
    cum /= cum[-1]
    return lambda m: np.interp(m, grid, cum)


def ks_p(samples, cdf):
    return stats.kstest(np.asarray(samples), cdf).pvalue


def binomial_z(k, n, p):
    """z-score of k successes in n trials with probability p."""
    return (k - n * p) / np.sqrt(max(n * p * (1 - p), 1e-300))


def chi2_two_hist_p(h1, h2, min_count=5):
    """Two-sample chi-square homogeneity test of count histograms (bins with a
    combined count below min_count are merged into their neighbours)."""
    h1 = np.asarray(h1, float)
    h2 = np.asarray(h2, float)
    a, b = [], []
    ca = cb = 0.0
    for x, y in zip(h1, h2):
        ca += x
        cb += y
        if ca + cb >= min_count:
            a.append(ca)
            b.append(cb)
            ca = cb = 0.0
    if ca + cb > 0 and a:
        a[-1] += ca
        b[-1] += cb
    a = np.array(a)
    b = np.array(b)
    if len(a) < 2:
        return 1.0
    table = np.vstack([a, b])
    return stats.chi2_contingency(table, correction=False)[1]


def sphere_J(x, atau0):
    """Emergent angle-averaged intensity of a static uniform sphere (eq. sphere)."""
    return (1.0 / 8.0) * np.sqrt(np.pi / 6.0) * x * x / atau0 / \
        np.cosh(np.sqrt(np.pi ** 3 / 54.0) * x ** 3 / atau0) ** 2


def slab_J(x, atau0):
    """Emergent angle-averaged intensity of a static uniform slab (eq. neufeld)."""
    return 1.0 / (4.0 * np.sqrt(6.0 * np.pi)) * x * x / atau0 / \
        np.cosh(np.sqrt(np.pi ** 3 / 54.0) * x ** 3 / atau0)


def mirror_walk(x):
    """Symmetry about zero of a sample: with the values ordered by |x|
    (largest first), the walk of their signs; under symmetry it is a simple
    random walk, so its largest excursion over sqrt(n) exceeds c with
    probability at most 4 Q(c) (reflection principle, both signs)."""
    x = np.asarray(x, float)
    x = x[x != 0]
    s = np.sign(x[np.argsort(-np.abs(x), kind="stable")])
    return np.abs(np.cumsum(s)).max() / np.sqrt(len(s))
