"""Pins of the oracle's Klein-Nishina cross-section, angular CDF and inverse
CDF (the conventional sampler), against mathematics it does not share code
with: high-precision mpmath quadrature of the Klein-Nishina angular density,
the textbook closed form evaluated at 50 digits, the Thomson limit and its
Cardano inverse, the large-x asymptote, and statistical tests of sampled
histograms against quadrature bin masses."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, stats

mp.mp.dps = 40


def kn_density(mu, x):
    """Klein-Nishina rest-frame density in mu = cos(theta), up to a constant:
    r^2 (r + 1/r - sin^2 theta) with r = 1/(1 + x(1 - mu))."""
    r = 1 / (1 + x * (1 - mu))
    return r * r * (r + 1 / r - (1 - mu * mu))


def s_quadrature(x):
    x = mp.mpf(x)
    return mp.mpf(3) / 8 * mp.quad(lambda m: kn_density(m, x), [-1, 0, 1])


def s_closed_form_mp(x):
    """Textbook sigma_KN / sigma_T, at 40 significant digits."""
    x = mp.mpf(x)
    l = mp.log(1 + 2 * x)
    return mp.mpf(3) / 4 * ((1 + x) / x**3 * (2 * x * (1 + x) / (1 + 2 * x) - l) + l / (2 * x)
                            - (1 + 3 * x) / (1 + 2 * x) ** 2)


X_GRID = [1e-8, 1e-6, 1e-4, 1e-3, 5e-3, 0.02, 0.1, 0.15, 0.1999999, 0.2, 0.2000001, 0.3, 0.5, 1.0, 2.0,
          10.0, 100.0, 1e3, 1e4]


@pytest.mark.parametrize("x", X_GRID)
def test_sigma_vs_quadrature(orc, x):
    ref = s_quadrature(x)
    got = orc.sigma_ratio(x)
    assert abs(got - float(ref)) <= 1e-14 * float(ref)


@pytest.mark.parametrize("x", [1e-3, 0.05, 0.2, 1.0, 7.5, 100.0, 1e4])
def test_sigma_vs_closed_form_high_precision(orc, x):
    ref = float(s_closed_form_mp(x))
    assert abs(orc.sigma_ratio(x) - ref) <= 1e-14 * ref


def test_sigma_thomson_limit_and_series(orc):
    assert orc.sigma_ratio(0.0) == 1.0
    # s = 1 - 2x + 26/5 x^2 - 133/10 x^3 + ... (Taylor expansion of the closed form)
    for x in [1e-7, 1e-5, 1e-4]:
        taylor = 1 - 2 * x + 26 / 5 * x**2 - 133 / 10 * x**3
        assert abs(orc.sigma_ratio(x) - taylor) <= 2e-16 + 40 * x**4


def test_sigma_asymptote(orc):
    """x >> 1: s -> (3/8)(ln 2x + 1/2)/x, with relative error O(ln x / x)."""
    prev = None
    for x in [1e2, 1e3, 1e4, 1e5]:
        asym = 3 / 8 * (math.log(2 * x) + 0.5) / x
        err = abs(orc.sigma_ratio(x) / asym - 1)
        assert err < 3 * math.log(x) / x
        if prev is not None:
            assert err < prev
        prev = err


def test_sigma_monotone_and_bounded(orc):
    xs = np.logspace(-9, 5, 400)
    s = orc.sigma_ratio(xs)
    assert np.all(np.diff(s) < 0)
    assert np.all((s > 0) & (s <= 1))


def cdf_quadrature(mu, x):
    x = mp.mpf(x)
    num = mp.quad(lambda m: kn_density(m, x), [-1, mu])
    den = mp.quad(lambda m: kn_density(m, x), [-1, 0, 1])
    return num / den


@pytest.mark.parametrize("x", [1e-6, 1e-3, 0.05, 0.19, 0.2, 0.21, 1.0, 10.0, 100.0])
def test_cdf_vs_quadrature(orc, x):
    for mu in [-0.999, -0.7, -0.2, 0.0, 0.3, 0.8, 0.99, 0.99999]:
        ref = float(cdf_quadrature(mu, x))
        assert abs(orc.angle_cdf(mu, x) - ref) <= 2e-15, (mu, x)


def test_cdf_endpoints_and_monotone(orc):
    for x in [0.0, 1e-5, 0.1, 0.2, 3.0, 100.0]:
        assert orc.angle_cdf(-1.0, x) == 0.0
        assert orc.angle_cdf(1.0, x) == 1.0
        mus = np.linspace(-1, 1, 801)
        F = orc.angle_cdf(mus, x)
        assert np.all(np.diff(F) >= 0)
        assert abs(F[1] - 0.0) < 0.01 and abs(F[-2] - 1.0) < 0.2


def test_pdf_is_cdf_derivative(orc):
    for x in [1e-3, 0.1, 0.5, 20.0]:
        for mu in [-0.9, -0.1, 0.4, 0.95]:
            h = 1e-5
            fd = (orc.angle_cdf(mu + h, x) - orc.angle_cdf(mu - h, x)) / (2 * h)
            assert abs(fd - orc.angle_pdf(mu, x)) < 1e-8 * max(1.0, orc.angle_pdf(mu, x))


def cardano_thomson(u):
    """Inverse of the Thomson CDF F0 = (mu^3 + 3 mu + 4)/8 (Cardano's root)."""
    q = 4 * u - 2
    r = math.sqrt(q * q + 1)
    return math.copysign(abs(q + r) ** (1 / 3), q + r) + math.copysign(abs(q - r) ** (1 / 3), q - r)


def test_icdf_thomson_limit_is_cardano(orc):
    for u in np.linspace(0.0, 1.0, 41):
        mu0 = cardano_thomson(u)
        assert abs(orc.angle_icdf(u, 1e-12) - mu0) < 1e-11
        assert abs(orc.angle_icdf(u, 0.0) - mu0) < 1e-13


@pytest.mark.parametrize("x", [1e-4, 1e-2, 0.19, 0.25, 1.0, 100.0])
def test_icdf_roundtrip(orc, x):
    rng = np.random.default_rng(3)
    for u in np.concatenate([[0.0, 1e-12, 0.5, 1 - 2**-53], rng.random(60)]):
        mu = orc.angle_icdf(u, x)
        assert -1.0 <= mu <= 1.0
        assert abs(orc.angle_cdf(mu, x) - u) <= 1.2e-15 + 4e-16 * orc.angle_pdf(mu, x)


@pytest.mark.parametrize("x", [1e-4, 1e-2, 1.0, 100.0])
def test_sampled_histogram_matches_kn(orc, x):
    """Sample mu with uniform u through the inverse CDF; compare the histogram
    (64 bins) with bin masses from scipy quadrature of the Klein-Nishina
    density (chi-square) and the empirical CDF with quadrature (KS)."""
    n = 1 << 15
    rng = np.random.default_rng(11)
    u = rng.random(n)
    mu, r = orc.sample_plain(np.full(n, x), u)
    # r = 1/(1 + x v) from the sampler's v = 1 - mu; mu itself is v rounded once
    assert np.allclose(r, 1 / (1 + x * (1 - mu)), rtol=4e-16 * (2 + 2 * x), atol=0)
    edges = np.linspace(-1, 1, 65)
    dens = lambda m: 1 / (1 + x * (1 - m)) ** 2 * (1 / (1 + x * (1 - m)) + 1 + x * (1 - m) - (1 - m * m))
    total = integrate.quad(dens, -1, 1, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
    mass = np.array([integrate.quad(dens, a, b, epsabs=1e-14, epsrel=1e-13)[0] for a, b in zip(edges[:-1], edges[1:])])
    mass /= total
    h, _ = np.histogram(mu, bins=edges)
    e = n * mass
    keep = e > 5
    chi2 = ((h[keep] - e[keep]) ** 2 / e[keep]).sum()
    dof = keep.sum() - 1
    assert stats.chi2.sf(chi2, dof) > 1e-3

    def cdf(m):
        return integrate.quad(dens, -1, m, epsabs=1e-14, epsrel=1e-13, limit=200)[0] / total

    xs = np.sort(mu[:4096])
    Fq = np.array([cdf(m) for m in xs])
    emp_hi = np.arange(1, xs.size + 1) / xs.size
    emp_lo = np.arange(0, xs.size) / xs.size
    D = max(np.max(emp_hi - Fq), np.max(Fq - emp_lo))
    assert D < 1.63 / math.sqrt(xs.size)  # 1% level of the KS distribution


@pytest.mark.parametrize("x", [1e-3, 0.1, 0.3, 5.0, 100.0])
def test_icdf_v_relative_accuracy_forward(orc, x):
    """Forward scatters: v = 1 - mu is solved with relative precision, so that
    sin(theta) = sqrt(v (2 - v)) stays accurate as mu -> 1.  Reference: the
    upper tail int_{1-v}^{1} f = (1 - u) int f solved in mpmath."""
    X = mp.mpf(x)
    dens = lambda m: kn_density(m, X)
    Z = mp.quad(dens, [-1, 0, 1])
    for one_minus_u in [1e-3, 1e-7, 1e-11, 2.0**-50]:
        u = 1.0 - one_minus_u
        tail_target = (1 - mp.mpf(u)) * Z
        v_ref = mp.findroot(lambda v: mp.quad(dens, [1 - v, 1]) - tail_target, mp.mpf(one_minus_u) * Z / dens(1))
        v = orc.angle_icdf_v(u, x)
        assert abs(v - float(v_ref)) <= 4e-15 * float(v_ref), (x, one_minus_u, v, float(v_ref))
