"""Pins of the screening factor c_{sigma,r}, the weight omega and the radial law
of the normalised Green density, against the paper's Bessel-function forms
evaluated by scipy / mpmath, quadrature of the paper's Green function, closed
forms for n = 3, the Laplace limit, and moment identities that follow from the
local representation (Lemma 2.1) for every n.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special


def c_bessel(n, sigma, r):
    """eq. def_c_sigma_r with mpmath Bessel I (any order)."""
    mp.mp.dps = 40
    nu = mp.mpf(n - 2) / 2
    X = mp.sqrt(sigma) * r
    return float(X ** nu / (2 ** nu * mp.gamma(nu + 1) * mp.besseli(nu, X)))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 10, 100, 1000])
@pytest.mark.parametrize("sigma,r", [(1.0, 0.57), (2.0, 0.57), (0.5, 0.1), (1.0, 0.2632), (4.0, 0.9)])
def test_c_matches_bessel_form(orc, n, sigma, r):
    c = orc.c_sigma_r(n, sigma, r)
    assert c == pytest.approx(c_bessel(n, sigma, r), rel=2e-15, abs=0)
    om = orc.omega(n, sigma, r)
    assert om == pytest.approx((1.0 - c_bessel(n, sigma, r)) / sigma, rel=1e-12)


def test_c_closed_forms_n2_n3(orc):
    for X in [0.05, 0.5, 0.806, 1.7]:
        lam = 1.3
        r = X / lam
        # n = 3: lambda r / sinh(lambda r); n = 2: 1 / I_0(lambda r)  (Remark after Lemma 2.1)
        assert orc.c_sigma_r(3, lam * lam, r) == pytest.approx(X / math.sinh(X), rel=1e-15)
        assert orc.c_sigma_r(2, lam * lam, r) == pytest.approx(1.0 / special.i0(X), rel=1e-15)


@pytest.mark.parametrize("n", [2, 3, 10, 1000])
def test_c_bound_lemma31(orc, n):
    for sigma, r in [(1.0, 0.57), (2000.0, 0.3), (0.01, 0.1)]:
        c = orc.c_sigma_r(n, sigma, r)
        assert 0.0 < c <= 1.0 / (1.0 + sigma * r * r / (2 * n))


def test_deterministic_walk_lengths_match_config_table(orc):
    # With constant r the closed-manifold walk length is the first K with c^K < tau_W.
    cases = [(2, 1.0, 0.57, 232), (3, 2.0, 0.57, 174), (100, 1.0, 0.57, 11340),
             (1000, 1.0, 0.57, 113393), (3, 1.0, 0.95 * 1.2 / (1 + 1 / 0.3), 1601)]
    for n, sigma, r, K in cases:
        c = c_bessel(n, sigma, r)
        assert math.ceil(math.log(1e-8) / math.log(c)) == K
        assert orc.c_sigma_r(n, sigma, r) == pytest.approx(c, rel=1e-15)


# --------------------------------------------------------------------------
# Green function of the Remark after Lemma 2.1 and its radial law
# --------------------------------------------------------------------------


def green_scipy(n, lam, r, rho):
    nu = (n - 2) / 2.0
    return (2 * np.pi) ** (-n / 2) * (lam / rho) ** nu * (
        special.kv(nu, lam * rho) - special.kv(nu, lam * r) / special.iv(nu, lam * r) * special.iv(nu, lam * rho))


def sphere_area(n):
    return 2 * math.pi ** (n / 2) / math.gamma(n / 2)


def radial_mass(n, lam, r, t):
    """|S^{n-1}| int_0^t rho^{n-1} G(rho) d rho by adaptive quadrature."""
    f = lambda rho: rho ** (n - 1) * green_scipy(n, lam, r, rho)
    val, err = integrate.quad(f, 0.0, t, limit=200, epsabs=0, epsrel=1e-13)
    return sphere_area(n) * val


@pytest.mark.parametrize("n", [2, 3, 4, 5, 10])
def test_omega_is_integral_of_green(orc, n):
    for lam, r in [(1.0, 0.57), (math.sqrt(2), 0.57), (math.sqrt(0.5), 0.3)]:
        om = orc.omega(n, lam * lam, r)
        assert om == pytest.approx(radial_mass(n, lam, r, r), rel=1e-9)


def test_green_n3_matches_closed_form():
    lam, r = 1.4, 0.57
    for rho in [0.01, 0.2, 0.5]:
        closed = math.sinh(lam * (r - rho)) / (4 * math.pi * rho * math.sinh(lam * r))
        assert green_scipy(3, lam, r, rho) == pytest.approx(closed, rel=1e-12)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 10])
@pytest.mark.parametrize("lam,r", [(1.0, 0.57), (math.sqrt(2), 0.57), (1.5, 1.0)])
def test_radial_cdf_matches_quadrature(orc, n, lam, r):
    X = lam * r
    tot = radial_mass(n, lam, r, r)
    for s in [0.05, 0.3, 0.5, 0.8, 0.97]:
        F = orc.radial_cdf(n, X, s)
        assert F == pytest.approx(radial_mass(n, lam, r, s * r) / tot, rel=2e-9, abs=1e-13)
        # density is the derivative of the CDF
        h = 1e-6
        fd = (orc.radial_cdf(n, X, s + h) - orc.radial_cdf(n, X, s - h)) / (2 * h)
        assert orc.radial_pdf(n, X, s) == pytest.approx(fd, rel=1e-6)


def test_radial_cdf_n3_closed_form(orc):
    for X in [0.2632, 0.57, 0.806, 1.5]:
        for s in np.linspace(0.01, 0.99, 23):
            ex = (math.sinh(X) - math.sinh(X * (1 - s)) - X * s * math.cosh(X * (1 - s))) / (math.sinh(X) - X)
            assert orc.radial_cdf(3, X, s) == pytest.approx(ex, rel=1e-11, abs=1e-15)


@pytest.mark.parametrize("n", [3, 4, 10, 100, 1000])
def test_radial_cdf_laplace_limit(orc, n):
    X = 1e-4
    for s in [0.1, 0.5, 0.9]:
        ex = (n * s * s - 2 * s ** n) / (n - 2)
        assert orc.radial_cdf(n, X, s) == pytest.approx(ex, rel=1e-7)


def test_radial_cdf_endpoints_and_monotone(orc):
    for n in [2, 3, 7, 100, 1000]:
        X = 0.7
        s = np.linspace(0, 1, 401)
        F = np.array([orc.radial_cdf(n, X, v) for v in s])
        assert F[0] == 0.0 and F[-1] == 1.0
        assert np.all(np.diff(F) >= 0)


@pytest.mark.parametrize("n,X", [(2, 0.8), (3, 0.8), (5, 0.8), (100, 0.8), (1000, 0.8), (1001, 12.975)])
def test_radial_inverse_roundtrip(orc, n, X):
    for u in [1e-9, 0.01, 0.3, 0.5, 0.77, 0.999, 1 - 1e-9]:
        s = orc.radial_inv(n, X, u)
        assert orc.radial_cdf(n, X, s) == pytest.approx(u, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("n,sigma,r", [(n, s, r) for n in (2, 3, 10, 100, 1000)
                                       for s, r in ((1.0, 0.57), (2.0, 0.57), (0.5, 0.3))]
                         # the dumbbell's regime: sigma = 2 (n - 1), r = 0.95 * 1.2 / (1 + 2.9294)
                         + [(11, 20.0, 0.290121), (101, 200.0, 0.290121), (1001, 2000.0, 0.290121)])
def test_radial_moments_from_local_representation(orc, n, sigma, r):
    """Lemma 2.1 applied to v = |z-y|^{2m} (for which -Lap v + sigma v is explicit)
    fixes every even moment of |Z - y| under the Green density:
        0 = c r^{2m} + omega (-2m(2m+n-2) E[t^{2m-2}] + sigma E[t^{2m}])."""
    X = math.sqrt(sigma) * r
    mp.mp.dps = 50
    nu = mp.mpf(n - 2) / 2
    Xm = mp.sqrt(mp.mpf(sigma)) * mp.mpf(r)
    c = Xm ** nu / (2 ** nu * mp.gamma(nu + 1) * mp.besseli(nu, Xm))
    om = (1 - c) / sigma
    Et_prev = mp.mpf(1)
    for m in (1, 2, 3):
        expect = (2 * m * (2 * m + n - 2) * Et_prev - c * mp.mpf(r) ** (2 * m) / om) / sigma
        # E[s^{2m}] = int_0^1 s^{2m} dF = 1 - 2m int_0^1 s^{2m-1} F(s) ds
        val, _ = integrate.quad(lambda s: s ** (2 * m - 1) * orc.radial_cdf(n, X, s), 0, 1,
                                limit=200, epsabs=1e-15, epsrel=1e-12)
        got = (1.0 - 2 * m * val) * r ** (2 * m)
        assert got == pytest.approx(float(expect), rel=1e-9)
        Et_prev = expect


def test_radial_sampling_distribution(orc):
    from scipy import stats
    n, X = 3, math.sqrt(2) * 0.57
    rng = np.random.default_rng(5)
    s = np.array([orc.radial_inv(n, X, u) for u in rng.uniform(size=4000)])
    cdf = np.vectorize(lambda v: orc.radial_cdf(n, X, v))
    assert stats.kstest(s, cdf).pvalue > 1e-4


def test_radial_domain_bound(orc):
    # 0.8 sqrt((nu+1)(nu+5)) stays below the first zero of J_nu
    for n in [2, 3, 4, 6, 10, 100, 1000]:
        nu = (n - 2) / 2
        if float(nu).is_integer():
            j1 = special.jn_zeros(int(nu), 1)[0]
        else:
            j1 = float(mp.besseljzero(nu, 1))
        assert orc.radial_xmax(n) < 0.9 * j1
