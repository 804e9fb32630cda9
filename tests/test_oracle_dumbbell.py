"""Pins of the oracle's implicit dumbbell (Sec. 4, Example 2): the closest
point against a brute-force search over the paper's own profile R(xs), the
principal curvatures against finite differences of the graph r = R(xs) and
the closed forms of the prolate spheroid, the source f = -Lap_M u + sigma u
against the spherical-harmonic closed form (a = 0, kc = 1 is the unit sphere)
and against the intrinsic Laplace-Beltrami operator of a hypersurface of
revolution at every dimension used, and the constant-solution invariant of
the estimator."""
import math

import numpy as np
import pytest
from scipy import optimize

from paper_2606_21883_amd import inputs

ALPHA, KC = 0.35, 1.2


def _R(z, a=ALPHA, kc=KC):
    return inputs.dumbbell_profile_radius(z, a, kc)


def _brute_cp(x, a=ALPHA, kc=KC):
    """Nearest point of M by brute force on the paper's profile R(xs): a dense
    grid in xs, then a bounded scalar refinement of the planar distance."""
    xh, xs = x[:-1], x[-1]
    rho = np.linalg.norm(xh)
    z = np.linspace(-kc, kc, 200001)
    d = (rho - _R(z, a, kc)) ** 2 + (xs - z) ** 2
    i = int(np.argmin(d))
    lo, hi = z[max(0, i - 2)], z[min(len(z) - 1, i + 2)]
    res = optimize.minimize_scalar(lambda t: (rho - _R(t, a, kc)) ** 2 + (xs - t) ** 2, bounds=(lo, hi),
                                   method="bounded", options={"xatol": 1e-14})
    zb = res.x
    return np.concatenate([xh / rho * _R(zb, a, kc), [zb]])


@pytest.mark.parametrize("n", [3, 4, 11])
def test_cp_against_brute_force(orc, n):
    prob = inputs.dumbbell_problem(n)
    P = orc.Problem(prob)
    Y = inputs.dumbbell_points(12, n, seed=4, phi_margin=0.2)
    rng = np.random.default_rng(5)
    for y in Y:
        # points of M are fixed points
        assert np.max(np.abs(orc.cp(P, y) - y)) < 1e-13
        # off M, inside the reach (within 0.25 of M; the reach is 1/2.93)
        x = y + rng.uniform(-0.25, 0.25) * rng.standard_normal(n) / math.sqrt(n)
        yc = orc.cp(P, x)
        yb = _brute_cp(x)
        assert np.max(np.abs(yc - yb)) < 1e-7, (x, yc, yb)
        # the oracle's point is a stationary point of the distance: x - y is
        # normal to M, so it has no component along the profile tangent
        assert abs(np.linalg.norm(yc[:-1]) - _R(yc[-1])) < 1e-12


def test_curvatures_against_the_graph_of_R(orc):
    """k1 = -R''/(1+R'^2)^{3/2} and k2 = 1/(R sqrt(1+R'^2)) for r = R(xs),
    by central differences, away from the poles."""
    h = 1e-3
    for xs in np.linspace(-1.1, 1.1, 23):
        # fourth-order central differences
        R0 = _R(xs)
        Rp, Rm, Rpp, Rmm = _R(xs + h), _R(xs - h), _R(xs + 2 * h), _R(xs - 2 * h)
        d1 = (-Rpp + 8 * Rp - 8 * Rm + Rmm) / (12 * h)
        d2 = (-Rpp + 16 * Rp - 30 * R0 + 16 * Rm - Rmm) / (12 * h * h)
        k1 = -d2 / (1 + d1 * d1) ** 1.5
        k2 = 1.0 / (R0 * math.sqrt(1 + d1 * d1))
        phi = math.acos(xs / KC)
        o1, o2 = orc.db_curvatures(ALPHA, KC, phi)
        assert o1 == pytest.approx(k1, rel=1e-6, abs=1e-7)
        assert o2 == pytest.approx(k2, rel=1e-8)


def test_curvatures_closed_forms(orc):
    for t in np.linspace(0.0, math.pi, 13):
        # a = 0, kc = 1: the unit sphere
        assert orc.db_curvatures(0.0, 1.0, t) == pytest.approx((1.0, 1.0), rel=1e-14)
        # a = 0, kc = 2: the prolate spheroid of semi-axes 1 (radial) and 2
        q = math.cos(t) ** 2 + 4.0 * math.sin(t) ** 2
        k1, k2 = orc.db_curvatures(0.0, 2.0, t)
        assert k1 == pytest.approx(2.0 / q ** 1.5, rel=1e-13)
        assert k2 == pytest.approx(2.0 / math.sqrt(q), rel=1e-13)
    # the bound used by the radius rule
    ks = [max(abs(v) for v in orc.db_curvatures(ALPHA, KC, t)) for t in np.linspace(0, math.pi, 20001)]
    assert max(ks) == pytest.approx(inputs.dumbbell_kappa_max(), rel=1e-6)


@pytest.mark.parametrize("n", [4, 11, 1001])
def test_source_on_the_unit_sphere_case(orc, n):
    """a = 0, kc = 1 makes M the unit sphere S^{n-1}: z and 1.xh are degree-1
    harmonics (eigenvalue n-1), xh^T A xh with tr A = 0 is degree 2
    (eigenvalue 2n), and z^2 = (z^2 - 1/n) + 1/n."""
    prob = inputs.dumbbell_problem(n, alpha=0.0, kc=1.0)
    P = orc.Problem(prob)
    sg = prob["sigma"]
    c0, c1, b1, b2 = prob["f"]["coef"]
    A = prob["f"]["values"]
    Y = inputs.dumbbell_points(6, n, alpha=0.0, kc=1.0, seed=7)
    for y in Y:
        xh, z = y[:-1], y[-1]
        f = (c0 * (n - 1 + sg) * z + c1 * ((2 * n + sg) * (z * z - 1.0 / n) + sg / n)
             + b1 * (n - 1 + sg) * xh.sum() / math.sqrt(n - 1) + b2 * (2 * n + sg) * (xh * xh * A).sum())
        assert orc.source(P, y) == pytest.approx(f, rel=1e-11, abs=1e-10)


def _intrinsic_f(prob, y):
    """-Lap_M u + sigma u by the intrinsic operator of a hypersurface of
    revolution with cross-sections S^{n-2} of radius r(t):
      Lap_M u = (1/(r^{n-2} L)) d/dt (r^{n-2}/L du/dt) + Lap_{S^{n-2}} u / r^2,
    profile (r, z)(t) from the paper's R with xs = kc cos t, derivatives by
    central differences; h1 = 1.e/sqrt(n-1) and h2 = e^T A e are harmonics of
    degree 1 and 2 on S^{n-2} (eigenvalues n-2 and 2(n-1))."""
    n = prob["n"]
    a, kc = prob["p"]
    c0, c1, b1, b2 = prob["f"]["coef"]
    A = prob["f"]["values"]
    xh, xs = y[:-1], y[-1]
    e = xh / np.linalg.norm(xh)
    h1 = e.sum() / math.sqrt(n - 1)
    h2 = (A * e * e).sum()
    t0 = math.acos(xs / kc)

    def rz(t):
        z = kc * math.cos(t)
        return float(_R(z, a, kc)), z

    def radial(g, t, h=1e-4):
        # (1/L) [(n-2) (r'/r) G + G'] with G = g'/L
        def G(tt):
            r1 = (rz(tt + h)[0] - rz(tt - h)[0]) / (2 * h)
            z1 = (rz(tt + h)[1] - rz(tt - h)[1]) / (2 * h)
            L = math.hypot(r1, z1)
            return (g(tt + h) - g(tt - h)) / (2 * h) / L, L, r1
        Gc, L, r1 = G(t)
        Gp = (G(t + h)[0] - G(t - h)[0]) / (2 * h)
        r = rz(t)[0]
        return ((n - 2) * (r1 / r) * Gc + Gp) / L

    r0, z0 = rz(t0)
    lap = (c0 * radial(lambda t: rz(t)[1], t0) + c1 * radial(lambda t: rz(t)[1] ** 2, t0)
           + b1 * h1 * radial(lambda t: rz(t)[0], t0) + b2 * h2 * radial(lambda t: rz(t)[0] ** 2, t0)
           - (b1 * h1 * r0 * (n - 2) + b2 * h2 * r0 * r0 * 2 * (n - 1)) / (r0 * r0))
    u = c0 * z0 + c1 * z0 * z0 + b1 * r0 * h1 + b2 * r0 * r0 * h2
    return -lap + prob["sigma"] * u


@pytest.mark.parametrize("n", [3, 4, 11, 1001])
def test_source_against_intrinsic_laplacian(orc, n):
    prob = inputs.dumbbell_problem(n)
    P = orc.Problem(prob)
    Y = inputs.dumbbell_points(8, n, seed=9, phi_margin=0.3)
    for y in Y:
        fi = _intrinsic_f(prob, y)
        assert orc.source(P, y) == pytest.approx(fi, rel=2e-5, abs=1e-4 * (1 + abs(fi) / 100)), y[-1]


def test_exact_u_matches_the_source_family(orc):
    """sigma u = f + Lap_M u: the closed form u used for scoring is the u the
    source was built from (checked on the sphere case, where Lap_M u is known)."""
    n = 11
    prob = inputs.dumbbell_problem(n, alpha=0.0, kc=1.0)
    y = inputs.dumbbell_points(3, n, alpha=0.0, kc=1.0, seed=2)
    u = inputs.exact_u(prob, y)
    c0, c1, b1, b2 = prob["f"]["coef"]
    A = prob["f"]["values"]
    lap = -((n - 1) * (c0 * y[:, -1] + b1 * y[:, :-1].sum(1) / math.sqrt(n - 1))
            + 2 * n * (c1 * (y[:, -1] ** 2 - 1.0 / n) + b2 * (y[:, :-1] ** 2 * A).sum(1)))
    f = np.array([orc.source(orc.Problem(prob), q) for q in y])
    np.testing.assert_allclose(prob["sigma"] * u, f + lap, rtol=1e-11, atol=1e-10)


def test_constant_solution_on_the_dumbbell(orc):
    """f = sigma C gives S = C (1 - W_K) on every walk, with the constant radius
    of the curvature bound and K = the first k with c^k < tau_W."""
    n = 11
    C = 0.7
    prob = dict(inputs.dumbbell_problem(n), f=dict(kind="const", coef=[2.0 * (n - 1) * C]), tau_w=1e-4)
    Q = inputs.dumbbell_points(4, n, seed=3)
    res = orc.solve(prob, Q, 16, seed=8)
    r = 0.95 * 1.2 / (1.0 + inputs.dumbbell_kappa_max())
    c = orc.c_sigma_r(n, prob["sigma"], r)
    K = int(res["walk_K"][0, 0])
    assert np.all(res["walk_K"] == K) and c ** K < 1e-4 <= c ** (K - 1)
    np.testing.assert_allclose(res["walk_S"], C * (1.0 - c ** K), rtol=1e-12)


def test_dumbbell_rejects_other_rules(orc):
    n = 11
    Q = inputs.dumbbell_points(2, n, seed=3)
    for bad in (dict(radius_rule="curvature"), dict(compensation="exact"), dict(kappa_bound=-1.0)):
        with pytest.raises(ValueError):
            orc.solve(dict(inputs.dumbbell_problem(n), **bad), Q, 2, seed=1)
