"""Pins of the oracle's product manifold S^1_Fourier(R) x S^2(a) in R^9 (Sec. 4,
Example 3): the closest point against a brute-force search over the curve
and the sphere's normalisation, the curve's curvature against finite
differences, the source against the intrinsic Laplace-Beltrami operator of
the product by finite differences in (phi, theta, psi), and the
constant-solution invariant of the estimator."""
import math

import numpy as np
import pytest

from paper_2606_21883_amd import inputs

R, A = 1.0, 0.65


def _curve(phi):
    return inputs.product_point(np.atleast_1d(phi), np.zeros((np.size(phi), 3)), R, A)[:, :6]


def test_cp_against_brute_force(orc):
    prob = inputs.product_problem()
    P = orc.Problem(prob)
    Y = inputs.product_points(20, seed=4)
    rng = np.random.default_rng(5)
    grid = np.linspace(0.0, 2 * np.pi, 400001)[:-1]
    C = _curve(grid)
    for y in Y:
        assert np.max(np.abs(orc.cp(P, y) - y)) < 1e-14
        x = y + 0.3 * rng.standard_normal(9) / 3.0
        yc = orc.cp(P, x)
        i = int(np.argmin(((C - x[:6]) ** 2).sum(1)))
        # refine the brute-force minimiser on a fine local grid
        loc = np.linspace(grid[i] - 2e-5, grid[i] + 2e-5, 4001)
        j = int(np.argmin(((_curve(loc) - x[:6]) ** 2).sum(1)))
        assert np.max(np.abs(yc[:6] - _curve(loc[j])[0])) < 1e-8
        assert np.allclose(yc[6:], A * x[6:] / np.linalg.norm(x[6:]), rtol=0, atol=1e-15)


def test_curve_curvature_and_radius(orc):
    h = 1e-3
    for phi in np.linspace(0, 2 * np.pi, 9):
        c0, cp, cm = _curve(phi)[0], _curve(phi + h)[0], _curve(phi - h)[0]
        d1 = (cp - cm) / (2 * h)
        d2 = (cp - 2 * c0 + cm) / (h * h)
        # curvature of a space curve: |d1 x d2| / |d1|^3 in any dimension
        k = math.sqrt(max(0.0, (d1 @ d1) * (d2 @ d2) - (d1 @ d2) ** 2)) / (d1 @ d1) ** 1.5
        assert k == pytest.approx(math.sqrt(14) / (3 * R), rel=1e-5)
    P = orc.Problem(inputs.product_problem())
    y = inputs.product_points(1, seed=2)[0]
    assert orc.radius(P, y) == pytest.approx(0.95 * 1.2 / (1 + max(math.sqrt(14) / 3, 1 / A)), rel=1e-15)


def _intrinsic_f(prob, phi, th, ps):
    """-Lap_M u + sigma u with Lap_M = (1/(3 R^2)) d^2/dphi^2 + Lap_{S^2(a)}, the
    latter in spherical angles, all by central differences."""
    c0, c1, c2 = prob["f"]["coef"]

    def u(p, t, s):
        w1, w2 = math.sin(t) * math.cos(s), math.sin(t) * math.sin(s)
        return c0 * math.cos(p) * w1 + c1 * math.sin(2 * p) * w2 + c2 * math.cos(3 * p) * (w1 * w1 - w2 * w2)

    h = 1e-4
    upp = (u(phi + h, th, ps) - 2 * u(phi, th, ps) + u(phi - h, th, ps)) / (h * h)
    ut = lambda t: (u(phi, t + h, ps) - u(phi, t - h, ps)) / (2 * h)
    uth = (math.sin(th + h / 2) * (u(phi, th + h, ps) - u(phi, th, ps)) / h
           - math.sin(th - h / 2) * (u(phi, th, ps) - u(phi, th - h, ps)) / h) / h
    uss = (u(phi, th, ps + h) - 2 * u(phi, th, ps) + u(phi, th, ps - h)) / (h * h)
    lap = upp / (3 * R * R) + (uth / math.sin(th) + uss / math.sin(th) ** 2) / (A * A)
    del ut
    return -lap + prob["sigma"] * u(phi, th, ps)


def test_source_against_intrinsic_laplacian(orc):
    prob = inputs.product_problem(sigma=1.0)
    P = orc.Problem(prob)
    rng = np.random.default_rng(7)
    for _ in range(12):
        phi, th, ps = rng.uniform(0, 2 * np.pi), rng.uniform(0.3, 2.8), rng.uniform(0, 2 * np.pi)
        w = np.array([[math.sin(th) * math.cos(ps), math.sin(th) * math.sin(ps), math.cos(th)]])
        y = inputs.product_point([phi], w, R, A)[0]
        assert orc.source(P, y) == pytest.approx(_intrinsic_f(prob, phi, th, ps), rel=1e-5, abs=1e-5)
        # the closed form u the source is built from
        assert inputs.exact_u(prob, y[None])[0] == pytest.approx(
            prob["f"]["coef"][0] * math.cos(phi) * w[0, 0] + prob["f"]["coef"][1] * math.sin(2 * phi) * w[0, 1]
            + prob["f"]["coef"][2] * math.cos(3 * phi) * (w[0, 0] ** 2 - w[0, 1] ** 2), rel=1e-13, abs=1e-15)


def test_constant_solution_on_the_product(orc):
    C = -0.4
    prob = dict(inputs.product_problem(), f=dict(kind="const", coef=[C]), tau_w=1e-3)
    Q = inputs.product_points(4, seed=3)
    res = orc.solve(prob, Q, 16, seed=8)
    r = 0.95 * 1.2 / (1.0 + 1.0 / A)
    c = orc.c_sigma_r(9, 1.0, r)
    K = int(res["walk_K"][0, 0])
    assert np.all(res["walk_K"] == K) and c ** K < 1e-3 <= c ** (K - 1)
    np.testing.assert_allclose(res["walk_S"], C * (1.0 - c ** K), rtol=1e-12)


def test_product_rejects_other_settings(orc):
    Q = inputs.product_points(2, seed=3)
    for bad in (dict(compensation="exact"), dict(n=8)):
        with pytest.raises(ValueError):
            orc.solve(dict(inputs.product_problem(), **bad), Q if "n" not in bad else Q[:, :8], 2, seed=1)
