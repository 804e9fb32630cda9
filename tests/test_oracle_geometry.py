"""Pins of the oracle's closest-point maps, boundary distance and sources.

- cp on the torus against brute-force minimisation over the parametrisation.
- delta_Gamma on the cap against brute-force distance to the normal disk
  (eq. extended_boundary_disk, eq. delta_Gamma_general) and its reduction to
  |y_3| near the cut.
- f and the exact compensation m (eq. mismatch_definition) together: for any x
  in the tube, f(cp x) + m(x) must equal -Lap(Eu)(x) + sigma Eu(x), computed
  here by a central finite-difference ambient Laplacian of the closest-point
  extension Eu = u o cp of the closed-form solution.  On M this is the identity
  Lap_Omega u = Lap(Eu) (eq. LB_cp_identity), so it pins f itself; off M it
  pins m.
"""
import math

import numpy as np
import pytest
from scipy import optimize

from paper_2606_21883_amd import inputs


def torus_xyz(R, a, phi, psi):
    return np.array([(R + a * math.cos(psi)) * math.cos(phi), (R + a * math.cos(psi)) * math.sin(phi),
                     a * math.sin(psi)])


def test_torus_cp_is_the_nearest_point(orc):
    prob = inputs.torus_problem()
    rng = np.random.default_rng(3)
    R, a = 1.0, 0.3
    P = orc.Problem(prob)
    for _ in range(40):
        base = torus_xyz(R, a, rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi))
        x = base + rng.uniform(-0.25, 0.25, 3)
        y = orc.cp(P, x)
        # brute force: best grid point, then a local polish of the parametrised distance
        ph = np.linspace(0, 2 * np.pi, 181)
        ps = np.linspace(0, 2 * np.pi, 181)
        PH, PS = np.meshgrid(ph, ps)
        pts = np.stack([(R + a * np.cos(PS)) * np.cos(PH), (R + a * np.cos(PS)) * np.sin(PH), a * np.sin(PS)], -1)
        d = np.linalg.norm(pts - x, axis=-1)
        i = np.unravel_index(np.argmin(d), d.shape)
        res = optimize.minimize(lambda v: np.sum((torus_xyz(R, a, v[0], v[1]) - x) ** 2),
                                [PH[i], PS[i]], method="Nelder-Mead",
                                options=dict(xatol=1e-12, fatol=1e-20, maxiter=4000))
        yb = torus_xyz(R, a, *res.x)
        assert np.linalg.norm(y - yb) < 1e-7
        assert np.linalg.norm(y - x) <= np.min(d) + 1e-12


def test_cap_delta_gamma_brute_force(orc):
    prob = inputs.cap_problem()
    P = orc.Problem(prob)
    rng = np.random.default_rng(4)
    ell = 1.2 / 2.0
    ys = inputs.cap_uniform(300, 3, 0.0, seed=9)
    for y in ys:
        d = orc.delta_gamma(P, y)
        rho = math.hypot(y[0], y[1])
        yg = np.array([y[0] / rho, y[1] / rho, 0.0])
        # normal disk of S^2 at y_Gamma: y_Gamma + xi * y_Gamma, |xi| <= ell
        xi = np.linspace(-ell, ell, 200001)
        seg = yg[None, :] * (1.0 + xi[:, None])
        brute = np.min(np.linalg.norm(seg - y, axis=1))
        assert d == pytest.approx(brute, abs=2e-6)
        if 1.0 - rho <= ell:
            assert d == pytest.approx(abs(y[2]), rel=1e-12, abs=1e-15)


def test_radius_rule_values(orc):
    # r = theta c_kappa / (1 + kappa) with kappa = 1 on the unit sphere, 1/a on the torus
    s = inputs.sphere_problem()
    assert orc.radius(s, np.array([1.0, 0, 0])) == pytest.approx(0.95 * 1.2 / 2, rel=1e-15)
    t = inputs.torus_problem()
    y = torus_xyz(1.0, 0.3, 0.3, 1.1)
    assert orc.radius(t, y) == pytest.approx(0.95 * 1.2 / (1 + 1 / 0.3), rel=1e-15)
    c = inputs.cap_problem()
    y = np.array([math.cos(0.1), 0.0, math.sin(0.1)])
    assert orc.radius(c, y) == pytest.approx(0.95 * math.sin(0.1), rel=1e-12)


# --------------------------------------------------------------------------
# f + m against a finite-difference Laplacian of the extension
# --------------------------------------------------------------------------


def cp_test(prob, x):
    """Closest point written out here (independent of the oracle)."""
    if prob["manifold"] in ("sphere", "sphere_cap"):
        return prob["p"][0] * x / np.linalg.norm(x)
    if prob["manifold"] == "torus":
        R, a = prob["p"][:2]
        rho = math.hypot(x[0], x[1])
        C = np.array([R * x[0] / rho, R * x[1] / rho, 0.0])
        d = x - C
        return C + a * d / np.linalg.norm(d)
    raise ValueError


def Eu(prob, x):
    return inputs.exact_u(prob, cp_test(prob, x)[None, :])[0]


def fd_operator(prob, x, h=2e-3):
    n = len(x)
    u0 = Eu(prob, x)
    lap = 0.0
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        # fourth-order central second difference
        lap += (-Eu(prob, x + 2 * e) + 16 * Eu(prob, x + e) - 30 * u0 + 16 * Eu(prob, x - e)
                - Eu(prob, x - 2 * e)) / (12 * h * h)
    return -lap + prob["sigma"] * u0


def points_near(prob, rng, m, spread):
    if prob["manifold"] == "torus":
        pts = []
        for _ in range(m):
            pts.append(torus_xyz(1.0, 0.3, rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi)))
        base = np.array(pts)
    else:
        base = inputs.sphere_uniform(m, prob["n"], seed=int(rng.integers(1 << 30)))
    off = rng.uniform(-spread, spread, base.shape)
    return base, base + off


FAMILIES = [
    inputs.sphere_problem(),
    inputs.cap_problem(),
    inputs.circle_problem(),
    inputs.hypersphere_problem(10),
    inputs.problem(manifold="sphere", n=3, p=[1.0], sigma=1.0,
                   f=dict(kind="legendre", coef=[0.0, 3.0, 0.0, 0.2 * 13.0, 0.0, 0.1 * 31.0])),
    inputs.problem(manifold="sphere", n=3, p=[1.0], sigma=0.7, f=dict(kind="const", coef=[2.1])),
    inputs.problem(manifold="sphere", n=2, p=[1.7], sigma=1.3,
                   f=dict(kind="circle_mode", idx=[2], coef=[0.4, -1.1])),
    inputs.torus_problem(),
]


@pytest.mark.parametrize("prob", FAMILIES, ids=lambda p: p["manifold"] + ":" + p["f"]["kind"] + str(p["n"]))
def test_source_plus_compensation_is_ambient_operator(orc, prob):
    rng = np.random.default_rng(17)
    P = orc.Problem(prob)
    spread = 0.15 if prob["manifold"] == "torus" else 0.3
    on, off = points_near(prob, rng, 12, spread)
    scale = max(1.0, np.max(np.abs(inputs.exact_u(prob, on))) * (prob["sigma"] + 2 * prob["n"] + 12))
    for x in list(on) + list(off):
        if prob["manifold"] == "sphere" and prob["p"][0] != 1.0:
            x = x * prob["p"][0]
        got = orc.source(P, x)
        ref = fd_operator(prob, x)
        assert got == pytest.approx(ref, abs=2e-6 * scale), (x, got, ref)


def test_compensation_none_drops_m(orc):
    prob = dict(inputs.sphere_problem(), compensation="none")
    x = np.array([0.9, 0.5, 0.3])
    y = x / np.linalg.norm(x)
    assert orc.source(prob, x) == pytest.approx(8.0 * y[0] * y[1], rel=1e-15)
