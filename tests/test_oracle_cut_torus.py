"""Pins of the oracle's torus with a planar cut (Sec. 4, Example 1) and of the
second-order compensation (the subsection on approximating the compensation
term): the boundary distance against a brute-force distance to the normal
segment, the stop test on the far side of the cut, the source against the
intrinsic Laplace-Beltrami operator of the torus by finite differences, the
exact compensation against the ambient finite-difference Laplacian of the
closest-point extension (its definition), the Fourier-sine series and its
discrete fit, the O(eta^3) error of m_* built from the exact solution, and the
estimator against the paper's closed-form u."""
import math

import numpy as np
import pytest

from paper_2606_21883_amd import inputs

R, A, PHI_C = 1.0, 0.45, 0.35 * math.pi


def _prob(**kw):
    return dict(inputs.cut_torus_problem(), **kw)


def _normal(th, s):
    """Outward unit normal of the tube at X(th, phi_c + s)."""
    ph = PHI_C + s
    return np.array([math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), math.sin(th)])


def test_closed_form_u_vanishes_on_the_cut():
    th = np.linspace(0, 2 * np.pi, 17)
    for s in (0.0, np.pi):
        assert np.max(np.abs(inputs.torus_sine_u(inputs.EX1_COEF, th, s))) < 1e-15
    # the paper's A, B, C written out
    t, s = 0.7, 1.1
    Av = 1 + 0.90 * math.cos(t) + 0.60 * math.sin(2 * t) + 0.35 * math.cos(3 * t)
    Bv = 0.45 * math.cos(2 * t)
    Cv = 0.30 * (0.5 + math.sin(t))
    assert inputs.torus_sine_u(inputs.EX1_COEF, t, s) == pytest.approx(
        math.sin(s) * Av + math.sin(2 * s) * Bv + math.sin(3 * s) * Cv, rel=1e-15)


def test_delta_gamma_against_brute_force(orc):
    """dist(y, E_Gamma(y_Gamma)): y_Gamma by a dense search over both cut
    circles, then the distance to the normal segment of half-length
    ell = c_kappa / (1 + 1/a) sampled densely."""
    P = orc.Problem(_prob())
    rng = np.random.default_rng(3)
    ell = 1.2 / (1.0 + 1.0 / A)
    tg = np.linspace(0, 2 * np.pi, 200001)[:-1]
    for _ in range(10):
        th, s = rng.uniform(0, 2 * np.pi), rng.choice([rng.uniform(0.01, 0.4), rng.uniform(2.7, 3.13)])
        y = inputs.cut_torus_point(th, s)
        # a point off M too (the walk only asks at points of M, but the
        # formula is defined for any y)
        y = y + rng.uniform(-0.05, 0.05) * _normal(th, s)
        best = None
        for sb in (0.0, np.pi):
            C = inputs.cut_torus_point(tg, np.full_like(tg, sb))
            d2 = ((C - y) ** 2).sum(1)
            i = int(np.argmin(d2))
            if best is None or d2[i] < best[0]:
                best = (d2[i], C[i], _normal(tg[i], sb))
        _, yg, ng = best
        t = np.linspace(-ell, ell, 40001)
        seg = yg[None, :] + t[:, None] * ng[None, :]
        dist = np.sqrt(((seg - y) ** 2).sum(1)).min()
        assert orc.delta_gamma(P, y) == pytest.approx(dist, abs=2e-5)


def test_far_side_of_the_cut_stops_at_once(orc):
    """A start in the layer or beyond the cut returns g with K = 0; a start
    in the interior takes at least one step."""
    prob = _prob(g=dict(kind="const", coef=[0.25]), n_v=1)
    for s, stops in ((-0.3, True), (math.pi + 0.2, True), (1e-7, True), (1.5, False)):
        y = inputs.cut_torus_point(0.4, s)
        S, K, _ = orc.walk(prob, y, 0, 0, 5)
        if stops:
            assert K == 0 and S == 0.25
        else:
            assert K > 0


def _intrinsic_f(th, s, sigma=4.0):
    """-Lap_T u + sigma u with Lap_T u = (1/sqrt g) d_i (sqrt g g^ii d_i u),
    sqrt g = a (R + a cos th), g^thth = 1/a^2, g^phiphi = 1/(R + a cos th)^2,
    by central differences of the closed-form u."""
    u = lambda t, v: float(inputs.torus_sine_u(inputs.EX1_COEF, t, v))
    q = lambda t: R + A * math.cos(t)
    h = 1e-4

    def flux(t):
        return A * q(t) / (A * A) * (u(t + h / 2, s) - u(t - h / 2, s)) / h
    lap = ((flux(th + h / 2) - flux(th - h / 2)) / h
           + A * q(th) / q(th) ** 2 * (u(th, s + h) - 2 * u(th, s) + u(th, s - h)) / h ** 2) / (A * q(th))
    return -lap + sigma * u(th, s)


def test_source_against_intrinsic_laplacian(orc):
    P = orc.Problem(_prob(compensation="none"))
    rng = np.random.default_rng(7)
    for _ in range(12):
        th, s = rng.uniform(0, 2 * np.pi), rng.uniform(0.1, 3.0)
        y = inputs.cut_torus_point(th, s)
        assert orc.source(P, y) == pytest.approx(_intrinsic_f(th, s), rel=1e-6, abs=1e-6)


def _ambient_m(orc, prob, x, h=1e-3):
    """m(x) = -Lap(Eu)(x) + sigma Eu(x) - f(x) (eq. mismatch_definition) with the
    ambient Laplacian by second differences along the axes, Eu = u(cp(.))."""
    Pn = orc.Problem(dict(prob, compensation="none"))
    Eu = lambda z: float(inputs.exact_u(prob, orc.cp(prob, z)[None])[0])
    lap = sum((Eu(x + h * e) - 2 * Eu(x) + Eu(x - h * e)) / h ** 2 for e in np.eye(3))
    return -lap + prob["sigma"] * Eu(x) - orc.source(Pn, orc.cp(prob, x))


def test_exact_compensation_against_its_definition(orc):
    prob = _prob(compensation="exact")
    P, Pn = orc.Problem(prob), orc.Problem(dict(prob, compensation="none"))
    rng = np.random.default_rng(9)
    for _ in range(6):
        th, s, eta = rng.uniform(0, 2 * np.pi), rng.uniform(0.3, 2.8), rng.uniform(-0.12, 0.12)
        x = inputs.cut_torus_point(th, s) + eta * _normal(th, s)
        m = orc.source(P, x) - orc.source(Pn, x)
        assert m == pytest.approx(_ambient_m(orc, prob, x), rel=2e-4, abs=2e-5)
        # m vanishes on M (eq. LB_cp_identity)
        y = inputs.cut_torus_point(th, s)
        assert abs(orc.source(P, y) - orc.source(Pn, y)) < 1e-12


def test_series_values_and_derivatives(orc):
    rng = np.random.default_rng(2)
    ks, kt = 4, 3
    c = rng.standard_normal((ks, 2 * kt + 1))
    h = 1e-4
    u = lambda t, v: float(inputs.torus_sine_u(c, t, v))
    for _ in range(5):
        th, s = rng.uniform(0, 2 * np.pi), rng.uniform(0, np.pi)
        v = orc.ts_value(c.ravel(), ks, kt, th, s)
        assert v[0] == pytest.approx(u(th, s), rel=1e-13, abs=1e-13)
        assert v[1] == pytest.approx((u(th + h, s) - u(th - h, s)) / (2 * h), rel=1e-6, abs=1e-7)
        assert v[2] == pytest.approx((u(th + h, s) - 2 * u(th, s) + u(th - h, s)) / h ** 2, rel=1e-5, abs=1e-5)
        assert v[3] == pytest.approx((u(th, s + h) - 2 * u(th, s) + u(th, s - h)) / h ** 2, rel=1e-5, abs=1e-5)


def test_fit_reproduces_series_within_its_range(orc):
    rng = np.random.default_rng(4)
    nt, ns, ks, kt = 16, 8, 5, 6
    c = rng.standard_normal((ks, 2 * kt + 1))
    th = 2 * np.pi * np.arange(nt) / nt
    s = np.pi * np.arange(1, ns) / ns
    T, S = np.meshgrid(th, s, indexing="ij")
    U = inputs.torus_sine_u(c, T, S)
    np.testing.assert_allclose(orc.ts_fit(U, kt, ks).reshape(ks, -1), c, rtol=0, atol=1e-13)
    # truncation: a fit to fewer modes keeps exactly the modes it has
    np.testing.assert_allclose(orc.ts_fit(U, 2, 3).reshape(3, -1), c[:3, :5], rtol=0, atol=1e-13)
    with pytest.raises(ValueError):
        orc.ts_fit(U, 8, 3)          # 2 kt >= nt
    with pytest.raises(ValueError):
        orc.ts_fit(U, 2, 8)          # ks >= ns


def test_second_order_compensation_from_the_exact_solution(orc):
    """With u_* = u the normal residual R_*(s; y) is m(y + s n(y)), so m_* is
    the second-order Taylor polynomial of m along the normal: m - m_* =
    O(eta^3), and eta m1 + eta^2 m2 / 2 matches one-sided derivatives of the
    exact m taken independently."""
    base = _prob()
    so = dict(base, compensation="second_order", h_eta=1e-3,
              predictor=dict(idx=[3, 3], values=inputs.EX1_COEF.ravel()))
    Pe, Ps, Pn = (orc.Problem(dict(base, compensation="exact")), orc.Problem(so),
                  orc.Problem(dict(base, compensation="none")))
    rng = np.random.default_rng(11)
    for _ in range(5):
        th, s = rng.uniform(0, 2 * np.pi), rng.uniform(0.3, 2.8)
        y = inputs.cut_torus_point(th, s)
        n = _normal(th, s)
        errs = []
        for eta in (0.08, 0.04, 0.02):
            x = y + eta * n
            m = orc.source(Pe, x) - orc.source(Pn, x)
            ms = orc.source(Ps, x) - orc.source(Pn, x)
            errs.append(abs(m - ms))
        assert 5.5 < errs[0] / errs[1] < 10.5 and 5.5 < errs[1] / errs[2] < 10.5, errs
        # Taylor coefficients of the exact m at eta = 0 by a five-point stencil
        hh = 2e-3
        mv = [orc.source(Pe, y + k * hh * n) - orc.source(Pn, y + k * hh * n) for k in (-2, -1, 0, 1, 2)]
        m1 = (-mv[4] + 8 * mv[3] - 8 * mv[1] + mv[0]) / (12 * hh)
        m2 = (-mv[4] + 16 * mv[3] - 30 * mv[2] + 16 * mv[1] - mv[0]) / (12 * hh * hh)
        # a finer normal step, so the difference quotients' own error
        # (h^2 m''' / 6) stays below the stencil's
        Pf = orc.Problem(dict(so, h_eta=1e-4))
        eta = 1e-2
        ms = orc.source(Pf, y + eta * n) - orc.source(Pn, y + eta * n)
        assert ms == pytest.approx(eta * m1 + 0.5 * eta * eta * m2, rel=1e-5, abs=1e-9)


def test_zero_predictor_gives_no_compensation(orc):
    """u_* = 0 makes R_*(s; y) = -f(y) for every s: both differences vanish."""
    base = _prob()
    so = orc.Problem(dict(base, compensation="second_order", h_eta=1e-3,
                          predictor=dict(idx=[2, 1], values=np.zeros(6))))
    Pn = orc.Problem(dict(base, compensation="none"))
    rng = np.random.default_rng(12)
    for _ in range(5):
        th, s, eta = rng.uniform(0, 2 * np.pi), rng.uniform(0.3, 2.8), rng.uniform(-0.1, 0.1)
        x = inputs.cut_torus_point(th, s) + eta * _normal(th, s)
        assert orc.source(so, x) == orc.source(Pn, x)


def test_estimator_matches_the_closed_form(orc):
    """Exact compensation: the estimate of Example 1 agrees with the paper's u
    within 4.5 standard errors (the boundary layer eps = 1e-5 adds a bias far
    below them)."""
    prob = inputs.cut_torus_problem(n_v=1, compensation="exact")
    Q = inputs.cut_torus_points(6, seed=3)
    res = orc.solve(prob, Q, 12000, seed=5)
    z = (res["u"] - inputs.exact_u(prob, Q)) / res["stderr"]
    assert np.all(np.abs(z) < 4.5), z


@pytest.mark.parametrize("c_kappa,ratio,floor", [(0.4, 0.1, 2e-3), (1.2, 0.5, 2e-2)])
def test_second_order_removes_most_of_the_bias(orc, c_kappa, ratio, floor):
    """m_* from the exact solution against the exact m on the same random
    numbers (the walks are identical; only the source values differ): the
    baseline m_* = 0 leaves a bias that the second-order term mostly removes,
    the more so the smaller the balls (its error is O(eta^3))."""
    Q = inputs.cut_torus_points(4, seed=3)
    out = {}
    for comp in ("none", "second_order", "exact"):
        prob = dict(inputs.cut_torus_problem(n_v=1, compensation=comp), c_kappa=c_kappa)
        if comp == "second_order":
            prob.update(h_eta=1e-3, predictor=dict(idx=[3, 3], values=inputs.EX1_COEF.ravel()))
        out[comp] = orc.solve(prob, Q, 1500 if c_kappa < 1 else 4000, seed=5)["u"]
    e_none = np.sqrt(np.mean((out["none"] - out["exact"]) ** 2))
    e_so = np.sqrt(np.mean((out["second_order"] - out["exact"]) ** 2))
    assert e_none > floor and e_so < ratio * e_none, (e_none, e_so)


def test_cut_torus_rejects_other_settings(orc):
    Q = inputs.cut_torus_points(2, seed=3)
    bad = [dict(compensation="second_order"),                                   # no predictor
           dict(compensation="second_order", h_eta=0.3, predictor=dict(idx=[1, 0], values=[0.0])),
           dict(g=dict(kind="sph_pair", idx=[0, 1], coef=[1.0])),
           dict(radius_rule="spacing"), dict(eps=0.0), dict(p=[1.0, 1.2, 0.0])]
    for b in bad:
        with pytest.raises(ValueError):
            orc.solve(_prob(**b), Q, 2, seed=1)
    # the series source and the predictor belong to the cut torus
    with pytest.raises(ValueError):
        orc.solve(dict(inputs.torus_problem(), f=_prob()["f"]), inputs.torus_area_uniform(2), 2, seed=1)
