"""Pins of the whole estimator (Algorithm 1, eq. path_score_definition,
eq. mc_estimator) in the oracle.

- Constant-solution invariants (telescoping of the one-step identity in the
  proof of Theorem 2.2): with f = sigma C and m = 0 every closed-manifold path
  scores exactly C (1 - W_K); with also g = C every boundary path scores C.
- Closed-form solutions (spherical harmonics on S^1, S^2, S^9, Legendre sums,
  the torus mode): the Monte Carlo mean is unbiased up to tau_W, within a few
  standard errors (Theorem 3.9).
- A circle problem with a non-eigenfunction source against a brute-force
  periodic finite-difference solve.
- Variance scaling with N and N_V (Lemma 3.2).
"""
import math

import numpy as np
import pytest

from paper_2606_21883_amd import inputs


def zscores(res, exact):
    return (res["u"] - exact) / res["stderr"]


def assert_unbiased(res, exact, zmax=4.5):
    z = zscores(res, exact)
    assert np.max(np.abs(z)) < zmax, z
    assert np.mean(z * z) < 2.0, np.mean(z * z)


def test_constant_solution_closed(orc):
    C = 1.7
    prob = inputs.problem(manifold="sphere", n=3, p=[1.0], sigma=2.0, compensation="none",
                          f=dict(kind="const", coef=[2.0 * C]))
    Q = inputs.sphere_uniform(8, 3, seed=2)
    res = orc.solve(prob, Q, 64, seed=5)
    c = orc.c_sigma_r(3, 2.0, 0.57)
    K = res["walk_K"]
    assert np.all(K == 174)
    W = 1.0
    for _ in range(174):
        W *= c
    np.testing.assert_allclose(res["walk_S"], C * (1.0 - W), rtol=1e-13)


def test_constant_solution_closed_torus(orc):
    C = -0.3
    prob = inputs.problem(manifold="torus", n=3, p=[1.0, 0.3], sigma=1.0, compensation="none",
                          tau_w=1e-3, f=dict(kind="const", coef=[C]))
    Q = inputs.torus_area_uniform(4, seed=2)
    res = orc.solve(prob, Q, 16, seed=5)
    c = orc.c_sigma_r(3, 1.0, 0.95 * 1.2 / (1 + 1 / 0.3))
    K = int(res["walk_K"][0, 0])
    assert np.all(res["walk_K"] == K) and c ** K < 1e-3 <= c ** (K - 1)
    np.testing.assert_allclose(res["walk_S"], C * (1.0 - c ** K), rtol=1e-12)


def test_constant_solution_boundary(orc):
    C = 0.8
    prob = dict(inputs.cap_problem(), f=dict(kind="const", coef=[0.5 * C]),
                g=dict(kind="const", coef=[C]), compensation="none")
    Q = inputs.cap_uniform(16, 3, 0.0, seed=3)
    res = orc.solve(prob, Q, 64, seed=6)
    np.testing.assert_allclose(res["walk_S"], C, rtol=1e-13)
    assert res["walk_K"].min() >= 1


def test_query_inside_layer_scores_boundary_value(orc):
    prob = inputs.cap_problem(eps=1e-3)
    y = np.array([math.cos(1e-4) * 0.6, math.cos(1e-4) * 0.8, math.sin(1e-4)])
    S, K, tr = orc.walk(prob, y, 0, 0, 1)
    assert K == 0
    assert S == pytest.approx(0.6 * 0.8, rel=1e-12)


def test_closed_form_circle(orc):
    prob, Q, _ = inputs.config("circle")
    Q = Q[::4]
    res = orc.solve(prob, Q, 400, seed=0)
    assert np.all(res["walk_K"] == 232)
    assert_unbiased(res, inputs.exact_u(prob, Q))


def test_closed_form_sphere(orc):
    prob = inputs.sphere_problem()
    Q = inputs.sphere_uniform(16, 3, seed=1)
    res = orc.solve(prob, Q, 500, seed=0)
    assert_unbiased(res, inputs.exact_u(prob, Q))


def test_closed_form_cap(orc):
    prob = inputs.cap_problem()
    Q = inputs.cap_uniform(24, 3, 0.0, seed=1)
    res = orc.solve(prob, Q, 500, seed=0)
    assert_unbiased(res, inputs.exact_u(prob, Q))
    K = res["walk_K"]
    assert 20 < K.mean() < 40


def test_closed_form_hypersphere_n10(orc):
    prob = inputs.hypersphere_problem(10)
    Q = inputs.hypersphere_queries(12, 10, seed=1)
    res = orc.solve(prob, Q, 300, seed=0)
    assert_unbiased(res, inputs.exact_u(prob, Q))


def test_closed_form_legendre_sphere(orc):
    # the Legendre solution form of the paper's point-cloud sphere example, sigma = 1
    sg = 1.0
    coef = [0.0, (sg + 2) * 1.0, 0.0, 0.2 * (sg + 12), 0.0, 0.1 * (sg + 30)]
    prob = inputs.problem(manifold="sphere", n=3, p=[1.0], sigma=sg, f=dict(kind="legendre", coef=coef))
    Q = inputs.sphere_uniform(12, 3, seed=4)
    res = orc.solve(prob, Q, 300, seed=1)
    t = Q[:, 2]
    u = t + 0.2 * 0.5 * (5 * t ** 3 - 3 * t) + 0.1 * (63 * t ** 5 - 70 * t ** 3 + 15 * t) / 8
    np.testing.assert_allclose(inputs.exact_u(prob, Q), u, rtol=1e-13)
    assert_unbiased(res, u)


def test_closed_form_torus(orc):
    prob = inputs.torus_problem()
    Q = inputs.torus_area_uniform(8, seed=1)
    res = orc.solve(prob, Q, 150, seed=0)
    assert np.all(res["walk_K"] == 1601)
    assert_unbiased(res, inputs.exact_u(prob, Q))


def test_compensation_matters(orc):
    # Without m the estimator is biased on S^2 at r = 0.57 (Lemma 3.5): the
    # bias is many standard errors at this N, with the sign of -u.
    prob = dict(inputs.sphere_problem(), compensation="none")
    Q = np.array([[math.sqrt(0.5), math.sqrt(0.5), 0.0]])
    res = orc.solve(prob, Q, 30000, seed=2)
    exact = 0.5
    assert (res["u"][0] - exact) / res["stderr"][0] < -4


def fd_circle(f_vals, sigma):
    """Periodic second-order finite differences for -u'' + sigma u = f on [0, 2 pi)."""
    M = f_vals.size
    h = 2 * np.pi / M
    main = np.full(M, 2.0 / h ** 2 + sigma)
    A = np.diag(main) + np.diag(np.full(M - 1, -1 / h ** 2), 1) + np.diag(np.full(M - 1, -1 / h ** 2), -1)
    A[0, -1] = A[-1, 0] = -1 / h ** 2
    return np.linalg.solve(A, f_vals)


def test_circle_non_eigen_source_vs_finite_differences(orc):
    M = 4096
    sigma = 1.0
    th = 2 * np.pi * np.arange(M) / M
    f = np.exp(np.cos(th))
    u_fd = fd_circle(f, sigma)
    # the compensation uses the finite-difference solution as its predictor u_*
    prob = inputs.problem(manifold="sphere", n=2, p=[1.0], sigma=sigma,
                          f=dict(kind="table_s1", values=np.concatenate([f, u_fd])))
    idx = np.arange(0, M, M // 16)
    Q = np.stack([np.cos(th[idx]), np.sin(th[idx])], 1)
    res = orc.solve(prob, Q, 800, seed=3)
    assert_unbiased(res, u_fd[idx])


def test_variance_scaling_in_N_and_NV(orc):
    prob = inputs.sphere_problem()
    Q = inputs.sphere_uniform(4, 3, seed=8)
    r1 = orc.solve(prob, Q, 200, seed=1)
    r4 = orc.solve(prob, Q, 800, seed=1)
    ratio = r1["stderr"] / r4["stderr"]
    assert np.all((ratio > 1.6) & (ratio < 2.5)), ratio
    rv = orc.solve(dict(prob, n_v=8), Q, 200, seed=1)
    # N_V only shrinks the Green-sample part of the variance
    assert np.all(rv["stderr"] < r1["stderr"])


def test_truncation_reported(orc):
    prob = dict(inputs.sphere_problem(), max_steps=10)
    Q = inputs.sphere_uniform(2, 3, seed=8)
    res = orc.solve(prob, Q, 4, seed=1)
    assert res["status"] == "WTRUNC" and res["truncated"] == 8
    assert np.all(res["walk_K"] == 10)


def test_invalid_arguments_rejected(orc):
    Q = inputs.sphere_uniform(2, 3, seed=8)
    for bad in [dict(sigma=0.0), dict(sigma=-1.0), dict(theta=1.0), dict(n_v=0), dict(tau_w=1.0)]:
        with pytest.raises(ValueError):
            orc.solve(dict(inputs.sphere_problem(), **bad), Q, 4, seed=1)
    with pytest.raises(ValueError, match="EOFFMANIFOLD"):
        orc.solve(inputs.sphere_problem(), Q * 1.01, 4, seed=1)
