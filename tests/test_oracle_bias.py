"""Pins of the two stopping biases of the estimator in the oracle.

- Boundary layer (Assumption 3.3, Lemma 3.4): stopping in Gamma_eps and
  scoring g(cp_Gamma(Y_K)) instead of u(Y_K) costs at most L_Gamma eps.  The
  problem is chosen so that the bias is first order in eps: u = x1 x3 on the
  cap x3 > 0 of S^2 vanishes on the equator Gamma but has a nonzero normal
  derivative there.  Near the equator delta_Gamma(y) = |x3| and
  |u(y) - u(cp_Gamma(y))| = |x1 x3| <= delta_Gamma(y), so L_Gamma = 1.
- Truncation (the tau_W bound, eq. tau_w_bound, in the proof of Theorem 3.9): stopping a
  closed-manifold walk at W_K < tau_W drops E[W_K u(Y_K)], at most M_u tau_W.
  With u = x3 on S^2 (M_u = 1) the dropped part is measured walk by walk:
  the random numbers depend only on (query, walk, step), so a run with a
  larger tau_W follows the same path as one with tau_W = 1e-8 and stops
  earlier, and the difference of the two scores is exactly the dropped tail.
"""
import math

import numpy as np

from paper_2606_21883_amd import inputs


def cap_x1x3(eps, sigma=0.5):
    # -Lap u = 6 u for the degree-2 harmonic x1 x3, so f = (6 + sigma) u
    return inputs.problem(manifold="sphere_cap", n=3, p=[1.0, 0.0], sigma=sigma, eps=eps,
                          f=dict(kind="sph_pair", idx=[0, 2], coef=[6.0 + sigma]),
                          g=dict(kind="sph_pair", idx=[0, 2], coef=[1.0]))


def test_boundary_layer_bias_bounded_by_eps(orc):
    # queries at latitudes 0.15, 0.3 and 0.6 on the x1 x3 great circle
    lat = np.array([0.15, 0.3, 0.6])
    Q = np.stack([np.cos(lat), np.zeros(3), np.sin(lat)], 1)
    exact = Q[:, 0] * Q[:, 2]
    bias = {}
    for eps in (0.2, 0.1, 0.05, 0.01):
        res = orc.solve(cap_x1x3(eps), Q, 20000, seed=4)
        b = res["u"] - exact
        bias[eps] = b
        # Lemma 3.4 with L_Gamma = 1, plus the Monte Carlo error
        assert np.all(np.abs(b) <= 1.0 * eps + 4.5 * res["stderr"]), (eps, b, res["stderr"])
        if eps == 0.2:
            # the first query lies inside the layer: K = 0 and the score is g(cp) = 0
            assert np.all(res["walk_K"][0] == 0) and np.all(res["walk_S"][0] == 0.0)
        if eps >= 0.05:
            # the bound is not vacuous: walks stopping early at x1 > 0 lose W_K x1 x3 > 0
            z = b[1:] / res["stderr"][1:]
            assert np.all(z < -4.0), (eps, z)
        else:
            assert np.all(np.abs(b / res["stderr"]) < 4.5), (eps, b)
    # the bias shrinks with the layer, roughly linearly (first order in eps)
    for q in (1, 2):
        assert bias[0.2][q] < bias[0.1][q] < bias[0.05][q] < 0.0, [bias[e][q] for e in bias]
        assert 1.2 < bias[0.1][q] / bias[0.05][q] < 3.5


def test_truncation_bias_bounded_by_tau_w(orc):
    sg = 2.0
    # u = P_1(x3) = x3: -Lap u = 2 u, f = (2 + sigma) x3, |u| <= M_u = 1
    prob = inputs.problem(manifold="sphere", n=3, p=[1.0], sigma=sg,
                          f=dict(kind="legendre", coef=[0.0, sg + 2.0]))
    Q = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.8], [0.8, 0.0, 0.6]])
    u = Q[:, 2]
    nw = 10000
    ref = orc.solve(dict(prob, tau_w=1e-8), Q, nw, seed=4)
    c = orc.c_sigma_r(3, sg, 0.95 * 1.2 / 2.0)
    ratios = {}
    for tw in (0.3, 0.1):
        res = orc.solve(dict(prob, tau_w=tw), Q, nw, seed=4)
        # constant radius: W_k = c^k, so every walk stops at the first K with c^K < tau_W
        K = int(math.ceil(math.log(tw) / math.log(c)))
        assert c ** K < tw <= c ** (K - 1)
        assert np.all(res["walk_K"] == K)
        d = res["walk_S"] - ref["walk_S"]  # minus the tail from step K on, walk by walk
        mean = d.mean(1)
        se = d.std(1) / math.sqrt(nw)
        assert np.all(np.abs(mean) <= 1.0 * tw + 4.5 * se), (tw, mean, se)
        # the dropped tail is W_K E[u(Y_K)] = c^K lambda^K u(y): on the sphere the
        # one-step mean of a harmonic is a fixed multiple of it, so the tail over
        # u(y) is the same at every query
        r = -mean / (c ** K * u)
        rse = se / (c ** K * u)
        assert np.all(r > 0.0) and np.all(r < 1.0), r
        assert np.ptp(r) < 4.5 * math.sqrt(2.0) * rse.max(), (tw, r, rse)
        ratios[tw] = (K, float(np.average(r, weights=1.0 / rse ** 2)))
    # lambda^K at the two truncation indices gives the same per-step multiplier
    (K1, r1), (K2, r2) = ratios[0.3], ratios[0.1]
    lam1, lam2 = r1 ** (1.0 / K1), r2 ** (1.0 / K2)
    assert abs(lam1 - lam2) < 0.01, (lam1, lam2)
    # with tau_W = 1e-8 the remaining truncation is far below the noise
    assert np.all(np.abs(ref["u"] - u) < 4.5 * ref["stderr"])
