"""GPU parity on the product manifold of Example 3 (S^1_Fourier x S^2(0.65)
in R^9, four lanes per walk): the closest point against the oracle in both
precisions, FP64 walks walk by walk, FP32 statistics against FP64."""
import numpy as np
import pytest

import oracle
from paper_2606_21883_amd import inputs, mpwos
from tests.gpu_util import announce, compare_walks

pytestmark = pytest.mark.gpu


def test_product_cp_matches_oracle():
    prob = inputs.product_problem()
    P = oracle.Problem(prob)
    rng = np.random.default_rng(3)
    Y = inputs.product_points(100, seed=4)
    X = np.concatenate([Y, Y + 0.45 * rng.standard_normal((100, 9)) / 3.0])
    m = mpwos.Manifold(prob)
    announce("product cp")
    y64 = mpwos.debug_cp(m, X, "fp64")
    y32 = mpwos.debug_cp(m, X, "fp32")
    m.close()
    yo = np.array([oracle.cp(P, x) for x in X])
    np.testing.assert_allclose(y64, yo, rtol=0, atol=1e-13)
    np.testing.assert_allclose(y32, yo, rtol=0, atol=5e-6)


@pytest.mark.parametrize("n_v,tau_w", [(1, 1e-3), (2, 1e-2)])
def test_product_walks_fp64_match_oracle(n_v, tau_w):
    prob = dict(inputs.product_problem(), n_v=n_v, tau_w=tau_w)
    Q = inputs.product_points(3, seed=5)
    announce(f"product walks fp64 3x8 n_v={n_v}")
    gpu = mpwos.solve(prob, Q, 8, 2, walk_outputs=True, precision="fp64")
    orc = oracle.solve(oracle.Problem(prob), Q, 8, 2)
    assert compare_walks(gpu, orc, prob) == 1.0
    np.testing.assert_allclose(gpu["u"], orc["u"], rtol=1e-10, atol=1e-12)


def test_product_fp32_statistics_and_closed_form():
    prob = inputs.product_problem()
    Q = inputs.product_points(8, seed=6)
    m = mpwos.Manifold(prob)
    announce("product fp64 vs fp32 8x2048")
    r64 = mpwos.solve(prob, Q, 2048, 7, manifold=m, precision="fp64")
    r32 = mpwos.solve(prob, Q, 2048, 7, manifold=m, precision="fp32")
    m.close()
    se = np.sqrt(r64["stderr"] ** 2 + r32["stderr"] ** 2)
    assert np.all(np.abs(r64["u"] - r32["u"]) < 5 * se + 1e-6), (r64["u"] - r32["u"], se)
    # m = 0 (as in the paper) leaves a small bias: the closed form within 5
    # standard errors plus 0.02
    u = inputs.exact_u(prob, Q)
    assert np.all(np.abs(r64["u"] - u) < 5 * r64["stderr"] + 0.02), (r64["u"] - u, r64["stderr"])
