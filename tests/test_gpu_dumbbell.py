"""GPU parity on the implicit dumbbell of Example 2 (n up to 1001, one lane
group per walk): the closest point against the oracle in both precisions,
whole FP64 walks against the oracle walk by walk, FP32 statistics against
FP64, and served requests against solo solves."""
import numpy as np
import pytest

import oracle
from paper_2606_21883_amd import inputs, mpwos
from tests.gpu_util import announce, compare_walks

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [11, 101, 1001])
def test_cp_matches_oracle(n):
    prob = inputs.dumbbell_problem(n)
    P = oracle.Problem(prob)
    rng = np.random.default_rng(n)
    Y = inputs.dumbbell_points(40, n, seed=n)
    X = Y + rng.uniform(-0.25, 0.25, (40, 1)) * rng.standard_normal((40, n)) / np.sqrt(n)
    X = np.concatenate([Y, X])
    m = mpwos.Manifold(prob)
    announce(f"dumbbell cp n={n}")
    y64 = mpwos.debug_cp(m, X, "fp64")
    y32 = mpwos.debug_cp(m, X, "fp32")
    m.close()
    yo = np.array([oracle.cp(P, x) for x in X])
    np.testing.assert_allclose(y64, yo, rtol=0, atol=1e-12)
    np.testing.assert_allclose(y32, yo, rtol=0, atol=5e-6)


# the last case is Table 1's setting: n = 1001, N_V = 50, tau_W = 1e-8 (K = 220)
@pytest.mark.parametrize("n,nq,nw,n_v,tau_w", [(11, 4, 32, 1, 1e-8), (11, 4, 16, 2, 1e-8), (1001, 2, 8, 1, 1e-3),
                                               (1001, 2, 8, 2, 1e-3), (1001, 2, 4, 50, 1e-8)])
def test_walks_fp64_match_oracle(n, nq, nw, n_v, tau_w):
    prob = dict(inputs.dumbbell_problem(n, n_v=n_v), tau_w=tau_w)
    Q = inputs.dumbbell_points(nq, n, seed=5)
    announce(f"dumbbell walks fp64 n={n} {nq}x{nw} n_v={n_v}")
    gpu = mpwos.solve(prob, Q, nw, 3, walk_outputs=True, precision="fp64")
    orc = oracle.solve(oracle.Problem(prob), Q, nw, 3)
    assert compare_walks(gpu, orc, prob) == 1.0
    np.testing.assert_allclose(gpu["u"], orc["u"], rtol=1e-10, atol=1e-12)
    # constant radius: every walk has the same length
    assert len(set(gpu["walk_K"].ravel().tolist())) == 1


def test_fp32_statistics_match_fp64():
    n = 1001
    prob = dict(inputs.dumbbell_problem(n), tau_w=1e-4)
    Q = inputs.dumbbell_points(6, n, seed=6)
    m = mpwos.Manifold(prob)
    announce("dumbbell fp64 vs fp32 6x512")
    r64 = mpwos.solve(prob, Q, 512, 7, manifold=m, precision="fp64")
    r32 = mpwos.solve(prob, Q, 512, 7, manifold=m, precision="fp32")
    m.close()
    se = np.sqrt(r64["stderr"] ** 2 + r32["stderr"] ** 2)
    assert np.all(np.abs(r64["u"] - r32["u"]) < 5 * se + 1e-6), (r64["u"] - r32["u"], se)


def test_served_dumbbell_equals_solo():
    """Table 1's N_V = 50 through the server: the same bits as a solo solve."""
    n = 1001
    prob = inputs.dumbbell_problem(n, n_v=50)
    Q = inputs.dumbbell_points(2, n, seed=8)
    m = mpwos.Manifold(prob)
    announce("dumbbell served n_v=50 2x16")
    solo = mpwos.solve(prob, Q, 16, 4, manifold=m, precision="fp32")
    srv = mpwos.Server(4 << 30)
    out = srv.wait(srv.submit(m, prob, Q, 16, 4, precision="fp32"), 120_000)
    srv.close()
    m.close()
    assert np.array_equal(solo["u"], out["u"]) and np.array_equal(solo["stderr"], out["stderr"])


def test_query_check_accepts_level_set_and_rejects_offsets():
    """The host's on-manifold check of dumbbell queries (Example 2's level set
    ||x_h|| = R(x_n)): points of the profile, also within 1e-6 of the tips,
    are accepted; points moved 1e-7 along the normal are refused."""
    n = 11
    prob = inputs.dumbbell_problem(n)
    m = mpwos.Manifold(prob)
    kc = prob["p"][1]
    Q = inputs.dumbbell_points(16, n, seed=9, phi_margin=0.0)
    # points near both tips: x_n = +-(kc - d), radius from the paper's R
    tips = []
    for d in (1e-6, 1e-9):
        for sgn in (1.0, -1.0):
            xs = sgn * (kc - d)
            e = np.zeros(n - 1)
            e[0] = 1.0
            tips.append(np.concatenate([e * inputs.dumbbell_profile_radius(xs), [xs]]))
    Q = np.concatenate([Q, np.array(tips)])
    announce("dumbbell query check n=11")
    mpwos.solve(prob, Q, 4, 0, manifold=m, precision="fp64", tau_w=0.5)
    # the normal at (R(xs) e, xs): the gradient of ||x_h|| - R(x_n), normalised
    for q in inputs.dumbbell_points(4, n, seed=10):
        xh, xs = q[:-1], q[-1]
        h = 1e-7
        dR = (inputs.dumbbell_profile_radius(xs + h) - inputs.dumbbell_profile_radius(xs - h)) / (2 * h)
        g = np.concatenate([xh / np.linalg.norm(xh), [-dR]])
        g /= np.linalg.norm(g)
        for s in (1e-7, -1e-7):
            with pytest.raises(mpwos.MpwosError) as ei:
                mpwos.solve(prob, (q + s * g)[None, :], 4, 0, manifold=m, precision="fp64", tau_w=0.5)
            assert ei.value.status == mpwos.EOFFMANIFOLD
    m.close()
