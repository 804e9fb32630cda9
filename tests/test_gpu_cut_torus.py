"""GPU parity on the torus with a planar cut of Example 1 (one lane per walk):
the closest point and the boundary stop against the oracle, whole FP64 walks
walk by walk with no, exact and second-order compensation, the device
predictor fit against the oracle's, FP32 statistics against FP64, and the
compensated estimate against the paper's closed-form u."""
import numpy as np
import pytest

import oracle
from paper_2606_21883_amd import inputs, mpwos
from tests.gpu_util import announce, compare_walks

pytestmark = pytest.mark.gpu


def _predictor(seed=1, ks=4, kt=4):
    """A predictor near Example 1's u: its coefficients, padded to ks x (2 kt + 1),
    plus seeded perturbations (so m_* differs from the exact m)."""
    c = np.zeros((ks, 2 * kt + 1))
    c[:3, :7] = inputs.EX1_COEF
    c += 0.02 * np.random.default_rng(seed).standard_normal(c.shape)
    return dict(idx=[ks, kt], values=c.ravel())


def test_cut_torus_cp_matches_oracle():
    prob = inputs.cut_torus_problem()
    P = oracle.Problem(prob)
    rng = np.random.default_rng(3)
    Y = inputs.cut_torus_points(200, seed=4)
    # off M within 0.4 < a (inside the reach of the tube; nearer the core
    # circle the nearest point stops being unique)
    d = rng.standard_normal((200, 3))
    d *= rng.uniform(-0.4, 0.4, (200, 1)) / np.linalg.norm(d, axis=1, keepdims=True)
    X = np.concatenate([Y, Y + d])
    m = mpwos.Manifold(prob)
    announce("cut torus cp")
    y64 = mpwos.debug_cp(m, X, "fp64")
    y32 = mpwos.debug_cp(m, X, "fp32")
    m.close()
    yo = np.array([oracle.cp(P, x) for x in X])
    np.testing.assert_allclose(y64, yo, rtol=0, atol=1e-13)
    np.testing.assert_allclose(y32, yo, rtol=0, atol=5e-6)


@pytest.mark.parametrize("comp,n_v", [("none", 1), ("exact", 1), ("second_order", 1), ("second_order", 3),
                                      ("exact", 2)])
def test_cut_torus_walks_fp64_match_oracle(comp, n_v):
    prob = inputs.cut_torus_problem(n_v=n_v, compensation=comp)
    if comp == "second_order":
        prob.update(h_eta=1e-2, predictor=_predictor())
    # a few queries near the cut, the rest anywhere in Omega
    Q = np.concatenate([inputs.cut_torus_points(4, seed=5),
                        inputs.cut_torus_point(np.array([0.3, 2.0]), np.array([0.02, 3.1]))])
    announce(f"cut torus walks fp64 {len(Q)}x64 {comp} n_v={n_v}")
    gpu = mpwos.solve(prob, Q, 64, 3, walk_outputs=True, precision="fp64")
    orc = oracle.solve(oracle.Problem(prob), Q, 64, 3)
    assert compare_walks(gpu, orc, prob) >= 0.999
    np.testing.assert_allclose(gpu["u"], orc["u"], rtol=1e-10, atol=1e-12)


def test_cut_torus_g_const_and_starts_in_the_layer():
    """A constant g: walks starting inside the layer return it at once."""
    prob = dict(inputs.cut_torus_problem(n_v=1), g=dict(kind="const", coef=[0.75]), eps=1e-2)
    Q = inputs.cut_torus_point(np.array([0.5, 1.0, 2.0]), np.array([0.005, np.pi - 0.004, 1.5]))
    announce("cut torus g const")
    gpu = mpwos.solve(prob, Q, 32, 4, walk_outputs=True, precision="fp64")
    orc = oracle.solve(oracle.Problem(prob), Q, 32, 4)
    assert compare_walks(gpu, orc, prob) == 1.0
    assert np.all(gpu["walk_K"][:2] == 0) and np.all(gpu["walk_S"][:2] == 0.75)


def test_device_fit_matches_oracle():
    rng = np.random.default_rng(6)
    for nt, ns, ks, kt in [(32, 16, 4, 4), (7, 3, 2, 3), (64, 40, 12, 20)]:
        U = rng.standard_normal((nt, ns - 1))
        announce(f"ts fit {nt}x{ns} {ks},{kt}")
        c = mpwos.debug_ts_fit(U, ks, kt)
        np.testing.assert_allclose(c.ravel(), oracle.ts_fit(U, kt, ks), rtol=0, atol=1e-13)
    with pytest.raises(mpwos.MpwosError):
        mpwos.debug_ts_fit(U, 40, 3)


def test_predictor_fit_matches_oracle_pipeline():
    """Device nodes, coarse solve and fit against the oracle doing the same
    steps (nodes from the inputs module, which holds the same grid)."""
    prob = inputs.cut_torus_problem(n_v=1)
    nt, ns, nw, ks, kt = 8, 6, 16, 3, 3
    announce("predictor fit 8x6x16")
    coef, st = mpwos.predictor_fit(prob, nt, ns, nw, 11, ks, kt, precision="fp64")
    nodes = inputs.cut_torus_nodes(nt, ns)
    orc = oracle.solve(oracle.Problem(dict(prob, compensation="none")), nodes, nw, 11)
    ref = oracle.ts_fit(orc["u"].reshape(nt, ns - 1), kt, ks)
    np.testing.assert_allclose(coef.ravel(), ref, rtol=0, atol=1e-9)
    assert st["walk_steps"] == int(orc["walk_K"].sum())


def test_cut_torus_fp32_statistics_match_fp64():
    prob = inputs.cut_torus_problem(n_v=1, compensation="second_order")
    prob.update(h_eta=1e-2, predictor=_predictor(2))
    Q = inputs.cut_torus_points(8, seed=6)
    m = mpwos.Manifold(prob)
    announce("cut torus fp64 vs fp32 8x4096")
    r64 = mpwos.solve(prob, Q, 4096, 7, manifold=m, precision="fp64")
    r32 = mpwos.solve(prob, Q, 4096, 7, manifold=m, precision="fp32")
    m.close()
    se = np.sqrt(r64["stderr"] ** 2 + r32["stderr"] ** 2)
    assert np.all(np.abs(r64["u"] - r32["u"]) < 5 * se + 1e-6), (r64["u"] - r32["u"], se)


def test_compensated_estimate_against_the_closed_form():
    """Example 1 at the paper's setting (N_V = 50, eps = 1e-5): exact
    compensation is unbiased; the second-order m_* from a coarse device
    predictor removes most of the bias the baseline leaves (the same random
    numbers drive all three solves, so their differences are the biases)."""
    base = inputs.cut_torus_problem()
    Q = inputs.cut_torus_points(16, seed=8)
    u = inputs.exact_u(base, Q)
    m = mpwos.Manifold(base)
    announce("cut torus predictor 32x16x256")
    coef, _ = mpwos.predictor_fit(base, 32, 16, 256, 21, 4, 4, manifold=m, precision="fp32")
    out = {}
    for comp in ("none", "exact", "second_order"):
        prob = dict(base, compensation=comp)
        if comp == "second_order":
            prob.update(h_eta=1e-2, predictor=dict(idx=[4, 4], values=coef.ravel()))
        announce(f"cut torus 16x8192 {comp}")
        out[comp] = mpwos.solve(prob, Q, 8192, 5, manifold=m, precision="fp32")
    m.close()
    ex = out["exact"]
    assert np.all(np.abs(ex["u"] - u) < 5 * ex["stderr"] + 2e-3), (ex["u"] - u, ex["stderr"])
    e_none = np.sqrt(np.mean((out["none"]["u"] - ex["u"]) ** 2))
    e_so = np.sqrt(np.mean((out["second_order"]["u"] - ex["u"]) ** 2))
    assert e_so < 0.6 * e_none, (e_none, e_so)


def test_served_and_planned_second_order_equal_solo():
    """The compensated cut-torus solve through the server and as a captured
    plan: the same bits as the solo solve (the predictor rows travel with
    the source family's values)."""
    import torch
    prob = inputs.cut_torus_problem(n_v=2, compensation="second_order")
    prob.update(h_eta=1e-2, predictor=_predictor(3))
    Q = inputs.cut_torus_points(12, seed=9)
    m = mpwos.Manifold(prob)
    announce("cut torus served + plan 12x256")
    solo = mpwos.solve(prob, Q, 256, 4, manifold=m, precision="fp32", persistent=1)
    srv = mpwos.Server(1 << 30)
    out = srv.wait(srv.submit(m, prob, Q, 256, 4, precision="fp32", persistent=1), 60_000)
    srv.close()
    assert np.array_equal(solo["u"], out["u"]) and np.array_equal(solo["stderr"], out["stderr"])
    plan = mpwos.Plan(m, prob, len(Q), 256, precision="fp32", persistent=1)
    stream = torch.cuda.current_stream().cuda_stream
    dq = torch.from_numpy(np.ascontiguousarray(Q)).to("cuda")
    u = torch.zeros(len(Q), dtype=torch.float64, device="cuda")
    se = torch.zeros(len(Q), dtype=torch.float64, device="cuda")
    for _ in range(2):
        plan.execute(dq.data_ptr(), u.data_ptr(), se.data_ptr(), 4, stream)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), solo["u"])
        torch.ones(1 << 16, device="cuda").sum().item()
    plan.close()
    m.close()


def test_predictor_fit_rejects_bad_grids():
    prob = inputs.cut_torus_problem(n_v=1)
    m = mpwos.Manifold(prob)
    announce("predictor fit argument checks")
    for nt, ns, ks, kt in [(8, 6, 6, 1), (8, 6, 2, 4), (0, 6, 2, 1), (8, 1, 1, 0), (2048, 1024, 2, 1)]:
        with pytest.raises(mpwos.MpwosError):
            mpwos.predictor_fit(prob, nt, ns, 4, 1, ks, kt, manifold=m)
    m.close()
    # the fit is defined on the cut torus only
    sph = inputs.sphere_problem()
    with pytest.raises(mpwos.MpwosError):
        mpwos.predictor_fit(dict(sph, f=prob["f"]), 8, 6, 4, 1, 2, 1)
    # a second-order solve without predictor rows, or with h_eta out of range
    Q = inputs.cut_torus_points(2, seed=1)
    with pytest.raises(mpwos.MpwosError):
        mpwos.solve(dict(prob, compensation="second_order"), Q, 4, 1)
    with pytest.raises(mpwos.MpwosError):
        mpwos.solve(dict(prob, compensation="second_order", h_eta=0.3,
                         predictor=dict(idx=[1, 0], values=[0.0])), Q, 4, 1)
