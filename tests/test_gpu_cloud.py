"""GPU parity of the point-cloud path (Sec. 2.3.2: nearest-neighbour search with
local reconstruction) against the oracle: the FP64 projection cp_h at cloud
points (which checks every patch, hence the device kNN build, through both the
MFMA grid-tile path and the KD-tree path) and at points off the surface; the
FP32 projection; whole FP64 walks on a small cloud and on the full 1e6-point
cloud (in the launch form the benchmark times), walk by walk; FP32 statistics;
query validation."""
import numpy as np
import pytest

import oracle
from paper_2606_21883_amd import inputs, mpwos
from tests.gpu_util import announce, compare_walks, score_scale

pytestmark = pytest.mark.gpu


def cloud(npts, seed, k=16, **kw):
    p = inputs.point_cloud_problem(inputs.torus_point_cloud(npts, seed=seed), k_nn=k)
    p.update(kw)
    return p


@pytest.mark.parametrize("k,fit_scale", [(16, 1.0), (28, 1.0), (16, 4.0)])
def test_cp_at_cloud_points_matches_oracle(k, fit_scale):
    """cp_h of a cloud point is the Newton foot point on its own patch: every
    sampled point checks its k nearest neighbours and its fit (over the k
    nearest, or over the ball of 4 r_k found on the device grid)."""
    prob = cloud(20000, seed=31, k=k, fit_scale=fit_scale)
    announce(f"cloud cp at cloud points k={k} fit_scale={fit_scale}")
    m = mpwos.Manifold(prob)
    info = mpwos.debug_cloud_info(m)
    if k <= 24:
        # the grid tiles settle almost every point
        assert info["knn_fallback_points"] < 0.05 * 20000, info
    else:
        assert info["knn_fallback_points"] == 20000, info
    P = oracle.Problem(prob)
    pts = prob["points"][np.random.default_rng(1).choice(20000, 600, replace=False)]
    y_gpu = mpwos.debug_cp(m, pts, "fp64")
    y_orc = np.array([oracle.cp(P, x) for x in pts])
    np.testing.assert_allclose(y_gpu, y_orc, rtol=0, atol=1e-11)
    m.close()


def test_cp_off_surface_matches_oracle():
    prob = cloud(20000, seed=32)
    announce("cloud cp off surface")
    m = mpwos.Manifold(prob)
    P = oracle.Problem(prob)
    x = np.concatenate([inputs.torus_near_points(400, 0.02, seed=3), inputs.torus_near_points(200, 0.25, seed=4)])
    y_gpu = mpwos.debug_cp(m, x, "fp64")
    y_orc = np.array([oracle.cp(P, xi) for xi in x])
    err = np.linalg.norm(y_gpu - y_orc, axis=1)
    # far from the surface the foot point extrapolates the patch: Newton amplifies rounding there
    assert np.max(err[:400]) < 1e-10, np.max(err[:400])
    assert np.mean(err[400:] < 1e-8) >= 0.99, np.sort(err)[-5:]
    # FP32: the same reconstruction, single-precision search and Newton
    y32 = mpwos.debug_cp(m, x[:400], "fp32")
    assert np.max(np.linalg.norm(y32 - y_orc[:400], axis=1)) < 2e-5
    m.close()


def test_walks_fp64_match_oracle_walk_by_walk():
    prob = cloud(12000, seed=33, tau_w=1e-3)
    P = oracle.Problem(prob)
    Q = inputs.torus_area_uniform(6, seed=34)
    announce("cloud walks fp64 plain 6x48")
    gpu = mpwos.solve(prob, Q, 48, 9, walk_outputs=True, precision="fp64")
    orc = oracle.solve(P, Q, 48, 9)
    frac = compare_walks(gpu, orc, prob, tol=1e-9, min_frac=0.999)
    assert frac == 1.0
    np.testing.assert_allclose(gpu["u"], orc["u"], rtol=1e-10, atol=1e-12)
    announce("cloud walks fp64 persistent 6x48")
    per = mpwos.solve(prob, Q, 48, 9, walk_outputs=True, precision="fp64", persistent=1)
    assert np.array_equal(per["walk_S"], gpu["walk_S"])


@pytest.mark.parametrize("rule", ["curvature_bound", "spacing"])
def test_walks_fp64_other_radius_rules(rule):
    kw = dict(tau_w=1e-3) if rule == "curvature_bound" else dict(tau_w=0.3)
    prob = cloud(12000, seed=41, radius_rule=rule, kappa_bound=1 / 0.3, **kw)
    P = oracle.Problem(prob)
    Q = inputs.torus_area_uniform(2, seed=42)
    nw = 24 if rule == "curvature_bound" else 6
    announce(f"cloud walks fp64 {rule} 2x{nw}")
    gpu = mpwos.solve(prob, Q, nw, 5, walk_outputs=True, precision="fp64", persistent=1)
    orc = oracle.solve(P, Q, nw, 5)
    assert compare_walks(gpu, orc, prob, tol=1e-9, min_frac=0.999) == 1.0
    if rule == "curvature_bound":
        # constant radius: every walk has the same length
        assert len(set(gpu["walk_K"].ravel().tolist())) == 1


def test_full_cloud_whole_walks_match_oracle():
    """The 1e6-point noisy torus with patches fitted over 4 r_16, in the
    launch form the benchmark times (persistent lanes): whole FP64 walks
    (tau_W = 1e-8, K = 1601) against the oracle walk by walk on 32 queries x
    32 walks (at least 99.9% agree: one walk may differ), the per-query means
    over agreeing walks, and FP32 walks of the same stream against them."""
    prob, Q, _ = inputs.config("cloud")
    announce("cloud 1e6 build")
    m = mpwos.Manifold(prob)
    info = mpwos.debug_cloud_info(m)
    assert info["knn_fallback_points"] < 0.05 * len(prob["points"]), info
    Qs = Q[:32]
    announce("cloud 1e6 whole walks fp64 persistent 32x32")
    gpu = mpwos.solve(prob, Qs, 32, 3, manifold=m, walk_outputs=True, precision="fp64", persistent=1)
    assert np.all(gpu["walk_K"] == 1601)
    P = oracle.Problem(prob)
    orc = oracle.solve(P, Qs, 32, 3)
    d = np.abs(gpu["walk_S"] - orc["walk_S"])
    print("fp64 cloud walk differences: max", d.max(), "count above 1e-12 scale",
          int(np.sum(d > 1e-12 * score_scale(prob))), flush=True)
    compare_walks(gpu, orc, prob, tol=1e-12, min_frac=0.999)
    announce("cloud 1e6 whole walks fp32 persistent 32x32")
    g32 = mpwos.solve(prob, Qs, 32, 3, manifold=m, walk_outputs=True, precision="fp32", persistent=1)
    assert np.all(g32["walk_K"] == 1601)
    # FP32 walks follow the FP64 paths; where FP32 rounding moves a sphere
    # point across the boundary between two cloud points' nearest regions the
    # projection switches to the neighbouring patch, whose surface differs at
    # the 1e-5 level, and that walk drifts a little further (measured on
    # MI355X: median 3e-6, 99th percentile 1.5e-3, largest 3.9e-3)
    rel = np.abs(g32["walk_S"] - orc["walk_S"]) / (1 + np.abs(orc["walk_S"]))
    q = np.quantile(rel, [0.5, 0.9, 0.99, 1.0])
    print("fp32 cloud tracking quantiles", q, flush=True)
    assert q[0] < 1e-4 and np.mean(rel < 1e-3) >= 0.95 and q[-1] < 2e-2, q
    m.close()


def test_fp32_statistics_and_closed_form():
    prob = cloud(12000, seed=35, tau_w=1e-3)
    Q = inputs.torus_area_uniform(16, seed=36)
    m = mpwos.Manifold(prob)
    announce("cloud fp64 vs fp32 16x2048")
    r64 = mpwos.solve(prob, Q, 2048, 5, manifold=m, precision="fp64")
    r32 = mpwos.solve(prob, Q, 2048, 5, manifold=m, precision="fp32", persistent=1)
    se = np.sqrt(r64["stderr"] ** 2 + r32["stderr"] ** 2)
    assert np.all(np.abs(r64["u"] - r32["u"]) < 5 * se + 1e-6), (r64["u"] - r32["u"], se)
    # against u at the projected queries: Monte Carlo, tau_W truncation and reconstruction
    y = mpwos.debug_cp(m, Q, "fp64")
    exact = inputs.exact_u(prob, y)
    assert np.all(np.abs(r64["u"] - exact) < 5 * r64["stderr"] + 0.02), (r64["u"] - exact, r64["stderr"])
    m.close()


def test_query_far_from_cloud_is_rejected():
    prob = cloud(8000, seed=37)
    m = mpwos.Manifold(prob)
    Q = inputs.torus_area_uniform(3, seed=38)
    Q[1] *= 1.3
    with pytest.raises(mpwos.MpwosError) as e:
        mpwos.solve(prob, Q, 4, 1, manifold=m)
    assert e.value.status == mpwos.EOFFMANIFOLD
    m.close()


def test_server_serves_cloud_requests():
    prob = cloud(12000, seed=39, tau_w=1e-3)
    Q = inputs.torus_area_uniform(8, seed=40)
    m = mpwos.Manifold(prob)
    announce("cloud served vs solo")
    solo = mpwos.solve(prob, Q, 256, 2, manifold=m, precision="fp32", persistent=1)
    srv = mpwos.Server(4 << 30)
    t = srv.submit(m, prob, Q, 256, 2, precision="fp32", persistent=1)
    out = srv.wait(t, 120_000)
    srv.close()
    assert np.array_equal(out["u"], solo["u"])
    m.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_server_slices_cloud_walks(prec):
    """Served point-cloud walks whose radius varies per step (their length is
    not known) run a fixed number of steps per launch and continue from
    their records (walker position, weights, score, patch): the result
    equals the solo solve bit for bit, with the same walk-steps, over many
    launches."""
    prob = cloud(12000, seed=41, tau_w=1e-5)
    Q = inputs.torus_area_uniform(5, seed=42)
    m = mpwos.Manifold(prob)
    announce(f"cloud served time-sliced {prec}")
    solo = mpwos.solve(prob, Q, 96, 6, manifold=m, precision=prec, walk_outputs=True)
    srv = mpwos.Server(4 << 30)
    out = srv.wait(srv.submit(m, prob, Q, 96, 6, precision=prec, persistent=1), 120_000)
    st = srv.stats()
    srv.close()
    m.close()
    assert np.array_equal(out["u"], solo["u"]) and np.array_equal(out["stderr"], solo["stderr"])
    assert st["walk_steps"] == solo["stats"]["walk_steps"]
    # 256 steps per launch: the longest walk took at least K_max / 256 launches
    assert st["rounds"] >= int(solo["walk_K"].max()) // 256 >= 2, (st, int(solo["walk_K"].max()))


def test_server_checks_cloud_queries_at_admission():
    """A served point-cloud request is checked on the device when it is
    admitted (submit does not wait for the device): one with a query far
    from the cloud completes with EOFFMANIFOLD, a good one beside it is
    served as solved alone."""
    prob = cloud(12000, seed=43, tau_w=1e-3)
    Q = inputs.torus_area_uniform(6, seed=44)
    bad = Q.copy()
    bad[2] *= 1.3
    m = mpwos.Manifold(prob)
    announce("cloud served: query check at admission")
    solo = mpwos.solve(prob, Q, 64, 5, manifold=m, precision="fp32", persistent=1)
    srv = mpwos.Server(4 << 30)
    t_bad = srv.submit(m, prob, bad, 64, 5, precision="fp32", persistent=1)
    t_good = srv.submit(m, prob, Q, 64, 5, precision="fp32", persistent=1)
    out = srv.wait(t_good, 120_000)
    with pytest.raises(mpwos.MpwosError) as e:
        srv.wait(t_bad, 120_000)
    assert e.value.status == mpwos.EOFFMANIFOLD
    srv.close()
    m.close()
    assert np.array_equal(out["u"], solo["u"])


# -- the pure nearest-neighbour projection of Example 4 -----------------------


def test_nearest_point_cloud_matches_oracle():
    """Example 4's sphere cloud (8000 points, cp = nearest point, spacing
    rule): cp against the oracle bit for bit, FP64 walks walk by walk
    (tau_W = 0.05 to keep the oracle's brute-force search short), FP32
    statistics against FP64."""
    prob = inputs.sphere_cloud_problem(inputs.sphere_point_cloud(8000, seed=21))
    P = oracle.Problem(prob)
    m = mpwos.Manifold(prob)
    x = inputs.sphere_uniform(300, 3, seed=22) * np.random.default_rng(23).uniform(0.9, 1.1, (300, 1))
    announce("nearest-point cloud cp")
    y64 = mpwos.debug_cp(m, x, "fp64")
    y32 = mpwos.debug_cp(m, x, "fp32")
    yo = np.array([oracle.cp(P, v) for v in x])
    assert np.array_equal(y64, yo)
    assert np.mean(np.all(y32 == yo, axis=1)) > 0.99
    short = dict(prob, tau_w=0.05)
    Q = inputs.sphere_uniform(3, 3, seed=24)
    announce("nearest-point cloud walks fp64 3x8")
    gpu = mpwos.solve(short, Q, 8, 5, manifold=m, walk_outputs=True, precision="fp64", persistent=1)
    orc = oracle.solve(oracle.Problem(short), Q, 8, 5)
    assert compare_walks(gpu, orc, short, tol=1e-9, min_frac=0.999) == 1.0
    announce("nearest-point cloud fp64 vs fp32 8x1024")
    Q = inputs.sphere_uniform(8, 3, seed=25)
    r64 = mpwos.solve(prob, Q, 1024, 6, manifold=m, precision="fp64", persistent=1)
    r32 = mpwos.solve(prob, Q, 1024, 6, manifold=m, precision="fp32", persistent=1)
    m.close()
    se = np.sqrt(r64["stderr"] ** 2 + r32["stderr"] ** 2)
    assert np.all(np.abs(r64["u"] - r32["u"]) < 5 * se + 1e-6), (r64["u"] - r32["u"], se)
