"""GPU test of the allocation-free solve (mpwos_solve_noalloc): called
through the C ABI with device-resident queries and outputs, it must give the
same bits as mpwos_solve on the same arguments, on two calls in a row (the
second smaller), with its inverse table and per-walk scores in the fixed
device array and the queries cut into batches that fit it."""
import numpy as np
import pytest

from paper_2606_21883_amd import inputs, mpwos
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

LIMIT_WALKS = (64 * 2 ** 20 - 2 ** 20 - 8) // 12


def _noalloc(m, prob, Q, nw, seed, stderr=True, walks=False, **opt):
    import torch
    dq = torch.from_numpy(np.ascontiguousarray(Q)).to("cuda")
    u = torch.full((len(Q),), float("nan"), dtype=torch.float64, device="cuda")
    se = torch.full((len(Q),), float("nan"), dtype=torch.float64, device="cuda")
    wS = torch.zeros((len(Q), nw), dtype=torch.float64, device="cuda") if walks else None
    wK = torch.zeros((len(Q), nw), dtype=torch.int32, device="cuda") if walks else None
    stream = torch.cuda.current_stream().cuda_stream
    st = mpwos.solve_noalloc(m, prob, dq.data_ptr(), len(Q), nw, seed, u.data_ptr(),
                             se.data_ptr() if stderr else 0, stream,
                             wS.data_ptr() if walks else None, wK.data_ptr() if walks else None, **opt)
    torch.cuda.synchronize()
    out = dict(u=u.cpu().numpy(), stderr=se.cpu().numpy(), stats=st)
    if walks:
        out.update(walk_S=wS.cpu().numpy(), walk_K=wK.cpu().numpy())
    return out


def test_noalloc_equals_solve_on_two_calls():
    # sigma values no other test uses, so the first call builds its inverse
    # table in the fixed array rather than finding it cached
    big = dict(inputs.sphere_problem(), sigma=2.3)
    small = dict(inputs.cap_problem(), sigma=0.55)
    Qa = inputs.sphere_uniform(2048, 3, seed=11)
    Qb = inputs.cap_uniform(96, 3, 0.0, seed=12)
    ma, mb = mpwos.Manifold(big), mpwos.Manifold(small)
    # 2048 x 4096 walks: more than one batch of the array (5.5e6 walks)
    announce("noalloc sphere 2048x4096 fp32 persistent")
    a = _noalloc(ma, big, Qa, 4096, 5, precision="fp32", persistent=1)
    announce("noalloc cap 96x256 fp64, walk outputs, no stderr")
    b = _noalloc(mb, small, Qb, 256, 6, stderr=False, walks=True, precision="fp64")
    announce("solve sphere / cap for comparison")
    ra = mpwos.solve(big, Qa, 4096, 5, manifold=ma, precision="fp32", persistent=1)
    rb = mpwos.solve(small, Qb, 256, 6, manifold=mb, walk_outputs=True, precision="fp64")
    assert np.array_equal(a["u"], ra["u"]) and np.array_equal(a["stderr"], ra["stderr"])
    assert a["stats"]["walk_steps"] == ra["stats"]["walk_steps"]
    assert a["stats"]["k_max"] == ra["stats"]["k_max"]
    assert (a["stats"]["k_p50"], a["stats"]["k_p99"]) == (ra["stats"]["k_p50"], ra["stats"]["k_p99"])
    assert np.array_equal(b["u"], rb["u"])
    assert np.array_equal(b["walk_S"], rb["walk_S"]) and np.array_equal(b["walk_K"], rb["walk_K"])
    assert b["stats"]["walk_steps"] == rb["stats"]["walk_steps"]
    # the same problems again, smaller, in the other order: the array now
    # holds the cap's table, the cache the sphere's
    announce("noalloc repeat smaller")
    a2 = _noalloc(ma, big, Qa[:100], 64, 7, precision="fp32", persistent=1)
    ra2 = mpwos.solve(big, Qa[:100], 64, 7, manifold=ma, precision="fp32", persistent=1)
    assert np.array_equal(a2["u"], ra2["u"]) and np.array_equal(a2["stderr"], ra2["stderr"])
    b2 = _noalloc(mb, small, Qb[:10], 32, 8, precision="fp32")
    rb2 = mpwos.solve(small, Qb[:10], 32, 8, manifold=mb, precision="fp32")
    assert np.array_equal(b2["u"], rb2["u"]) and np.array_equal(b2["stderr"], rb2["stderr"])
    ma.close()
    mb.close()


def test_noalloc_group_kernel_and_point_cloud():
    prob = dict(inputs.hypersphere_problem(10), tau_w=1e-4)
    Q = inputs.hypersphere_queries(64, 10, seed=3)
    m = mpwos.Manifold(prob)
    announce("noalloc hypersphere n=10 64x512 fp32, then 8x64 fp64")
    for nq, nw, prec in ((64, 512, "fp32"), (8, 64, "fp64")):
        a = _noalloc(m, prob, Q[:nq], nw, 4, precision=prec)
        r = mpwos.solve(prob, Q[:nq], nw, 4, manifold=m, precision=prec)
        assert np.array_equal(a["u"], r["u"]) and np.array_equal(a["stderr"], r["stderr"])
    m.close()
    pts = inputs.torus_point_cloud(20000, 1.0, 0.3, 0.0, seed=4)
    cprob = inputs.point_cloud_problem(pts, radius_rule="curvature_bound", kappa_bound=1.0 / 0.3)
    cq = inputs.torus_area_uniform(32, 1.0, 0.3, seed=5)
    cm = mpwos.Manifold(cprob)
    announce("noalloc point cloud 32x64 fp64, then 4x16")
    for nq, nw in ((32, 64), (4, 16)):
        a = _noalloc(cm, cprob, cq[:nq], nw, 2, precision="fp64")
        r = mpwos.solve(cprob, cq[:nq], nw, 2, manifold=cm, precision="fp64")
        assert np.array_equal(a["u"], r["u"]) and np.array_equal(a["stderr"], r["stderr"])
    cm.close()


def test_noalloc_rejects_beyond_its_limits():
    prob = inputs.sphere_problem()
    Q = inputs.sphere_uniform(2, 3, seed=1)
    m = mpwos.Manifold(prob)
    announce("noalloc limits")
    with pytest.raises(mpwos.MpwosError) as ei:
        _noalloc(m, prob, Q, LIMIT_WALKS + 1, 0)
    assert ei.value.status == mpwos.EINVAL and "allocation-free" in str(ei.value)
    bad = Q.copy()
    bad[1] *= 1.01
    with pytest.raises(mpwos.MpwosError) as ei:
        _noalloc(m, prob, bad, 16, 0)
    assert ei.value.status == mpwos.EOFFMANIFOLD
    # at the limit a single query runs
    r = _noalloc(m, prob, Q[:1], LIMIT_WALKS, 0, stderr=False, precision="fp32")
    assert np.isfinite(r["u"][0])
    m.close()
