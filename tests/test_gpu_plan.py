"""GPU tests of the graph-captured solve (mpwos_plan_*) and of the launch
autotuner (mpwos_autotune).  Every replay of a captured graph is compared with
the eager solve of the same arguments, with eager work and synchronisations
between the replays."""
import numpy as np
import pytest

from paper_2606_21883_amd import inputs, mpwos
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("name,opt", [
    ("sphere", dict(precision="fp32", persistent=1)),
    ("cap", dict(precision="fp64")),
    ("hyper10", dict(precision="fp32", persistent=1)),
])
def test_plan_replays_equal_eager_solves(name, opt):
    import torch
    if name == "hyper10":
        prob = dict(inputs.hypersphere_problem(10), tau_w=1e-4)
        qa = inputs.hypersphere_queries(24, 10, seed=1)
        qb = inputs.hypersphere_queries(24, 10, seed=2)
        nw = 96
    else:
        prob, qa, nw = inputs.config(name, scale=0.03)
        _, qb, _ = inputs.config(name, scale=0.03, seed=5)
    m = mpwos.Manifold(prob)
    announce(f"plan {name} {len(qa)}x{nw} {opt}")
    plan = mpwos.Plan(m, prob, len(qa), nw, **opt)
    stream = torch.cuda.current_stream().cuda_stream
    u = torch.zeros(len(qa), dtype=torch.float64, device="cuda")
    se = torch.zeros(len(qa), dtype=torch.float64, device="cuda")
    for Q, seed in [(qa, 3), (qb, 4), (qa, 3), (qb, 9)]:
        dq = _dev(Q)
        plan.execute(dq.data_ptr(), u.data_ptr(), se.data_ptr(), seed, stream)
        torch.cuda.synchronize()
        pst = plan.stats(stream)
        eager = mpwos.solve(prob, Q, nw, seed, manifold=m, **opt)
        assert np.array_equal(u.cpu().numpy(), eager["u"]), (name, seed)
        assert np.array_equal(se.cpu().numpy(), eager["stderr"])
        assert pst["walk_steps"] == eager["stats"]["walk_steps"]
        assert (pst["k_p50"], pst["k_p99"]) == (eager["stats"]["k_p50"], eager["stats"]["k_p99"])
        # unrelated eager work on the same stream between replays
        torch.ones(1 << 20, device="cuda").sum().item()
    plan.close()
    m.close()


def test_plan_rejects_bad_arguments():
    prob, Q, nw = inputs.config("sphere", scale=0.01)
    m = mpwos.Manifold(prob)
    with pytest.raises(mpwos.MpwosError):
        mpwos.Plan(m, dict(prob, sigma=-1.0), len(Q), nw)
    with pytest.raises(mpwos.MpwosError):
        mpwos.Plan(m, prob, 1 << 20, 1 << 20)
    m.close()


def test_autotune_returns_a_working_shape():
    prob, Q, nw = inputs.config("sphere", scale=0.1)
    m = mpwos.Manifold(prob)
    announce("autotune sphere")
    best, ms = mpwos.autotune(prob, Q, nw, manifold=m, precision="fp32")
    assert best["block_size"] in (64, 128, 192, 256) and best["persistent"] in (0, 1) and ms > 0
    # block size and launch form do not change the walks
    a = mpwos.solve(prob, Q, nw, 5, manifold=m, precision="fp32", **best)
    b = mpwos.solve(prob, Q, nw, 5, manifold=m, precision="fp32")
    assert np.array_equal(a["u"], b["u"])
    m.close()
    prob = dict(inputs.hypersphere_problem(100), tau_w=1e-3)
    Q = inputs.hypersphere_queries(16, 100, seed=1)
    m = mpwos.Manifold(prob)
    announce("autotune hyper100")
    best, ms = mpwos.autotune(prob, Q, 64, manifold=m, precision="fp32")
    assert best["lanes_per_walk"] in (4, 8, 16, 32, 64)
    a = mpwos.solve(prob, Q, 64, 5, manifold=m, precision="fp32", **best)
    b = mpwos.solve(prob, Q, 64, 5, manifold=m, precision="fp32")
    # lane groups of another width sum coordinates in another order
    np.testing.assert_allclose(a["u"], b["u"], rtol=1e-4, atol=1e-6)
    m.close()
