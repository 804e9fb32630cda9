"""GPU tests of the continuous-batching server (mpwos_server_*): each request's
result in a mix equals the same solve run alone, bit for bit; admission by HBM
budget; requests that arrive while others run join them."""
import time

import numpy as np
import pytest

from paper_2606_21883_amd import inputs, mpwos
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def mix():
    out = []
    p, Q, _ = inputs.config("sphere", scale=0.05)
    out.append((p, Q, 257, 11, dict(precision="fp32", persistent=1)))
    p, Q, _ = inputs.config("cap", scale=0.05)
    out.append((p, Q, 300, 12, dict(precision="fp32", persistent=1)))
    p, Q, _ = inputs.config("torus", scale=0.01)
    out.append((p, Q, 64, 13, dict(precision="fp64")))
    p = inputs.hypersphere_problem(10)
    out.append((p, inputs.hypersphere_queries(40, 10, seed=3), 100, 14, dict(precision="fp32")))
    p, Q, _ = inputs.config("circle", scale=0.5)
    out.append((p, Q, 333, 15, dict(precision="fp64", persistent=1)))
    p = dict(inputs.hypersphere_problem(100), tau_w=1e-3)
    out.append((p, inputs.hypersphere_queries(6, 100, seed=3), 16, 16, dict(precision="fp32")))
    return out


def test_served_results_equal_solo_results():
    reqs = mix()
    announce("server mix solo")
    solo = [mpwos.solve(p, Q, nw, seed, **kw) for p, Q, nw, seed, kw in reqs]
    announce("server mix served")
    mans = [mpwos.Manifold(p) for p, *_ in reqs]
    srv = mpwos.Server(8 << 30)
    tickets = [srv.submit(m, p, Q, nw, seed, **kw) for m, (p, Q, nw, seed, kw) in zip(mans, reqs)]
    outs = [srv.wait(t, 120_000) for t in tickets]
    st = srv.stats()
    srv.close()
    for s, o, (p, *_ ) in zip(solo, outs, reqs):
        assert np.array_equal(s["u"], o["u"]), p["manifold"]
        assert np.array_equal(s["stderr"], o["stderr"])
    assert st["completed"] == len(reqs) and st["admitted"] == len(reqs)
    assert st["walk_steps"] > 0 and st["rounds"] >= 1
    for m in mans:
        m.close()


def test_budget_rejects_and_queues():
    p, Q, _ = inputs.config("sphere", scale=0.02)
    m = mpwos.Manifold(p)
    need = len(Q) * 3 * 8 + len(Q) * 2048 * 12 + 4096
    assert need > 1 << 20
    srv = mpwos.Server(int(need * 1.5))
    with pytest.raises(mpwos.MpwosError) as e:
        srv.submit(m, p, np.repeat(Q, 40, axis=0), 2048, 1, precision="fp32")
    assert e.value.status == mpwos.ENOMEM
    # three requests that fit only one at a time all complete, in order
    announce("server budget queue")
    ts = [srv.submit(m, p, Q, 2048, s, precision="fp32") for s in (1, 2, 3)]
    outs = [srv.wait(t, 120_000) for t in ts]
    st = srv.stats()
    srv.close()
    assert st["rejected"] == 1 and st["completed"] == 3
    alone = mpwos.solve(p, Q, 2048, 2, precision="fp32")
    assert np.array_equal(alone["u"], outs[1]["u"])
    m.close()


def test_late_arrival_joins_running_work():
    big, Qb, _ = inputs.config("sphere", scale=0.25)
    small, Qs, _ = inputs.config("cap", scale=0.02)
    mb, ms = mpwos.Manifold(big), mpwos.Manifold(small)
    announce("server late arrival")
    srv = mpwos.Server(16 << 30, slice_walk_steps=1 << 24)
    tb = srv.submit(mb, big, Qb, 1024, 5, precision="fp64")
    time.sleep(0.05)
    ts = srv.submit(ms, small, Qs, 256, 6, precision="fp32", persistent=1)
    t0 = time.perf_counter()
    os_ = srv.wait(ts, 120_000)
    t_small = time.perf_counter() - t0
    done_big, _ = srv.poll(tb)
    ob = srv.wait(tb, 120_000)
    st = srv.stats()
    srv.close()
    assert st["rounds"] >= 2
    # the small request did not wait for the big one to finish
    assert not done_big or t_small < 1.0
    assert np.array_equal(os_["u"], mpwos.solve(small, Qs, 256, 6, precision="fp32", persistent=1)["u"])
    assert np.array_equal(ob["u"], mpwos.solve(big, Qb, 1024, 5, precision="fp64")["u"])
    mb.close()
    ms.close()


def test_manifold_busy_while_referenced():
    p, Q, _ = inputs.config("sphere", scale=0.02)
    m = mpwos.Manifold(p)
    srv = mpwos.Server(4 << 30)
    t = srv.submit(m, p, Q, 4096, 1, precision="fp64")
    with pytest.raises(mpwos.MpwosError) as e:
        m.close()
    assert e.value.status == mpwos.EBUSY
    srv.wait(t, 120_000)
    srv.close()
    m.close()


def test_invalid_requests_are_rejected_at_submit():
    p, Q, _ = inputs.config("sphere", scale=0.01)
    m = mpwos.Manifold(p)
    srv = mpwos.Server(1 << 30)
    with pytest.raises(mpwos.MpwosError) as e:
        srv.submit(m, dict(p, sigma=-1.0), Q, 16, 1)
    assert e.value.status == mpwos.EINVAL
    with pytest.raises(mpwos.MpwosError):
        srv.submit(m, p, Q, 0, 1)
    assert srv.stats()["rejected"] == 2
    srv.close()
    m.close()


def test_small_requests_share_launches():
    """Many small requests of a few classes (same manifold and problem; their
    own queries, walk counts and seeds) run in shared launches: far fewer
    launches than requests, and every result equals its solo solve bit for
    bit.  Covers the lane kernels (FP32 closed sphere, FP64 cap with two Green
    samples, whose walks have uneven lengths), the lane-group kernel at
    n = 100 (eight walks per wavefront) and TABLE_S1 sources (one class per
    request)."""
    sph, _, _ = inputs.config("sphere", scale=0.01)
    cap = dict(inputs.cap_problem(), n_v=2)
    hyp = dict(inputs.hypersphere_problem(100), tau_w=1e-3)
    M = 64
    th = 2 * np.pi * np.arange(M) / M
    f = np.exp(np.cos(th))
    tab = inputs.problem(manifold="sphere", n=2, p=[1.0], sigma=1.0,
                         f=dict(kind="table_s1", values=np.concatenate([f, f / 2.0])))
    kinds = [(sph, dict(precision="fp32", persistent=1)), (cap, dict(precision="fp64")),
             (hyp, dict(precision="fp32")), (tab, dict(precision="fp64"))]
    mans = [mpwos.Manifold(p) for p, _ in kinds]
    rng = np.random.default_rng(8)
    reqs = []
    for i in range(48):
        j = i % 4
        p, kw = kinds[j]
        nq = int(rng.integers(1, 6))
        qs = int(rng.integers(1 << 20))
        if j == 0:
            Q = inputs.sphere_uniform(nq, 3, qs)
        elif j == 1:
            Q = inputs.cap_uniform(nq, 3, 0.0, qs)
        elif j == 2:
            Q = inputs.hypersphere_queries(max(nq, 2), 100, qs)
        else:
            t = np.random.default_rng(qs).uniform(0, 2 * np.pi, nq)
            Q = np.stack([np.cos(t), np.sin(t)], 1)
        nw = int(rng.integers(1, 100)) if j != 2 else int(rng.integers(1, 12))
        reqs.append((j, Q, nw, int(rng.integers(1 << 62))))
    announce("server small requests served")
    srv = mpwos.Server(8 << 30)
    # a long request of another class holds the launch slots (8 launches of
    # 32768 walks) while the small ones arrive, so these queue up and share
    blocker = srv.submit(mans[2], hyp, inputs.hypersphere_queries(64, 100, 99), 4096, 1, precision="fp64")
    tickets = [srv.submit(mans[j], kinds[j][0], Q, nw, sd, **kinds[j][1]) for j, Q, nw, sd in reqs]
    outs = [srv.wait(t, 120_000) for t in tickets]
    srv.wait(blocker, 120_000)
    st = srv.stats()
    srv.close()
    announce("server small requests solo")
    for (j, Q, nw, sd), o in zip(reqs, outs):
        p, kw = kinds[j]
        solo = mpwos.solve(p, Q, nw, sd, manifold=mans[j], **kw)
        assert np.array_equal(solo["u"], o["u"]), (j, len(Q), nw)
        assert np.array_equal(solo["stderr"], o["stderr"]), (j, len(Q), nw)
    assert st["completed"] == len(reqs) + 1
    # the 36 requests of the three shared classes go out in a few launches;
    # the 12 TABLE_S1 requests each form a class of their own
    assert st["rounds"] < 8 + 12 + 18, st
    for m in mans:
        m.close()


@pytest.mark.parametrize("n,tau_w,prec", [(1000, 1e-3, "fp32"), (200, 1e-8, "fp64")])
def test_long_walks_are_time_sliced(n, tau_w, prec):
    """Lane-group walks longer than the per-launch step budget save their state
    and continue in later launches: the served result still equals the solo
    solve bit for bit, and the request took many launches.  At n = 200 a
    wavefront holds four walks, so ranges resume with padding."""
    p = dict(inputs.hypersphere_problem(n), tau_w=tau_w)
    Q = inputs.hypersphere_queries(3, n, seed=4)
    m = mpwos.Manifold(p)
    announce(f"server time-sliced S^{n - 1} {prec}")
    solo = mpwos.solve(p, Q, 7, 21, manifold=m, precision=prec)
    srv = mpwos.Server(4 << 30)
    out = srv.wait(srv.submit(m, p, Q, 7, 21, precision=prec), 120_000)
    st = srv.stats()
    srv.close()
    m.close()
    assert np.array_equal(solo["u"], out["u"]) and np.array_equal(solo["stderr"], out["stderr"])
    assert st["walk_steps"] == solo["stats"]["walk_steps"]
    k = solo["stats"]["walk_steps"] / (len(Q) * 7)
    budget = max(256, 1e6 / (1 + 2 * ((n + 3) // 4)))
    assert st["rounds"] >= int(k // budget), (st, k, budget)
