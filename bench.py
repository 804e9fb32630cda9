"""Benchmark of the MPWoS hot path on one MI355X.

One step = one pass of the whole walk path over the unit-sphere workload:
  - S^2 closed, u = x1 x2, sigma = 2, f = 8 x1 x2: 4096 queries x 4096 walks;
  - S^2 cap x3 > 0, Dirichlet g = u, sigma = 0.5, eps = 1e-3: 4096 x 4096 walks;
in the FP32-mixed persistent form (FP32 walk arithmetic, FP64 weights,
scores and per-query compensated sums).  Queries and outputs are resident in
device memory when the timed region starts.

metric: walk-steps/s (one walk-step = one iteration of Algorithm 1 with its
N_V = 1 Green sample), with queries/s and the closed-form RMSE beside it.
The same workload in the plain one-launch-per-solve FP64 form, and the FP64
CPU oracle on a bounded sample of the workload, are reported for comparison.

The roofline of the dominant kernel (the closed-sphere FP32 walk) is the
VALU issue rate: the algorithmic operations of one walk-step (step_ops) are
weighted by their measured issue cost relative to a full-rate FP32 FMA
(valu_weights, from the library's VALU probe run live) and divided by the
kernel's time from HIP events on its stream; the peak is 256 CUs x 128
FP32 lanes per clock x 2.4 GHz (157.3 TFLOP/s counted per FMA).

Other workloads (--workload) time the remaining configurations in the same
way for profiling; they are not the headline line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walk-steps/s and queries/s at fixed RMSE vs FP64 oracle; served p50/p99 ms"
# Full-rate VALU lane-operations per second: 256 CUs x 128 FP32 FMA lanes per
# clock x 2.4 GHz, the published FP32 vector peak (157.3 TFLOP/s) counted per
# FMA.  The VALU probe reaches about 72% of it with a pure fma_f32 stream.
PEAK_SLOTS = 256 * 128 * 2.4e9

# HBM bytes of one launch of the closed-sphere FP32 walk kernel on the
# headline workload (4096 x 4096 walks, plain lanes, 256 per block), from rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE (KiB per dispatch), each scaled by the reading of a plain
# copy kernel of known size (FETCH_SIZE reads half the bytes a copy moves,
# WRITE_SIZE all of them).  Valid only for the kernel sources they were taken
# on (their SHA-256 below); any change to those sources makes traffic null.
TRAFFIC = {
    "kernel_sha256": "c4481decb522f947feff325db9346fe6eb900aca5d827fef52cf3a80aef3511c",
    "fetch_kib": 456.1875, "fetch_factor": 2.0,
    "write_kib": 196608.0, "write_factor": 1.0,
}
KERNEL_SOURCES = ["walk_lane.hip", "mpwos_dev.h", "kernel_args.h", "cloud_dev.h"]


def kernel_sha256():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_21883_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def step_ops(kind, n, n_v=1):
    """Algorithmic VALU operations of one FP32-mixed walk-step (n <= 3, one lane
    per walk), by issue class.  Counts what the method as specified must do:
      - Philox4x32-10 blocks: one for the direction and one per Green sample
        (direction words and the radius word); 10 rounds of two 32x32->64
        multiplies and two three-way xors per block (one v_bitop3_b32 each;
        the key schedule is scalar);
      - two operations per uniform; per direction cos and sin of the angle,
        and on S^2 the axis coordinate and its radius (one square root, three
        multiply-adds, two multiplies; the kernel folds the step's scale into
        the radius, which the count does not credit);
      - per n-vector update Y + r zeta (n) and projection: a squared norm (n),
        a reciprocal square root and the scaling (n + 1), for Theta and for
        each Green point Z;
      - the Green radius from the inverse-CDF table (w = sqrt(min(u, 1-u)),
        index, two loads, one interpolation);
      - the source (the pair product, its compensation with one reciprocal);
      - FP64: F to FP64 and its 1/N_V, W omega, the score update (a plain
        FP64 sum in this mode), W c, the stop test.
    """
    sets = 1 + n_v                        # the direction of Theta and each Green sample
    ops = {"mad_u64_u32": 20 * sets, "bitop3_b32": 20 * sets, "f32": 0, "trans": 0, "f64": 6}
    words = (n - 1) + n_v * n             # direction words, plus the radius word per sample
    ops["f32"] += 2 * words
    ops["trans"] += sets * (3 if n == 3 else 2)
    ops["f32"] += sets * (5 if n == 3 else 0)
    ops["f32"] += sets * (3 * n + 1)      # update and projection
    ops["trans"] += sets
    ops["f32"] += n_v * (10 + 8)          # radius table, source
    ops["trans"] += n_v * (1 + 1)
    ops["f32"] += 2                       # step counter and bound
    if kind == "cap":
        ops["f32"] += 25 + 8              # delta_Gamma, two-slice table
        ops["trans"] += 2
        ops["f64"] += 40                  # per-step weight series and radial norm
    return ops


def valu_weights():
    """Issue cost of each operation class relative to fma_f32, from the VALU
    probe: isolated rates for xor and FP64, and for transcendentals and the
    64-bit multiply-add the extra time they add beside three independent FMAs
    (the walk interleaves them with other work)."""
    from paper_2606_21883_amd import mpwos
    r = {op: mpwos.valu_probe(op) for op in mpwos.VALU_OPS}
    base = r["fma_f32"]

    def mixed(name):
        return max(0.0, (4.0 / r[name] - 3.0 / base) * base)

    w = {"f32": 1.0, "bitop3_b32": base / r["bitop3_b32"], "f64": base / r["fma_f64"],
         "trans": mixed("sin_f32+3fma"), "mad_u64_u32": mixed("mad_u64_u32+3fma")}
    return w, r


def make_workload(name, scale=1.0):
    from paper_2606_21883_amd import inputs
    if name == "sphere":
        ps, Qs, nws = inputs.config("sphere", scale)
        pc, Qc, nwc = inputs.config("cap", scale)
        return [("sphere", ps, Qs, nws), ("cap", pc, Qc, nwc)]
    p, Q, nw = inputs.config(name, scale)
    return [(name, p, Q, nw)]


def parse_launch(spec):
    """NAME=FORM:BLOCK[,...] (FORM plain or persistent) -> {NAME: launch options}."""
    out = {}
    for part in filter(None, (spec or "").split(",")):
        name, shape = part.split("=")
        form, block = shape.split(":")
        out[name] = {"persistent": 1 if form == "persistent" else 0, "block_size": int(block)}
    return out


def run_gpu(work, steps, warmup, precision, persistent, block_size=0, graph=False, tune=False, launch=None):
    """Times `steps` passes over the workload.  graph: each solve is a captured
    plan (mpwos_plan_*) replayed per step, with its device time from HIP events
    around the replay on the launch stream; otherwise one mpwos_solve per solve
    and step, with the library's own kernel time.  tune: the launch shape of
    each solve comes from mpwos_autotune first (untimed)."""
    import torch

    from paper_2606_21883_amd import inputs, mpwos
    dev = torch.device("cuda:0")
    # a stream of its own (default priority): torch's events and the library's
    # launches then share it (the legacy default stream has handle 0, which the
    # library would read as "use your own stream")
    tstream = torch.cuda.Stream()
    torch.cuda.set_stream(tstream)
    stream = tstream.cuda_stream
    items = []
    for name, prob, Q, nw in work:
        m = mpwos.Manifold(prob)
        opt = dict(precision=precision, persistent=persistent, block_size=block_size)
        if launch and name in launch:
            opt.update(launch[name])
        elif tune:
            # a predictor pipeline is tuned on its baseline solve (same kernel, m_* = 0)
            tprob = dict(prob, compensation="none") if "predictor_grid" in prob else prob
            best, _ = mpwos.autotune(tprob, Q, nw, manifold=m, precision=precision)
            opt.update(best)
            print(f"[bench] {name}: tuned launch shape {best}", file=sys.stderr, flush=True)
        q = torch.from_numpy(np.ascontiguousarray(Q)).to(dev)
        u = torch.zeros(len(Q), dtype=torch.float64, device=dev)
        se = torch.zeros(len(Q), dtype=torch.float64, device=dev)
        # a predictor pipeline (second-order compensation) refits u_* every
        # step, so its solve cannot be one captured plan
        pipeline = "predictor_grid" in prob
        plan = mpwos.Plan(m, prob, len(Q), nw, **opt) if graph and not pipeline else None
        items.append(dict(name=name, prob=prob, q=q, nw=nw, m=m, u=u, se=se, opt=opt, plan=plan))

    def pipeline_step(it):
        """Predictor fit (coarse baseline solve at the nodes and the series
        fit, on the device) and then the compensated solve."""
        g = it["prob"]["predictor_grid"]
        coef, pst = mpwos.predictor_fit(it["prob"], g["nt"], g["ns"], g["n_walks"], 1, g["ks"], g["kt"],
                                        manifold=it["m"], stream=stream, **it["opt"])
        prob = dict(it["prob"], predictor=dict(idx=[g["ks"], g["kt"]], values=coef.ravel()))
        sst = mpwos.solve_device(it["m"], prob, it["q"].data_ptr(), it["q"].shape[0], it["nw"], 0,
                                 it["u"].data_ptr(), it["se"].data_ptr(), stream=stream, **it["opt"])
        it["last_predictor"] = coef
        return dict(sst, kernel_ms=sst["kernel_ms"] + pst["kernel_ms"],
                    walk_steps=sst["walk_steps"] + pst["walk_steps"], predictor_walk_steps=pst["walk_steps"],
                    predictor_kernel_ms=pst["kernel_ms"])

    def one_step():
        st = []
        for it in items:
            if it["plan"] is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(tstream)
                it["plan"].execute(it["q"].data_ptr(), it["u"].data_ptr(), it["se"].data_ptr(), 0, stream)
                e1.record(tstream)
                st.append((e0, e1))
            elif "predictor_grid" in it["prob"]:
                st.append(pipeline_step(it))
            else:
                st.append(mpwos.solve_device(it["m"], it["prob"], it["q"].data_ptr(), it["q"].shape[0], it["nw"], 0,
                                             it["u"].data_ptr(), it["se"].data_ptr(), stream=stream, **it["opt"]))
        return st

    t0 = time.perf_counter()
    for i in range(warmup):
        one_step()
        torch.cuda.synchronize()
        print(f"[bench] {precision} warmup {i + 1}/{warmup} {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(steps):
        stats.append(one_step())
        print(f"[bench] {precision} step {i + 1}/{steps} queued {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = {"seconds": dt, "steps": steps, "form": ("graph replay" if graph else "mpwos_solve per step") +
           (", autotuned launch shape" if tune else "")}
    per = {}
    total_ws = 0
    for i, it in enumerate(items):
        if it["plan"] is not None:
            kms = float(np.mean([s[i][0].elapsed_time(s[i][1]) for s in stats]))
            pst = it["plan"].stats(stream)
            ws, k_mean = pst["walk_steps"], pst["k_mean"]
        else:
            kms = float(np.mean([s[i]["kernel_ms"] for s in stats]))
            ws, k_mean = stats[0][i]["walk_steps"], stats[0][i]["k_mean"]
        total_ws += ws
        Qh = it["q"].cpu().numpy()
        if it["prob"]["manifold"] == "point_cloud":
            Qh = mpwos.debug_cp(it["m"], Qh, "fp64")       # the estimate refers to cp_h(q)
        exact = inputs.exact_u(it["prob"], Qh)
        per[it["name"]] = {"kernel_ms": kms, "walk_steps": ws, "k_mean": k_mean,
                           "walk_steps_per_s": ws / (kms * 1e-3),
                           "rmse": inputs.rmse(it["u"].cpu().numpy(), exact),
                           "mean_stderr": float(np.sqrt(np.mean(it["se"].cpu().numpy() ** 2))),
                           "n_queries": int(it["q"].shape[0]), "n_walks": int(it["nw"]),
                           "launch": {k: v for k, v in it["opt"].items() if k != "precision"}}
        if "predictor_grid" in it["prob"]:
            per[it["name"]].update(
                predictor_walk_steps=stats[0][i]["predictor_walk_steps"],
                predictor_kernel_ms=float(np.mean([s[i]["predictor_kernel_ms"] for s in stats])),
                compensation_legs=compensation_legs(it, stream))
    res["walk_steps_per_step"] = total_ws
    res["per"] = per
    for it in items:
        if it["plan"] is not None:
            it["plan"].close()
        it["m"].close()
    torch.cuda.synchronize()
    torch.cuda.set_stream(torch.cuda.default_stream())
    return res


def compensation_legs(it, stream):
    """Untimed: the same solve with m_* = 0 (the baseline) and with the exact m,
    beside the timed second-order solve, scored against the closed-form u
    (Example 1's comparison; the three share their random numbers)."""
    from paper_2606_21883_amd import inputs, mpwos
    Qh = it["q"].cpu().numpy()
    exact = inputs.exact_u(it["prob"], Qh)
    out = {"second_order": {"rmse": inputs.rmse(it["u"].cpu().numpy(), exact)}}
    for comp in ("none", "exact"):
        prob = {k: v for k, v in it["prob"].items() if k != "predictor_grid"}
        prob["compensation"] = comp
        r = mpwos.solve(prob, Qh, it["nw"], 0, manifold=it["m"], **it["opt"])
        out[comp] = {"rmse": inputs.rmse(r["u"], exact), "mean_stderr": float(np.sqrt(np.mean(r["stderr"] ** 2)))}
    return out


def host_io_rate(work, per, steps=3):
    """The same step through mpwos_solve with host (numpy) queries and outputs:
    each solve copies its queries in and its estimates out over PCIe inside
    the call.  Reported beside the device-resident value, never as it."""
    from paper_2606_21883_amd import mpwos
    items = []
    for name, prob, Q, nw in work:
        m = mpwos.Manifold(prob)
        opt = {k: v for k, v in per[name]["launch"].items() if k in ("persistent", "block_size", "lanes_per_walk")}
        items.append((m, prob, np.ascontiguousarray(Q), nw, opt))
    for m, prob, Q, nw, opt in items:  # warm-up
        mpwos.solve(prob, Q, nw, 0, manifold=m, precision="fp32", **opt)
    t0 = time.perf_counter()
    ws = 0
    for _ in range(steps):
        for m, prob, Q, nw, opt in items:
            ws += mpwos.solve(prob, Q, nw, 0, manifold=m, precision="fp32", **opt)["stats"]["walk_steps"]
    dt = time.perf_counter() - t0
    for it in items:
        it[0].close()
    return {"value": ws / dt, "unit": "walk-steps/s", "ms_per_step": 1e3 * dt / steps,
            "form": "mpwos_solve per solve with host buffers (PCIe copies and the host query check inside)"}


def compensation_sweep(walks):
    """Example 1's comparison as a function of the walk count N: the same 100
    points solved with m_* = 0, with the second-order m_* from one device
    predictor fit, and with the exact m, each scored against the closed-form
    u (the three share their random numbers at each N)."""
    from paper_2606_21883_amd import inputs, mpwos
    prob, Q, _ = inputs.config("cut_torus")
    g = prob["predictor_grid"]
    base = {k: v for k, v in prob.items() if k != "predictor_grid"}
    exact = inputs.exact_u(base, Q)
    m = mpwos.Manifold(base)
    coef, _ = mpwos.predictor_fit(base, g["nt"], g["ns"], g["n_walks"], 1, g["ks"], g["kt"], manifold=m,
                                  precision="fp32", persistent=1)
    rows = []
    for nw in walks:
        row = {"n_walks": nw}
        for comp in ("none", "second_order", "exact"):
            pr = dict(base, compensation=comp)
            if comp == "second_order":
                pr["predictor"] = dict(idx=[g["ks"], g["kt"]], values=coef.ravel())
            r = mpwos.solve(pr, Q, nw, 0, manifold=m, precision="fp32", persistent=1)
            row[comp] = {"rmse": inputs.rmse(r["u"], exact), "mean_stderr": float(np.sqrt(np.mean(r["stderr"] ** 2)))}
        print(f"[bench] compensation sweep N={nw}: " + ", ".join(f"{k} {row[k]['rmse']:.4g}"
              for k in ("none", "second_order", "exact")), file=sys.stderr, flush=True)
        rows.append(row)
    m.close()
    return {"workload": "cut torus (Example 1), 100 points, N_V = 50, eps = 1e-5, FP32", "sweep": rows}


def cpu_baseline(work):
    """The FP64 oracle on the host cores over a bounded sample of the workload
    (about 10-20 s of CPU work)."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    sample = {"sphere": (64, 4096), "cap": (64, 4096), "dumbbell": (1, 32), "sphere_cloud": (2, 8), "product": (4, 64)}
    total_steps, total_t, parts = 0, 0.0, []
    for name, prob, Q, nw in work:
        nq, nws = sample.get(name, (8, 256))
        t0 = time.perf_counter()
        k = 0
        if "predictor_grid" in prob:
            # the oracle's own pipeline, shrunk: a coarse baseline solve at
            # 8 x 3 nodes, its series fit, then the compensated solve
            from paper_2606_21883_amd import inputs
            base = {kk: v for kk, v in prob.items() if kk != "predictor_grid"}
            rc = oracle.solve(dict(base, compensation="none"), inputs.cut_torus_nodes(8, 4), 16, 1, threads=threads)
            coef = oracle.ts_fit(rc["u"].reshape(8, 3), 2, 2)
            prob = dict(base, predictor=dict(idx=[2, 2], values=coef))
            k += int(rc["walk_K"].sum())
        r = oracle.solve(prob, Q[:nq], nws, 0, threads=threads)
        dt = time.perf_counter() - t0
        k += int(r["walk_K"].sum())
        total_steps += k
        total_t += dt
        parts.append(f"{name}: {nq} queries x {nws} walks ({k} walk-steps, {dt:.1f} s)")
    return {"value": total_steps / total_t, "unit": "walk-steps/s", "cores": threads, "kind": "oracle",
            "sample": "; ".join(parts)}


# Served mix: manifolds of the S^1, S^2 (closed and cap), S^99, S^999 and
# implicit-torus configurations with their walk lengths K at tau_W = 1e-8.
SERVED_KINDS = {"circle": 232, "sphere": 174, "cap": 29, "torus": 1601, "hyper100": 11340, "hyper1000": 113393}


def served_mix(rate=200.0, window=3.0, seed=2, work_range=(1e4, 1e7), q_range=(1, 16), min_walks=8, solo=True):
    """Poisson arrivals at `rate` per second for `window` seconds, served by the
    continuous-batching server (FP32 persistent kernels).  Each request draws a
    manifold uniformly, a query count log-uniform in q_range and a total work
    log-uniform in work_range walk-steps (walks per query = work / (queries K),
    at least min_walks).  Latency = completion - arrival.  Every estimate is
    checked against the closed-form solution at its query.  With `solo`, the
    same requests run alone and first-in first-out through mpwos_solve give
    the per-solve comparison (its latencies from the measured service times)
    and the bitwise check."""
    import torch  # noqa: F401  (one HIP runtime with torch)

    from paper_2606_21883_amd import inputs, mpwos
    rng = np.random.default_rng(seed)
    probs, mans = {}, {}
    for name in SERVED_KINDS:
        p, _, _ = inputs.config(name, 1.0 / 1024)
        probs[name] = p
        mans[name] = mpwos.Manifold(p)
    t, reqs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window:
            break
        name = list(SERVED_KINDS)[rng.integers(len(SERVED_KINDS))]
        nq = int(round(math.exp(rng.uniform(math.log(q_range[0]), math.log(q_range[1])))))
        work = math.exp(rng.uniform(math.log(work_range[0]), math.log(work_range[1])))
        nw = max(min_walks, int(work / (nq * SERVED_KINDS[name])))
        qs = int(rng.integers(1 << 30))
        if name == "circle":
            th = np.random.default_rng(qs).uniform(0, 2 * np.pi, nq)
            Q = np.stack([np.cos(th), np.sin(th)], 1)
        elif name == "sphere":
            Q = inputs.sphere_uniform(nq, 3, qs)
        elif name == "cap":
            Q = inputs.cap_uniform(nq, 3, 0.0, qs)
        elif name == "torus":
            Q = inputs.torus_area_uniform(nq, seed=qs)
        else:
            Q = inputs.hypersphere_queries(max(nq, 2), probs[name]["n"], qs)
        reqs.append((t, name, Q, nw, int(rng.integers(1 << 62))))
    opt = dict(precision="fp32", persistent=1)
    srv = mpwos.Server(64 << 30)
    t0 = time.perf_counter()
    tickets, pending, done_at = [], {}, {}

    def poll_all():
        for tk in list(pending):
            if srv.poll(tk)[0]:
                done_at[tk] = time.perf_counter() - t0
                del pending[tk]

    for (ta, name, Q, nw, sd) in reqs:
        while time.perf_counter() - t0 < ta:
            poll_all()
            time.sleep(0.0005)
        tk = srv.submit(mans[name], probs[name], Q, nw, sd, **opt)
        tickets.append(tk)
        pending[tk] = ta
    last_print = time.perf_counter()
    while pending:
        poll_all()
        time.sleep(0.0005)
        if time.perf_counter() - last_print > 20:
            print(f"[bench] served: {len(pending)} requests outstanding", file=sys.stderr, flush=True)
            last_print = time.perf_counter()
    wall = time.perf_counter() - t0
    outs = [srv.wait(tk) for tk in tickets]
    st = srv.stats()
    tl = [srv.times(tk) for tk in tickets]
    srv.close()
    lat = np.array([done_at[tk] - r[0] for tk, r in zip(tickets, reqs)])
    # accuracy against the closed form: Monte Carlo error within 4 standard
    # errors, plus 1e-3 for the tau_W truncation and the cap's eps-layer bias
    ok, nqs, zs = 0, 0, []
    for (ta, name, Q, nw, sd), o in zip(reqs, outs):
        ex = inputs.exact_u(probs[name], Q)
        err = np.abs(o["u"] - ex)
        ok += int(np.sum(err <= 4 * o["stderr"] + 1e-3))
        nqs += len(Q)
        zs.extend((err / np.maximum(o["stderr"], 1e-300)).tolist())
    res = {"rate_req_per_s": rate, "window_s": window, "requests": len(reqs),
           "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "drain_s": max(0.0, wall - window), "backlog_growth": backlog_growth(reqs, lat),
           "walk_steps": int(st["walk_steps"]),
           "walk_steps_per_s": st["walk_steps"] / wall, "launches": st["rounds"],
           "closed_form_check": {"queries": nqs, "within_4se_plus_1e-3": ok / nqs,
                                 "median_abs_z": float(np.median(zs))},
           "by_manifold": {}}
    # where the time goes (server timeline, medians): admission wait, wait for
    # the first launch, walks, reduction and delivery
    phases = {"admit": (0, 1), "start": (1, 2), "walks": (2, 3), "deliver": (3, 4)}
    for name in SERVED_KINDS:
        sel = [i for i, r in enumerate(reqs) if r[1] == name]
        if not sel:
            continue
        ln = lat[sel]
        d = {"requests": len(sel), "p50_ms": float(np.percentile(ln, 50) * 1e3),
             "p99_ms": float(np.percentile(ln, 99) * 1e3)}
        for ph, (a, b) in phases.items():
            d[ph + "_p50_ms"] = float(np.median([(tl[i][list(tl[i])[b]] - tl[i][list(tl[i])[a]]) * 1e3
                                                 for i in sel]))
        res["by_manifold"][name] = d
    if not solo:
        for m in mans.values():
            m.close()
        return res
    print(f"[bench] served: {len(reqs)} requests done in {wall:.1f} s; solving them alone", file=sys.stderr,
          flush=True)
    # the same requests alone, first in first out, with the per-solve entry point
    service, same = [], 0
    for (ta, name, Q, nw, sd), o in zip(reqs, outs):
        ts = time.perf_counter()
        r = mpwos.solve(probs[name], Q, nw, sd, manifold=mans[name], **opt)
        service.append(time.perf_counter() - ts)
        same += int(np.array_equal(r["u"], o["u"]))
    finish, fifo = 0.0, []
    for (ta, *_), sv in zip(reqs, service):
        finish = max(finish, ta) + sv
        fifo.append(finish - ta)
    fifo = np.array(fifo)
    for m in mans.values():
        m.close()
    res.update({"request_mix": "manifold uniform over S^1, S^2, S^2 cap, implicit torus, S^99, S^999; queries "
                               f"log-uniform in [{q_range[0]}, {q_range[1]}]; work log-uniform in "
                               f"[{work_range[0]:.0e}, {work_range[1]:.0e}] walk-steps per request, at least "
                               f"{min_walks} walks per query",
                "results_equal_alone": f"{same}/{len(reqs)}",
                "per_solve_fifo": {"p50_ms": float(np.percentile(fifo, 50) * 1e3),
                                   "p99_ms": float(np.percentile(fifo, 99) * 1e3),
                                   "busy_s": float(sum(service))}})
    return res


def backlog_growth(reqs, lat):
    """Median latency of the requests that arrived in the last third of the
    window over that of the first third, per manifold, the largest: near 1
    while the server keeps up, growing with the backlog when it does not."""
    t = np.array([r[0] for r in reqs])
    lo, hi = np.percentile(t, 100 / 3), np.percentile(t, 200 / 3)
    worst = 0.0
    for name in SERVED_KINDS:
        sel = np.array([r[1] == name for r in reqs])
        a, b = lat[sel & (t <= lo)], lat[sel & (t >= hi)]
        if len(a) >= 3 and len(b) >= 3:
            worst = max(worst, float(np.median(b) / np.median(a)))
    return worst


def served_sweep(rates, window=3.0):
    """The served mix at several arrival rates (no solo runs).  A rate is
    stable when no manifold's median latency grows by more than half from
    the first third of the arrivals to the last (backlog_growth <= 1.5)."""
    runs = []
    for r in rates:
        runs.append(served_mix(rate=r, window=window, solo=False))
        print(f"[bench] served sweep: {r:g} req/s p50 {runs[-1]['p50_ms']:.0f} ms p99 {runs[-1]['p99_ms']:.0f} ms "
              f"drain {runs[-1]['drain_s']:.2f} s backlog growth {runs[-1]['backlog_growth']:.2f}", file=sys.stderr,
              flush=True)
    stable = [x["rate_req_per_s"] for x in runs if x["backlog_growth"] <= 1.5]
    return {"runs": [{k: x[k] for k in ("rate_req_per_s", "requests", "p50_ms", "p99_ms", "drain_s", "backlog_growth",
                                        "walk_steps_per_s", "launches", "closed_form_check", "by_manifold")}
                     for x in runs],
            "max_stable_rate_req_per_s": max(stable) if stable else None}


def roofline(fast, dom_name, kind, n, n_v, precision):
    w, rates = valu_weights()
    ops = step_ops(kind, n, n_v)
    slots = sum(ops[k] * w[k] for k in ops)
    dom = fast["per"][dom_name]
    achieved = slots * dom["walk_steps"] / (dom["kernel_ms"] * 1e-3)
    traffic = None
    if TRAFFIC["kernel_sha256"] is not None and TRAFFIC["kernel_sha256"] == kernel_sha256() \
            and dom_name == "sphere" and dom["walk_steps"] == 4096 * 4096 * 174 and precision == "fp32":
        traffic = 1024 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_factor"] +
                          TRAFFIC["write_kib"] * TRAFFIC["write_factor"])
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12, "unit": "Tslot/s",
            "frac": achieved / PEAK_SLOTS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch",
            "kernel": ("walk_lane_kernel<float,%d,%s> %s" % (n, kind, "persistent" if dom["launch"].get("persistent")
                                                              else "plain")) if precision == "fp32"
            else f"walk_lane_kernel<double,{n},{kind}>",
            "launch": dom["launch"],
            "timing": "HIP events on the launch stream around each " + ("graph replay (copy in, seed, counter "
                      "reset, walk kernel, per-query reduction, copy out)" if "graph" in fast["form"] else
                      "walk launch"),
            "launch_walk_steps": dom["walk_steps"], "launch_ms": dom["kernel_ms"],
            "ops_per_walk_step": ops, "slot_weights": {k: round(v, 3) for k, v in w.items()},
            "slots_per_walk_step": slots,
            "probe_lane_ops_per_s": {k: float("%.4g" % v) for k, v in rates.items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sphere",
                    choices=["sphere", "circle", "torus", "cloud", "hyper100", "hyper1000", "dumbbell",
                             "sphere_cloud", "product", "cut_torus"],
                    help="sphere (closed + cap) is the headline workload; the others are for profiling")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink queries and walks (profiling only)")
    ap.add_argument("--block-size", type=int, default=0, help="workgroup size of the walk kernels (0 = autotuned)")
    ap.add_argument("--launch", default="", metavar="NAME=FORM:BLOCK,...",
                    help="fixed launch shapes instead of the autotuner, e.g. sphere=plain:256,cap=persistent:192")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the FP32 form through mpwos_solve per step instead of graph replays")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--no-roofline", action="store_true", help="skip the VALU probe (profiling runs)")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None, help="time only one form (profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="time the library's plain copy kernel on BYTES (HBM calibration) and exit")
    ap.add_argument("--valu-probe", action="store_true", help="print the VALU operation rates and exit")
    ap.add_argument("--no-served", action="store_true", help="skip the served-mix leg")
    ap.add_argument("--served-rates", default="100,400,800",
                    help="arrival rates (req/s) of the served sweep besides 200; empty to skip")
    ap.add_argument("--served-only", action="store_true", help="run only the served-mix leg and print it")
    ap.add_argument("--compensation-sweep", default="", metavar="N1,N2,...",
                    help="Example 1: RMSE against the closed form of the baseline, second-order and exact "
                         "compensation at these walk counts (100 points, N_V = 50, FP32), printed and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the walk path runs on a "
              "single device here)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        from paper_2606_21883_amd import mpwos
        ms = mpwos.copy_probe(args.copy_probe, 5)
        print(json.dumps({"copy_bytes": args.copy_probe, "ms": ms,
                          "GB_per_s": 2 * args.copy_probe / (ms * 1e-3) / 1e9}), flush=True)
        return
    if args.valu_probe:
        w, r = valu_weights()
        print(json.dumps({"lane_ops_per_s": r, "weights": w, "peak_lane_ops_per_s": PEAK_SLOTS}), flush=True)
        return
    if args.compensation_sweep:
        print(json.dumps(compensation_sweep([int(v) for v in args.compensation_sweep.split(",")])), flush=True)
        return
    if args.served_only:
        out = served_mix()
        if args.served_rates:
            out["sweep"] = served_sweep([float(x) for x in args.served_rates.split(",")])
        print(json.dumps(out), flush=True)
        return
    rank = int(os.environ.get("RANK", "0"))
    work = make_workload(args.workload, args.scale)
    prec = "fp64" if args.only == "fp64" else "fp32"
    headline = prec == "fp32" and not args.no_graph
    fast = run_gpu(work, args.steps, args.warmup, prec, 0 if prec == "fp64" else 1, args.block_size,
                   graph=headline, tune=headline and not args.block_size, launch=parse_launch(args.launch))
    slow = None
    if not args.no_fp64 and args.only is None:
        slow = run_gpu(work, max(1, min(args.steps, 3)), 1, "fp64", 0)
    ws = fast["walk_steps_per_step"]
    ms = 1e3 * fast["seconds"] / fast["steps"]
    value = ws * fast["steps"] / fast["seconds"]
    nq_total = sum(p["n_queries"] for p in fast["per"].values())
    first = work[0]
    prob0 = first[1]
    desc = {
        "sphere": "unit sphere S^2: closed (u=x1x2, sigma=2, 4096 queries x 4096 walks) + cap x3>0 "
                  "(Dirichlet g=u, sigma=0.5, eps=1e-3, 4096 x 4096)",
        "circle": "unit circle S^1: u=cos(3 theta), sigma=1, 64 queries x 1000 walks",
        "torus": "implicit torus R=1, a=0.3: u=sin(phi)cos(2psi), sigma=1, 8192 queries x 1024 walks",
        "cloud": "point-cloud torus, 1e6 points, noise 1e-4, k=16 + quadratic fit: 8192 queries x 1024 walks",
        "hyper100": "S^99 in R^100: u=x1x2, sigma=1, 1024 queries x 2048 walks",
        "hyper1000": "S^999 in R^1000: u=x1x2, sigma=1, 1024 queries x 2048 walks",
        "dumbbell": "1000-dimensional implicit dumbbell in R^1001 (a=0.35, kc=1.2), sigma=2000, m=0, "
                    "N_V=50, 20 points x 1000 paths",
        "sphere_cloud": "point-cloud S^2, 8000 points, nearest-point projection, spacing rule (6 neighbours, "
                        "c_h=2.4), u=P1+0.2P3+0.1P5, sigma=1, m=0: 1024 queries x 1024 walks",
        "product": "S^1_Fourier(1) x S^2(0.65) in R^9, u=cos(phi)w1+0.3sin(2phi)w2+0.2cos(3phi)(w1^2-w2^2), "
                   "sigma=1, m=0: 4096 queries x 1024 walks",
        "cut_torus": "torus R=1, a=0.45 cut at phi_c=0.35pi (Example 1), u=sin(s)A+sin(2s)B+sin(3s)C, sigma=4, "
                     "eps=1e-5, N_V=50, second-order m_* from a device predictor (baseline solve, 32x15 nodes x "
                     "256 walks, 4x9 Fourier-sine fit) refitted every step: 100 points x 10000 walks",
    }[args.workload]
    if args.scale != 1.0:
        desc += f" (scaled by {args.scale})"
    out = {
        "metric": METRIC, "value": value, "unit": "walk-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": desc,
                   "precision": "f32 walk arithmetic, f64 path weight/scores/per-query sums" if prec == "fp32"
                   else "f64",
                   "form": fast["form"] if prec == "fp32" else "plain one launch per solve",
                   "n_v": prob0.get("n_v", 1), "tau_w": prob0.get("tau_w"), "theta": prob0.get("theta"),
                   "c_kappa": prob0.get("c_kappa"), "seed": 0},
        "queries_per_s": nq_total * fast["steps"] / fast["seconds"],
        "per_solve": fast["per"],
    }
    n0 = prob0["n"]
    if not args.no_roofline and n0 <= 3 and prob0["manifold"] == "sphere":
        out["roofline"] = roofline(fast, first[0], "sphere", n0, prob0.get("n_v", 1), prec)
    # the host-buffer rate of the headline step (the unit-sphere workload only:
    # the others' pipelines, such as the cut torus predictor, are not single solves)
    if headline and args.only is None and args.workload == "sphere":
        out["host_io"] = host_io_rate(work, fast["per"])
    if slow is not None:
        v64 = slow["walk_steps_per_step"] * slow["steps"] / slow["seconds"]
        out["fp64_plain"] = {"value": v64, "ms_per_step": 1e3 * slow["seconds"] / slow["steps"],
                             "per_solve": slow["per"]}
        out["speedup_vs_fp64_plain"] = value / v64
        out["rmse_ratio_fp32_over_fp64"] = {k: fast["per"][k]["rmse"] / slow["per"][k]["rmse"]
                                            for k in fast["per"]}
    if args.workload == "dumbbell":
        # Table 1 of the paper (N = 1000 paths, N_V = 50, one point at a time,
        # 24 laptop CPU cores): 11.43 s per point, 1.78e4 walk-steps/s derived;
        # another machine's number, quoted for context
        per = next(iter(fast["per"].values()))
        out["paper_table1"] = {"seconds_per_point": 11.43, "walk_steps_per_s": 1.78e4, "avg_steps": 204,
                               "hardware": "24 CPU cores, MATLAB"}
        out["ms_per_point"] = per["kernel_ms"] / per["n_queries"]
        out["avg_steps"] = per["k_mean"]
        out["vs_baseline"] = value / 1.78e4
    if not args.no_served and args.workload == "sphere" and args.only is None:
        out["served"] = served_mix()
        if args.served_rates:
            out["served"]["sweep"] = served_sweep([float(x) for x in args.served_rates.split(",")])
    if not args.no_cpu and rank == 0:
        out["cpu_baseline"] = cpu_baseline(work)
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
