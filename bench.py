"""Benchmark of the MPWoS hot path on one MI355X.

One step = one pass of the whole walk path over the unit-sphere workload:
  - S^2 closed, u = x1 x2, sigma = 2, f = 8 x1 x2: 4096 queries x 4096 walks;
  - S^2 cap x3 > 0, Dirichlet g = u, sigma = 0.5, eps = 1e-3: 4096 x 4096 walks;
in the FP32-mixed form (FP32 walk arithmetic, FP64 path weight, scores and
per-query compensated sums), one mpwos_solve per solve with device-resident
queries and outputs, in the launch shape the library's autotuner picks.

metric: walk-steps/s (one walk-step = one iteration of Algorithm 1 with its
N_V = 1 Green sample), with queries/s and the closed-form RMSE beside it.
Reported beside the headline:
  - the same step as graph replays (mpwos_plan_*) and in the plain FP64
    one-launch-per-solve form;
  - every other configuration (S^1; S^99 and S^999 at their full 1024 x 2048
    walks; the implicit torus; the 1e6-point cloud), each with the roofline of
    its kernel, long walks timed over a fixed number of steps per walk;
  - the served mix through the continuous-batching server;
  - the FP64 CPU oracle on bounded samples.

Roofline of a walk kernel (VALU-bound: walk state lives in registers):
  achieved = algorithmic operations of one walk-step (step_ops, the method's
  own work) weighted by their issue cost relative to a full-rate FP32 FMA
  (SLOT_WEIGHTS, frozen from the library's VALU probe on MI355X) x walk-steps
  of the launch / the launch's kernel time from HIP events on its stream;
  peak = 256 CUs x 128 FP32 lanes per clock x 2.4 GHz (the published FP32
  vector peak, 157.3 TFLOP/s, counted per FMA).  Beside it: the FP32 FLOP
  fraction of 157.3 TFLOP/s and the unweighted VALU issue fraction from the
  rocprofv3 counters of the same kernel sources.
"""
import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The server runs its launches on GPU_MAX_HW_QUEUES - 2 streams (two at
# least); the runtime reads the variable when it starts, so it is raised here,
# before anything touches the device, to eight when it is lower (HIP's default
# is four).  Eight hardware queues give the served mix three streams for its
# long classes (point cloud, dumbbell, S^99) and three for the rest; with four,
# the long classes share one stream and queue behind each other.  One-stream
# legs are unaffected.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

METRIC = "walk-steps/s and queries/s at fixed RMSE vs FP64 oracle; served p50/p99 ms"
# Full-rate VALU lane-operations per second: 256 CUs x 128 FP32 FMA lanes per
# clock x 2.4 GHz, the published FP32 vector peak (157.3 TFLOP/s) counted per FMA.
PEAK_SLOTS = 256 * 128 * 2.4e9
PEAK_FP32_FLOPS = 157.3e12
PEAK_HBM_BYTES = 8.0e12

# Issue cost of each operation class relative to fma_f32, from the library's
# VALU probe on MI355X (python bench.py --valu-probe; the committed run is in
# profiles/valu_probe_slot_weights.txt): bitop3 and FP64 isolated, the
# transcendentals and the 64-bit multiply-add by the time they add beside
# three independent FMAs.  Frozen, so that every run divides by the same model.
SLOT_WEIGHTS = {"f32": 1.0, "bitop3_b32": 1.53, "f64": 1.72, "trans": 3.06, "mad_u64_u32": 0.91}

# Device sources of the walk kernels: the counter constants below hold only for
# the sources whose SHA-256 they carry.
KERNEL_SOURCES = ["walk_lane.hip", "walk_group.hip", "walk_group_dev.h", "walk_group_sphere.hip", "mpwos_dev.h",
                  "kernel_args.h", "cloud_dev.h", "cloud.hip"]

# Per-kernel figures from rocprofv3 counters (profiles/walk_kernels_all_configs_counters.txt),
# per walk-step of the benchmark's launches in the launch shape given: VALU and
# SALU lane-instructions (wave instructions x 64 / walk-steps) and the counted
# FETCH_SIZE and WRITE_SIZE (KiB per launch); HBM bytes = FETCH_SIZE x 2 +
# WRITE_SIZE x 1, the factors read off a plain copy kernel of known size
# (profiles/copy_kernel_hbm_probe.txt).  They apply to a run only when the
# kernel sources hash to kernel_sha256 and the launch has the same form.
PROFILED = {
    "kernel_sha256": "678fb807edc7587baff4f6b961eca95f5b52da0d50d835d765f06cddd98ec4c0",
    "kernels": {
        "sphere": {"valu_per_walk_step": 157.45, "salu_per_walk_step": 31.26, "walk_steps": 2919235584, "fetch_kib": 462.9, "write_kib": 196608.0, "launch": {"persistent": 0, "block_size": 256}},
        "cap": {"valu_per_walk_step": 280.18, "salu_per_walk_step": 92.01, "walk_steps": 478364829, "fetch_kib": 983.3, "write_kib": 289523.8, "launch": {"persistent": 1, "block_size": 256}},
        "circle": {"valu_per_walk_step": 153.28, "salu_per_walk_step": 30.33, "walk_steps": 14848000, "fetch_kib": 94.9, "write_kib": 750.0, "launch": {"persistent": 0, "block_size": 0}},
        "hyper100": {"valu_per_walk_step": 6867.68, "salu_per_walk_step": 897.22, "walk_steps": 2097152000, "fetch_kib": 3355.2, "write_kib": 24576.0, "launch": {"persistent": 0, "block_size": 0}},
        "hyper1000": {"valu_per_walk_step": 55837.12, "salu_per_walk_step": 7216.96, "walk_steps": 419430400, "fetch_kib": 34250.6, "write_kib": 38912.0, "launch": {"persistent": 0, "block_size": 0}},
        "torus": {"valu_per_walk_step": 516.53, "salu_per_walk_step": 68.97, "walk_steps": 13430161408, "fetch_kib": 843.8, "write_kib": 98304.0, "launch": {"persistent": 0, "block_size": 0}},
        "cloud": {"valu_per_walk_step": 25527.95, "salu_per_walk_step": 16584.77, "walk_steps": 536870912, "fetch_kib": 3187984563.8, "write_kib": 99219.2, "launch": {"persistent": 1, "block_size": 0}},
    },
}
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0


def kernel_sha256():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_21883_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# ---------------------------------------------------------------------------
# algorithmic work of one walk-step
# ---------------------------------------------------------------------------

def step_ops(kind, n, n_v=1):
    """Algorithmic operations of one FP32-mixed walk-step by issue class.

    Counts what the method as specified must do, once per walk (work a lane
    group repeats in every lane is implementation cost and is not counted):
      - Philox4x32-10 blocks: n <= 3, one for the direction and one per Green
        sample; n >= 4, a block per four normals plus the radius word; 10
        rounds of two 32x32->64 multiplies and two three-way xors each;
      - two operations per uniform; n = 2, cos and sin of the angle; n = 3,
        the hat-box axis coordinate, its radius and the azimuth (a square
        root, cos, sin and five FP32 operations); n >= 4, Box-Muller pairs
        (log, square root, cos, sin and three FP32 operations per pair);
      - per n-vector update Y + r zeta: a squared norm (n), the update (n);
        the projection: sphere, a squared norm (n), a reciprocal square root
        and the scaling (n + 1); implicit torus, Newton on the level set (four
        steps of 13 operations and a reciprocal square root on average at
        walk radii); point cloud, the patch transform and six Newton steps on
        the quadratic (the nearest-point search is counted in bytes, not here);
      - the Green radius from the inverse-CDF table; the source with its exact
        compensation;
      - FP64: F to FP64 and its 1/N_V, W omega, the score sum, W c, the stop
        test;
      - cap: the boundary distance, the two-slice table, the per-step weight
        series (eight terms and a reciprocal) and the radius.
    """
    if n >= 4:
        nb_dir = (n + 3) // 4
        blocks = nb_dir + n_v * (nb_dir + 1)
        words = n + n_v * (n + 1)
        pairs = (1 + n_v) * ((n + 1) // 2)
        ops = {"mad_u64_u32": 20 * blocks, "bitop3_b32": 20 * blocks, "f32": 2 * words + 3 * pairs,
               "trans": 4 * pairs, "f64": 6}
        ops["f32"] += 4 * n + n_v * 3 * n          # Theta: |g|^2, update, |Theta|^2, scale; Z: |g'|^2, update, |Z|^2
        ops["trans"] += 2 + 2 * n_v                # the four reciprocal square roots
        ops["f32"] += n_v * (10 + 8)               # radius table, source
        ops["trans"] += n_v * 2
        return ops
    sets = 1 + n_v
    ops = {"mad_u64_u32": 20 * sets, "bitop3_b32": 20 * sets, "f32": 0, "trans": 0, "f64": 6}
    words = (n - 1) + n_v * n
    ops["f32"] += 2 * words
    ops["trans"] += sets * (3 if n == 3 else 2)
    ops["f32"] += sets * (5 if n == 3 else 0)
    if kind == "torus":
        ops["f32"] += sets * (n + 4 * 13)
        ops["trans"] += sets * 4
        ops["f32"] += n_v * (10 + 40)              # radius table, torus-mode source with its compensation
        ops["trans"] += n_v * (1 + 5)
    elif kind == "cloud":
        ops["f32"] += sets * (n + 15 + 6 * 35)
        ops["f32"] += n_v * (10 + 40)
        ops["trans"] += n_v * (1 + 5)
    else:
        ops["f32"] += sets * (3 * n + 1)
        ops["trans"] += sets
        ops["f32"] += n_v * (10 + 8)
        ops["trans"] += n_v * (1 + 1)
    ops["f32"] += 2                                # step counter and bound
    if kind == "cap":
        ops["f32"] += 18 + 8 + 11 + 3              # delta_Gamma, two-slice table, weight series, radius
        ops["trans"] += 3
    return ops


def fp32_flops(ops):
    """FP32 FLOPs of the step model, one per FP32 operation or transcendental
    (a lower bound: a fused multiply-add counts once)."""
    return ops["f32"] + ops["trans"]


def kernel_label(kind, n, precision, launch):
    if n >= 4:
        return f"walk_group_kernel ({'FP32' if precision == 'fp32' else 'FP64'}, n={n}, " \
               f"{'persistent' if launch.get('persistent') else 'plain'})"
    k = {"sphere": 0, "cap": 1, "torus": 2, "cloud": 3}[kind]
    t = "float" if precision == "fp32" else "double"
    return f"walk_lane_kernel<{t}, {n}, {k}> ({'persistent' if launch.get('persistent') else 'plain'})"


def roofline_alu(name, kind, n, n_v, walk_steps, kernel_ms, launch, precision="fp32"):
    """VALU roofline of one walk kernel launch (see the module docstring)."""
    ops = step_ops(kind, n, n_v)
    slots = sum(ops[k] * SLOT_WEIGHTS[k] for k in ops)
    secs = kernel_ms * 1e-3
    achieved = slots * walk_steps / secs
    out = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12, "unit": "Tslot/s",
           "frac": achieved / PEAK_SLOTS, "traffic": None,
           "kernel": kernel_label(kind, n, precision, launch),
           "timing": "HIP events on the launch stream around each walk-kernel launch (library kernel_ms)",
           "launch_walk_steps": int(walk_steps), "launch_ms": kernel_ms,
           "ops_per_walk_step": ops, "slots_per_walk_step": slots, "slot_weights": SLOT_WEIGHTS,
           "fp32_flop_frac": fp32_flops(ops) * walk_steps / secs / PEAK_FP32_FLOPS}
    prof = profiled(name, launch)
    if prof:
        out["counted_launch"] = prof["launch"]
        out["valu_issue_frac"] = prof["valu_per_walk_step"] * walk_steps / secs / PEAK_SLOTS
        out["valu_per_walk_step_counted"] = prof["valu_per_walk_step"]
        if prof.get("walk_steps") == walk_steps and "fetch_kib" in prof:
            out["traffic"] = 1024 * (prof["fetch_kib"] * FETCH_FACTOR + prof["write_kib"] * WRITE_FACTOR)
            out["traffic_unit"] = "HBM bytes per launch"
    return out


def roofline_cloud(name, n_queries, n_walks, walk_steps, kernel_ms, launch):
    """The point-cloud walk: its nearest-point search is a chain of dependent
    node loads, so the kernel is bound by memory latency; the roofline given
    is the HBM one over the algorithmic bytes of a walk-step: two projections,
    each reading the nearest point's FP32 patch (80 B) and its point record
    (16 B), plus the query and the per-walk outputs."""
    per_step = 2 * (80 + 16)
    algo = per_step * walk_steps + n_queries * 24 + n_queries * n_walks * 12
    secs = kernel_ms * 1e-3
    out = {"bound": "hbm", "achieved": algo / secs / 1e9, "peak": PEAK_HBM_BYTES / 1e9, "unit": "GB/s",
           "frac": algo / secs / PEAK_HBM_BYTES, "traffic": None,
           "kernel": kernel_label("cloud", 3, "fp32", launch),
           "timing": "HIP events on the launch stream around each walk-kernel launch (library kernel_ms)",
           "algorithmic_bytes_per_walk_step": per_step, "launch_walk_steps": int(walk_steps),
           "launch_ms": kernel_ms,
           "note": "latency-bound: each projection is a depth-first KD-tree nearest-point search"}
    prof = profiled(name, launch)
    if prof:
        out["counted_launch"] = prof["launch"]
        out["valu_issue_frac"] = prof["valu_per_walk_step"] * walk_steps / secs / PEAK_SLOTS
        out["valu_per_walk_step_counted"] = prof["valu_per_walk_step"]
    if prof and prof.get("walk_steps") == walk_steps and "fetch_kib" in prof:
        out["traffic"] = 1024 * (prof["fetch_kib"] * FETCH_FACTOR + prof["write_kib"] * WRITE_FACTOR)
        out["traffic_unit"] = "HBM bytes per launch"
        out["traffic_frac"] = out["traffic"] / secs / PEAK_HBM_BYTES
    return out


def profiled(name, launch=None):
    if PROFILED.get("kernel_sha256") != kernel_sha256():
        return None
    prof = PROFILED["kernels"].get(name)
    if prof is None or launch is None:
        return prof
    # the same form (plain or persistent); the workgroup size the autotuner
    # picks moves the counts per walk-step by little
    return prof if launch.get("persistent", 0) == prof["launch"]["persistent"] else None


def valu_weights_live():
    """Issue cost of each operation class relative to fma_f32, from the VALU
    probe run now (the frozen SLOT_WEIGHTS come from such a run)."""
    from paper_2606_21883_amd import mpwos
    r = {op: mpwos.valu_probe(op) for op in mpwos.VALU_OPS}
    base = r["fma_f32"]

    def mixed(name):
        return max(0.0, (4.0 / r[name] - 3.0 / base) * base)

    w = {"f32": 1.0, "bitop3_b32": base / r["bitop3_b32"], "f64": base / r["fma_f64"],
         "trans": mixed("sin_f32+3fma"), "mad_u64_u32": mixed("mad_u64_u32+3fma")}
    return w, r


# ---------------------------------------------------------------------------
# timed solves
# ---------------------------------------------------------------------------

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


def run_gpu(work, steps, warmup, precision, persistent, block_size=0, graph=False, tune=False, launch=None,
            extra=None, score=True):
    """Times `steps` passes over the workload.  Eager (graph=False): one
    mpwos_solve per solve and step, device-resident queries and outputs, the
    walk kernel's time from the library's HIP events on the launch stream.
    graph: each solve is a captured plan replayed per step, timed by HIP events
    around the replay.  tune: the launch shape of each solve comes from
    mpwos_autotune first (untimed).  extra: options for every solve (such as
    a max_steps budget)."""
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
        opt.update(extra or {})
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
    res = {"seconds": dt, "steps": steps, "form": ("graph replay" if graph else "mpwos_solve per solve") +
           (", autotuned launch shape" if tune else "")}
    per = {}
    total_ws = 0
    for i, it in enumerate(items):
        if it["plan"] is not None:
            kms = float(np.mean([s[i][0].elapsed_time(s[i][1]) for s in stats]))
            pst = it["plan"].stats(stream)
        else:
            kms = float(np.mean([s[i]["kernel_ms"] for s in stats]))
            pst = stats[0][i]
        ws = pst["walk_steps"]
        total_ws += ws
        d = {"kernel_ms": kms, "walk_steps": ws, "k_mean": pst["k_mean"], "k_p50": pst.get("k_p50"),
             "k_p99": pst.get("k_p99"), "k_max": pst.get("k_max"), "walk_steps_per_s": ws / (kms * 1e-3),
             "n_queries": int(it["q"].shape[0]), "n_walks": int(it["nw"]),
             "launch": {k: v for k, v in it["opt"].items() if k not in ("precision", "max_steps")}}
        if score:
            Qh = it["q"].cpu().numpy()
            if it["prob"]["manifold"] == "point_cloud":
                Qh = mpwos.debug_cp(it["m"], Qh, "fp64")       # the estimate refers to cp_h(q)
            exact = inputs.exact_u(it["prob"], Qh)
            d.update(rmse=inputs.rmse(it["u"].cpu().numpy(), exact),
                     mean_stderr=float(np.sqrt(np.mean(it["se"].cpu().numpy() ** 2))))
        per[it["name"]] = d
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


# ---------------------------------------------------------------------------
# the other configurations, each at its full query and walk counts
# ---------------------------------------------------------------------------

# name -> (kind, FP32 steps per walk timed (None = whole walks), FP64 steps per walk,
#          whole-walk length at tau_W = 1e-8 for queries/s)
CONFIGS = {
    "circle": ("sphere", None, None, 232),
    "hyper100": ("sphere", 1000, 100, 11340),
    "hyper1000": ("sphere", 200, 20, 113393),
    "torus": ("torus", None, None, 1601),
    "cloud": ("cloud", 64, 16, 1601),
}


def measure_configs(names, reps=2):
    """Each configuration at its full shape in the FP32 form (and FP64 plain
    beside it): walk-steps/s from the walk kernel's HIP events, the roofline
    of that kernel, and queries/s (extrapolated to whole walks where the
    walks were timed over a fixed number of steps)."""
    out = {}
    for name in names:
        kind, b32, b64, K = CONFIGS[name]
        work = make_workload(name)
        prob = work[0][1]
        n = prob["n"]
        print(f"[bench] config {name}: {len(work[0][2])} queries x {work[0][3]} walks", file=sys.stderr, flush=True)
        e32 = dict(max_steps=b32) if b32 else {}
        r32 = run_gpu(work, reps, 1, "fp32", 1 if kind in ("cap", "cloud") else 0, extra=e32, score=b32 is None)
        p32 = r32["per"][name]
        row = {"walk_steps_per_s": p32["walk_steps_per_s"], "kernel_ms": p32["kernel_ms"],
               "walk_steps": p32["walk_steps"], "n_queries": p32["n_queries"], "n_walks": p32["n_walks"],
               "steps_per_walk_timed": b32 or "whole walks", "whole_walk_steps": K,
               "queries_per_s": p32["n_queries"] / (p32["kernel_ms"] * 1e-3 * (K / b32 if b32 else 1.0)),
               "launch": p32["launch"]}
        if b32 is None:
            row.update(rmse=p32["rmse"], mean_stderr=p32["mean_stderr"])
        if kind == "cloud":
            row["roofline"] = roofline_cloud(name, p32["n_queries"], p32["n_walks"], p32["walk_steps"],
                                             p32["kernel_ms"], p32["launch"])
        else:
            row["roofline"] = roofline_alu(name, kind, n, prob.get("n_v", 1), p32["walk_steps"], p32["kernel_ms"],
                                           p32["launch"])
        e64 = dict(max_steps=b64) if b64 else {}
        r64 = run_gpu(work, 1, 0, "fp64", 0, extra=e64, score=b64 is None)
        p64 = r64["per"][name]
        row["fp64_plain"] = {"walk_steps_per_s": p64["walk_steps_per_s"], "kernel_ms": p64["kernel_ms"],
                             "steps_per_walk_timed": b64 or "whole walks"}
        if b64 is None:
            row["fp64_plain"]["rmse"] = p64["rmse"]
            row["rmse_ratio_fp32_over_fp64"] = p32["rmse"] / p64["rmse"]
        row["speedup_vs_fp64_plain"] = p32["walk_steps_per_s"] / p64["walk_steps_per_s"]
        out[name] = row
        print(f"[bench] config {name}: {row['walk_steps_per_s']:.3g} walk-steps/s FP32, "
              f"roofline {row['roofline']['frac']:.3f}", file=sys.stderr, flush=True)
    return out


# ---------------------------------------------------------------------------
# the FP64 CPU oracle
# ---------------------------------------------------------------------------

def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_rate(prob, Q, nw, threads):
    import oracle
    t0 = time.perf_counter()
    r = oracle.solve(prob, Q, nw, 0, threads=threads)
    dt = time.perf_counter() - t0
    k = int(r["walk_K"].sum())
    return k, dt


def cpu_baseline(work, per_config=True):
    """The FP64 oracle on the host cores over a bounded sample of the headline
    workload (about 12 s), on one core, and on small samples of the other
    configurations (whole walks)."""
    from paper_2606_21883_amd import inputs
    nproc = os.cpu_count() or 1
    threads = min(16, nproc)
    sample = {"sphere": (64, 4096), "cap": (64, 4096), "dumbbell": (1, 32), "sphere_cloud": (2, 8), "product": (4, 64)}
    total_steps, total_t, parts = 0, 0.0, []
    for name, prob, Q, nw in work:
        nq, nws = sample.get(name, (8, 256))
        if "predictor_grid" in prob:
            # the oracle's own pipeline, shrunk: a coarse baseline solve at
            # 8 x 3 nodes, its series fit, then the compensated solve
            import oracle
            base = {kk: v for kk, v in prob.items() if kk != "predictor_grid"}
            t0 = time.perf_counter()
            rc = oracle.solve(dict(base, compensation="none"), inputs.cut_torus_nodes(8, 4), 16, 1, threads=threads)
            coef = oracle.ts_fit(rc["u"].reshape(8, 3), 2, 2)
            total_t += time.perf_counter() - t0
            total_steps += int(rc["walk_K"].sum())
            prob = dict(base, predictor=dict(idx=[2, 2], values=coef))
        k, dt = oracle_rate(prob, Q[:nq], nws, threads)
        total_steps += k
        total_t += dt
        parts.append(f"{name}: {nq} queries x {nws} walks ({k} walk-steps, {dt:.1f} s)")
    out = {"value": total_steps / total_t, "unit": "walk-steps/s", "cores": threads, "kind": "oracle",
           "sample": "; ".join(parts), "nproc": nproc, "cpu_model": cpu_model(),
           "build": "gcc -O2 -ffp-contract=off, FP64, pthreads over (query, walk)"}
    # one core, on a quarter of the first solve's sample
    name, prob, Q, nw = work[0]
    nq, nws = sample.get(name, (8, 256))
    k, dt = oracle_rate(prob, Q[:max(1, nq // 16)], nws, 1)
    out["single_core"] = {"value": k / dt, "sample": f"{name}: {max(1, nq // 16)} queries x {nws} walks ({dt:.1f} s)"}
    if per_config:
        # whole walks of every configuration on small query and walk samples:
        # a walk-step rate, so the sample size does not enter it
        subsets = {"circle": (64, 1000), "torus": (16, 256), "hyper100": (2, 16), "hyper1000": (1, 4),
                   "cloud": (2, 16)}
        rows = {}
        for cname, (nq, nws) in subsets.items():
            prob, Q, _ = inputs.config(cname)
            k, dt = oracle_rate(prob, Q[:nq], nws, threads)
            rows[cname] = {"walk_steps_per_s": k / dt, "sample": f"{nq} queries x {nws} walks ({k} walk-steps, "
                                                                  f"{dt:.1f} s)"}
            print(f"[bench] oracle {cname}: {k / dt:.3g} walk-steps/s", file=sys.stderr, flush=True)
        out["configs"] = rows
    return out


# ---------------------------------------------------------------------------
# the served mix
# ---------------------------------------------------------------------------

# Kinds of the served mix: the configuration, its walk length at tau_W = 1e-8,
# and the FP32 walk-steps per second one request of it runs at on MI355X
# (round figures from the configurations section), which turns a request's
# drawn GPU time into its size.
SERVED_KINDS = {"circle": (232, 5e10), "sphere": (174, 2e11), "cap": (29, 1e11), "torus": (1601, 5e10),
                "hyper100": (11340, 5e9), "hyper1000": (113393, 7e8), "cloud": (1601, 3e8),
                "dumbbell": (220, 1e7)}


def served_mix(rate=200.0, window=30.0, seed=2, ms_range=(0.02, 20.0), q_range=(1, 65536), min_walks=8,
               fp64_sample=200, kinds=None, deadline=180.0):
    """Poisson arrivals at `rate` per second for `window` seconds, served by the
    continuous-batching server (FP32 persistent kernels).  Each request draws a
    manifold uniformly from the configurations (S^1, S^2, S^2 cap, implicit
    torus, S^99, S^999, the resident 1e6-point cloud and the resident
    1000-dimensional dumbbell of Example 2), a query count log-uniform in
    q_range and a GPU time log-uniform in ms_range, which sets its walks from
    the kind's throughput (at least min_walks per query; query counts are cut
    so that the minimum fits).  Latency = completion - arrival.  Every
    estimate is checked against the closed-form solution where one exists.
    The plain per-solve FP64 path (mpwos_solve, one launch per solve, FIFO) is
    timed on a sample of the same requests, its FIFO latencies simulated from
    the measured service times over the same arrival trace."""
    import torch  # noqa: F401  (one HIP runtime with torch)

    from paper_2606_21883_amd import inputs, mpwos
    kinds = kinds or list(SERVED_KINDS)
    rng = np.random.default_rng(seed)
    probs, mans, qsets = {}, {}, {}
    for name in kinds:
        if name == "dumbbell":
            p = inputs.dumbbell_problem(1001, n_v=50)   # Table 1's setting
        else:
            p, _, _ = inputs.config(name, 1.0 / 1024)
        probs[name] = p
        mans[name] = mpwos.Manifold(p)
    t, reqs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window:
            break
        name = kinds[rng.integers(len(kinds))]
        K, thr = SERVED_KINDS[name]
        ms = math.exp(rng.uniform(math.log(ms_range[0]), math.log(ms_range[1])))
        work = ms * 1e-3 * thr
        nq = int(round(math.exp(rng.uniform(math.log(q_range[0]), math.log(q_range[1])))))
        nq = max(1, min(nq, int(work / (min_walks * K))))
        nw = max(min_walks, int(work / (nq * K)))
        qs = int(rng.integers(1 << 30))
        if name == "circle":
            th = np.random.default_rng(qs).uniform(0, 2 * np.pi, nq)
            Q = np.stack([np.cos(th), np.sin(th)], 1)
        elif name == "sphere":
            Q = inputs.sphere_uniform(nq, 3, qs)
        elif name == "cap":
            Q = inputs.cap_uniform(nq, 3, 0.0, qs)
        elif name in ("torus", "cloud"):
            Q = inputs.torus_area_uniform(nq, seed=qs)
        elif name == "dumbbell":
            Q = inputs.dumbbell_points(nq, 1001, seed=qs)
        else:
            Q = inputs.hypersphere_queries(max(nq, 2), probs[name]["n"], qs)
        reqs.append((t, name, Q, nw, int(rng.integers(1 << 62))))
    opt = dict(precision="fp32", persistent=1)
    srv = mpwos.Server(64 << 30)
    t0 = time.perf_counter()
    tickets, pending, done_at = [], {}, {}
    last_poll = [0.0]

    def poll_all():
        # every pending ticket, at most once a millisecond (each poll takes the
        # server's lock, which its scheduling thread needs too)
        now = time.perf_counter()
        if now - last_poll[0] < 1e-3:
            return
        last_poll[0] = now
        for tk in list(pending):
            if srv.poll(tk)[0]:
                done_at[tk] = time.perf_counter() - t0
                del pending[tk]

    last_print = time.perf_counter()
    for (ta, name, Q, nw, sd) in reqs:
        poll_all()
        while time.perf_counter() - t0 < ta:
            poll_all()
            time.sleep(0.0002)
        tk = srv.submit(mans[name], probs[name], Q, nw, sd, **opt)
        tickets.append(tk)
        pending[tk] = ta
        if time.perf_counter() - last_print > 10:
            print(f"[bench] served: {len(tickets)} submitted, {len(pending)} outstanding", file=sys.stderr, flush=True)
            last_print = time.perf_counter()
    while pending:
        poll_all()
        time.sleep(0.0005)
        if time.perf_counter() - last_print > 10:
            print(f"[bench] served: {len(pending)} requests outstanding", file=sys.stderr, flush=True)
            last_print = time.perf_counter()
        if time.perf_counter() - t0 > window + deadline:
            raise RuntimeError(f"served mix: {len(pending)} requests still outstanding {deadline:.0f} s after the "
                               "last arrival")
    wall = time.perf_counter() - t0
    outs = [srv.wait(tk) for tk in tickets]
    st = srv.stats()
    tl = [srv.times(tk) for tk in tickets]
    srv.close()
    lat = np.array([done_at[tk] - r[0] for tk, r in zip(tickets, reqs)])
    # accuracy against the closed form: Monte Carlo error within 4 standard
    # errors, plus 1e-3 for the tau_W truncation and the cap's eps-layer bias
    # (the cloud against u at the query's projection, with 0.02 for the
    # reconstruction; the dumbbell, whose m = 0 leaves a bias, is not scored)
    ok, nqs, zs = 0, 0, []
    rmses = {}
    for (ta, name, Q, nw, sd), o in zip(reqs, outs):
        if name == "dumbbell":
            continue
        Qe = mpwos.debug_cp(mans[name], Q, "fp64") if name == "cloud" else Q
        ex = inputs.exact_u(probs[name], Qe)
        err = np.abs(o["u"] - ex)
        tol = 4 * o["stderr"] + (0.02 if name == "cloud" else 1e-3)
        ok += int(np.sum(err <= tol))
        nqs += len(Q)
        zs.extend((err / np.maximum(o["stderr"], 1e-300)).tolist())
        rmses.setdefault(name, []).append(float(np.sqrt(np.mean(err ** 2))))
    res = {"rate_req_per_s": rate, "window_s": window, "requests": len(reqs),
           "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "drain_s": max(0.0, wall - window), "backlog_growth": backlog_growth(reqs, lat),
           "walk_steps": int(st["walk_steps"]),
           "walk_steps_per_s": st["walk_steps"] / wall, "launches": st["rounds"],
           "slots_busy_s": st["busy_seconds"], "wall_s": wall,
           "gpu_max_hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
           "closed_form_check": {"queries": nqs, "within_4se_plus_bias": ok / max(1, nqs),
                                 "median_abs_z": float(np.median(zs)) if zs else None,
                                 "request_rmse": {k: {"median": float(np.median(v)), "max": float(np.max(v)),
                                                      "within_1e-2": float(np.mean(np.array(v) <= 1e-2))}
                                                  for k, v in rmses.items()}},
           "by_manifold": {}}
    phases = {"admit": (0, 1), "start": (1, 2), "walks": (2, 3), "deliver": (3, 4)}
    for name in kinds:
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
    res["request_mix"] = (f"manifold uniform over {', '.join(kinds)}; queries log-uniform in "
                          f"[{q_range[0]}, {q_range[1]}] (cut to fit); GPU time log-uniform in "
                          f"[{ms_range[0]}, {ms_range[1]}] ms per request at the kind's FP32 rate; at least "
                          f"{min_walks} walks per query")
    if fp64_sample:
        # the same requests (a sample) alone through the plain per-solve FP64
        # path and again through the FP32 per-solve path: service times, and the
        # FP32 results compared bit for bit with the served ones
        idx = sorted(np.random.default_rng(seed + 1).choice(len(reqs), min(fp64_sample, len(reqs)), replace=False))
        s64, s32, same = [], [], 0
        print(f"[bench] served: {len(reqs)} requests in {wall:.1f} s; {len(idx)} alone per solve (FP64, FP32)",
              file=sys.stderr, flush=True)
        for i in idx:
            ta, name, Q, nw, sd = reqs[i]
            ts = time.perf_counter()
            mpwos.solve(probs[name], Q, nw, sd, manifold=mans[name], precision="fp64")
            s64.append(time.perf_counter() - ts)
            ts = time.perf_counter()
            r = mpwos.solve(probs[name], Q, nw, sd, manifold=mans[name], **opt)
            s32.append(time.perf_counter() - ts)
            same += int(np.array_equal(r["u"], outs[i]["u"]))
        # FIFO over the sampled requests' arrival times, time-scaled so that the
        # sample carries the full trace's offered load
        frac = len(idx) / len(reqs)

        def fifo(service):
            finish, lat_f = 0.0, []
            for i, sv in zip(idx, service):
                ta = reqs[i][0] * frac
                finish = max(finish, ta) + sv
                lat_f.append(finish - ta)
            return np.array(lat_f)

        f64, f32 = fifo(s64), fifo(s32)
        res["per_solve_fp64_fifo"] = {"requests_sampled": len(idx), "p50_ms": float(np.percentile(f64, 50) * 1e3),
                                      "p99_ms": float(np.percentile(f64, 99) * 1e3), "busy_s": float(sum(s64)),
                                      "walk_steps_per_s_vs_served": float(sum(s32)) / max(1e-9, float(sum(s64)))}
        res["per_solve_fp32_fifo"] = {"p50_ms": float(np.percentile(f32, 50) * 1e3),
                                      "p99_ms": float(np.percentile(f32, 99) * 1e3), "busy_s": float(sum(s32))}
        res["results_equal_alone"] = f"{same}/{len(idx)}"
        res["served_busy_s_sampled"] = float(sum(s32))
    for m in mans.values():
        m.close()
    return res


def backlog_growth(reqs, lat):
    """Growth of the latency over the window: each request's latency over the
    median latency of its manifold (all arrivals), then the median of that
    ratio over the last third of the arrivals over its median over the first
    third.  Near 1 while the server keeps up, growing with the backlog when
    it does not; normalising per manifold keeps the mix of manifolds that
    arrive in each third from moving it."""
    t = np.array([r[0] for r in reqs])
    kinds = np.array([r[1] for r in reqs])
    norm = np.array(lat, dtype=float)
    for name in set(kinds.tolist()):
        sel = kinds == name
        norm[sel] = norm[sel] / max(float(np.median(norm[sel])), 1e-12)
    lo, hi = np.percentile(t, 100 / 3), np.percentile(t, 200 / 3)
    a, b = norm[t <= lo], norm[t >= hi]
    if len(a) < 3 or len(b) < 3:
        return 1.0
    return float(np.median(b) / np.median(a))


def served_sweep(rates, window=20.0):
    """The served mix at several arrival rates (no per-solve runs).  A rate is
    stable when the latency, relative to each manifold's median, grows by no
    more than a fifth from the first third of the arrivals to the last
    (backlog_growth <= 1.2) and the queue drains within a tenth of the window
    after the last arrival."""
    runs = []
    for r in rates:
        runs.append(served_mix(rate=r, window=window, fp64_sample=0))
        print(f"[bench] served sweep: {r:g} req/s p50 {runs[-1]['p50_ms']:.0f} ms p99 {runs[-1]['p99_ms']:.0f} ms "
              f"drain {runs[-1]['drain_s']:.2f} s backlog growth {runs[-1]['backlog_growth']:.2f}", file=sys.stderr,
              flush=True)
    stable = [x["rate_req_per_s"] for x in runs
              if x["backlog_growth"] <= 1.2 and x["drain_s"] <= 0.1 * x["window_s"]]
    return {"runs": [{k: x[k] for k in ("rate_req_per_s", "window_s", "requests", "p50_ms", "p99_ms", "drain_s",
                                        "backlog_growth", "walk_steps_per_s", "launches", "closed_form_check",
                                        "by_manifold")}
                     for x in runs],
            "stability": "backlog_growth <= 1.2 and drain <= 0.1 window",
            "max_stable_rate_req_per_s": max(stable) if stable else None}


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


DESC = {
    "sphere": "unit sphere S^2: closed (u=x1x2, sigma=2, 4096 queries x 4096 walks) + cap x3>0 "
              "(Dirichlet g=u, sigma=0.5, eps=1e-3, 4096 x 4096)",
    "circle": "unit circle S^1: u=cos(3 theta), sigma=1, 64 queries x 1000 walks",
    "torus": "implicit torus R=1, a=0.3: u=sin(phi)cos(2psi), sigma=1, 8192 queries x 1024 walks",
    "cloud": "point-cloud torus, 1e6 points, noise 1e-4, k=16, quadratic patches fitted over 4 r_16: "
             "8192 queries x 1024 walks",
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
}


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
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay form of the headline step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--no-configs", action="store_true", help="skip the other configurations")
    ap.add_argument("--configs", default=",".join(CONFIGS), help="configurations of the configurations section")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None, help="time only one form (profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="time the library's plain copy kernel on BYTES (HBM calibration) and exit")
    ap.add_argument("--valu-probe", action="store_true", help="print the VALU operation rates and exit")
    ap.add_argument("--no-served", action="store_true", help="skip the served-mix leg")
    ap.add_argument("--served-window", type=float, default=30.0, help="seconds of arrivals at 200 req/s")
    ap.add_argument("--served-rates", default="100,200,300,400",
                    help="arrival rates (req/s) of the served sweep, 20 s windows; empty to skip")
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
        w, r = valu_weights_live()
        print(json.dumps({"lane_ops_per_s": r, "weights": w, "peak_lane_ops_per_s": PEAK_SLOTS}), flush=True)
        return
    if args.compensation_sweep:
        print(json.dumps(compensation_sweep([int(v) for v in args.compensation_sweep.split(",")])), flush=True)
        return
    if args.served_only:
        out = served_mix(window=args.served_window)
        if args.served_rates:
            out["sweep"] = served_sweep([float(x) for x in args.served_rates.split(",")])
        print(json.dumps(out), flush=True)
        return
    rank = int(os.environ.get("RANK", "0"))
    work = make_workload(args.workload, args.scale)
    prec = "fp64" if args.only == "fp64" else "fp32"
    tune = prec == "fp32" and not args.block_size and not args.launch
    fast = run_gpu(work, args.steps, args.warmup, prec, 0 if prec == "fp64" else 1, args.block_size,
                   graph=False, tune=tune, launch=parse_launch(args.launch))
    ws = fast["walk_steps_per_step"]
    ms = 1e3 * fast["seconds"] / fast["steps"]
    value = ws * fast["steps"] / fast["seconds"]
    nq_total = sum(p["n_queries"] for p in fast["per"].values())
    first = work[0]
    prob0 = first[1]
    desc = DESC[args.workload]
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
    kind0 = {"sphere": "sphere", "circle": "sphere", "hyper100": "sphere", "hyper1000": "sphere",
             "torus": "torus", "cloud": "cloud"}.get(args.workload)
    dom = fast["per"][first[0]]
    if kind0 == "cloud":
        out["roofline"] = roofline_cloud(first[0], dom["n_queries"], dom["n_walks"], dom["walk_steps"],
                                         dom["kernel_ms"], dom["launch"])
    elif kind0 is not None and prec == "fp32":
        out["roofline"] = roofline_alu(first[0], kind0, prob0["n"], prob0.get("n_v", 1), dom["walk_steps"],
                                       dom["kernel_ms"], dom["launch"])
        if args.workload == "sphere":
            cp = fast["per"]["cap"]
            out["roofline_cap"] = roofline_alu("cap", "cap", 3, 1, cp["walk_steps"], cp["kernel_ms"], cp["launch"])
    launch_used = {k: {kk: vv for kk, vv in v["launch"].items() if kk in ("persistent", "block_size")}
                   for k, v in fast["per"].items()}
    if prec == "fp32" and not args.no_graph and args.workload != "cut_torus":
        gr = run_gpu(work, args.steps, 1, "fp32", 1, graph=True, launch=launch_used)
        out["graph_replay"] = {"value": gr["walk_steps_per_step"] * gr["steps"] / gr["seconds"],
                               "ms_per_step": 1e3 * gr["seconds"] / gr["steps"],
                               "form": "each solve a captured HIP graph (mpwos_plan_execute) replayed per step"}
    if prec == "fp32" and args.only is None and args.workload == "sphere":
        out["host_io"] = host_io_rate(work, fast["per"])
    if not args.no_fp64 and args.only is None:
        slow = run_gpu(work, max(1, min(args.steps, 3)), 1, "fp64", 0)
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
    if args.workload == "sphere" and args.only is None and not args.no_configs:
        out["configs"] = measure_configs([c for c in args.configs.split(",") if c])
    if not args.no_served and args.workload == "sphere" and args.only is None:
        out["served"] = served_mix(window=args.served_window)
        if args.served_rates:
            out["served"]["sweep"] = served_sweep([float(x) for x in args.served_rates.split(",")])
    if not args.no_cpu and rank == 0:
        out["cpu_baseline"] = cpu_baseline(work, per_config=args.workload == "sphere")
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
