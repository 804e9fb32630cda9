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
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_SLOTS = 256 * 64 * 2.4e9      # VALU lane-slots per second: 256 CUs x 64 lanes x 2.4 GHz


def slots_per_step(n, kind, precision, n_v=1):
    """Algorithmic VALU issue slots of one walk-step (model documented in the design doc).

    Philox4x32-10 block: 10 rounds x (2 wide multiplies at 4 slots + 2 three-way xors) = 100.
    Box-Muller pair: log, sqrt, sin, cos at 4 slots + 3 multiplies = 19.
    Per coordinate: sum of squares, scale-and-add, projection scale = 3 per vector pass.
    """
    nb_dir = (n + 3) // 4
    rw = 2 * ((n + 1) // 2)
    nb_green = max(nb_dir, rw // 4 + 1)
    pairs = (n + 1) // 2
    philox = 100 * (nb_dir + n_v * nb_green)
    words = 3 * (2 * pairs * (1 + n_v) + n_v)
    bm = 19 * pairs * (1 + n_v)
    vec = (3 * n + 8) * 2 * (1 + n_v)          # normalise + update + project, Theta and each Z
    radial = 60 if precision == "fp32" else 400
    source = 16
    accum = 12
    extra = 0
    if kind == "cap":
        extra = 25 + 100                         # delta_Gamma and the per-step weight series
        radial = 15 if precision == "fp32" else 600
    return philox + words + bm + vec + n_v * (radial + source) + accum + extra


def make_workload():
    from paper_2606_21883_amd import inputs
    ps, Qs, nws = inputs.config("sphere")
    pc, Qc, nwc = inputs.config("cap")
    return [("sphere", ps, Qs, nws), ("cap", pc, Qc, nwc)]


def run_gpu(work, steps, warmup, precision, persistent):
    import torch

    from paper_2606_21883_amd import inputs, mpwos
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    items = []
    for name, prob, Q, nw in work:
        m = mpwos.Manifold(prob)
        q = torch.from_numpy(np.ascontiguousarray(Q)).to(dev)
        u = torch.zeros(len(Q), dtype=torch.float64, device=dev)
        se = torch.zeros(len(Q), dtype=torch.float64, device=dev)
        items.append((name, prob, q, nw, m, u, se))

    def one_step():
        st = []
        for name, prob, q, nw, m, u, se in items:
            s = mpwos.solve_device(m, prob, q.data_ptr(), q.shape[0], nw, 0, u.data_ptr(), se.data_ptr(),
                                   stream=stream, precision=precision, persistent=persistent)
            st.append(s)
        return st

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [one_step() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = {"seconds": dt, "steps": steps}
    res["walk_steps_per_step"] = sum(s["walk_steps"] for s in stats[0])
    per = {}
    for i, (name, prob, q, nw, m, u, se) in enumerate(items):
        kms = float(np.mean([s[i]["kernel_ms"] for s in stats]))
        ws = stats[0][i]["walk_steps"]
        exact = inputs.exact_u(prob, q.cpu().numpy())
        per[name] = {"kernel_ms": kms, "walk_steps": ws, "k_mean": stats[0][i]["k_mean"],
                     "rmse": inputs.rmse(u.cpu().numpy(), exact),
                     "mean_stderr": float(np.sqrt(np.mean(se.cpu().numpy() ** 2))),
                     "n_queries": int(q.shape[0]), "n_walks": int(nw)}
    res["per"] = per
    for it in items:
        it[4].close()
    return res


def cpu_baseline(work, budget_s=20.0):
    """The FP64 oracle on the host cores over a bounded sample of the workload."""
    import oracle
    threads = os.cpu_count() or 1
    total_steps, total_t, parts = 0, 0.0, []
    for name, prob, Q, nw in work:
        nq, nws = (32, 512) if name == "sphere" else (32, 1536)
        t0 = time.perf_counter()
        r = oracle.solve(prob, Q[:nq], nws, 0, threads=threads)
        dt = time.perf_counter() - t0
        k = int(r["walk_K"].sum())
        total_steps += k
        total_t += dt
        parts.append(f"{name}: {nq} queries x {nws} walks ({k} walk-steps)")
        if total_t > budget_s:
            break
    return {"value": total_steps / total_t, "unit": "walk-steps/s", "cores": threads, "kind": "oracle",
            "sample": "; ".join(parts) + f"; {total_t:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None, help="time only one form (profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="time the library's plain copy kernel on BYTES (HBM calibration) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        from paper_2606_21883_amd import mpwos
        ms = mpwos.copy_probe(args.copy_probe, 5)
        print(json.dumps({"copy_bytes": args.copy_probe, "ms": ms,
                          "GB_per_s": 2 * args.copy_probe / (ms * 1e-3) / 1e9}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    work = make_workload()
    out = {}
    if args.only != "fp64":
        fast = run_gpu(work, args.steps, args.warmup, "fp32", 1)
    else:
        fast = run_gpu(work, args.steps, args.warmup, "fp64", 0)
    slow = None
    if not args.no_fp64 and args.only is None:
        slow = run_gpu(work, max(1, min(args.steps, 3)), 1, "fp64", 0)
    ws = fast["walk_steps_per_step"]
    ms = 1e3 * fast["seconds"] / fast["steps"]
    value = ws * fast["steps"] / fast["seconds"]
    nq_total = sum(p["n_queries"] for p in fast["per"].values())
    prec = "fp32" if args.only != "fp64" else "fp64"
    dom = fast["per"]["sphere"]
    slots = slots_per_step(3, "sphere", prec)
    achieved = slots * dom["walk_steps"] / (dom["kernel_ms"] * 1e-3) / 1e12
    out = {
        "metric": "walk-steps/s", "value": value, "unit": "walk-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32" if prec == "fp32" else "fp64",
        "data": "synthetic",
        "config": {"workload": "unit sphere S^2: closed (u=x1x2, sigma=2, 4096 queries x 4096 walks) + "
                               "cap x3>0 (Dirichlet g=u, sigma=0.5, eps=1e-3, 4096 x 4096)",
                   "precision": "fp32 walk, fp64 weights/scores" if prec == "fp32" else "fp64",
                   "form": "persistent queue-refill" if prec == "fp32" else "plain",
                   "n_v": 1, "tau_w": 1e-8, "theta": 0.95, "c_kappa": 1.2, "parallelism": "single-gpu"},
        "queries_per_s": nq_total * fast["steps"] / fast["seconds"],
        "per_solve": fast["per"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_SLOTS / 1e12, "unit": "Tslot/s",
                     "frac": achieved / (PEAK_SLOTS / 1e12), "traffic": None,
                     "kernel": "walk_lane_kernel<float,3,sphere> (persistent)",
                     "slots_per_walk_step": slots},
    }
    if slow is not None:
        v64 = slow["walk_steps_per_step"] * slow["steps"] / slow["seconds"]
        out["fp64_plain"] = {"value": v64, "ms_per_step": 1e3 * slow["seconds"] / slow["steps"],
                             "per_solve": slow["per"]}
        out["speedup_vs_fp64_plain"] = value / v64
        out["rmse_ratio_fp32_over_fp64"] = {k: fast["per"][k]["rmse"] / slow["per"][k]["rmse"]
                                            for k in fast["per"]}
    if not args.no_cpu and rank == 0:
        out["cpu_baseline"] = cpu_baseline(work)
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
