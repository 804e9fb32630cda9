"""The benchmark's cost model and contract pieces that need no GPU: the
algorithmic operation counts of a walk-step (the roofline's numerator), the
counter gate on the kernel sources' hash, and the single-GPU exit."""
import subprocess
import sys

import numpy as np
import pytest

import bench


def test_sphere_step_counts():
    ops = bench.step_ops("sphere", 3, 1)
    # two Philox blocks (direction, one Green sample): 20 multiply-adds and 20
    # three-way xors each; 60 FP32 operations, 10 transcendentals, 6 FP64
    assert ops == {"mad_u64_u32": 40, "bitop3_b32": 40, "f32": 60, "trans": 10, "f64": 6}
    # every extra Green sample adds a block and its sample work
    ops2 = bench.step_ops("sphere", 3, 2)
    assert ops2["mad_u64_u32"] == 60 and ops2["bitop3_b32"] == 60 and ops2["f32"] > ops["f32"]
    # the cap adds the boundary distance, two-slice table, the weight series and the radius
    cap = bench.step_ops("cap", 3, 1)
    assert cap["f32"] == ops["f32"] + 40 and cap["trans"] == ops["trans"] + 3
    # the torus replaces the sphere's projection by the level-set Newton steps
    tor = bench.step_ops("torus", 3, 1)
    assert tor["f32"] > ops["f32"] and tor["mad_u64_u32"] == 40


def test_high_dimension_step_counts():
    # n = 1000, N_V = 1: 250 blocks of normals for the direction, 251 for the
    # Green sample (its normals and the radius word); 1000 Box-Muller pairs
    ops = bench.step_ops("sphere", 1000, 1)
    assert ops["mad_u64_u32"] == 20 * 501 and ops["bitop3_b32"] == 20 * 501
    assert ops["trans"] == 4 * 1000 + 4 + 2
    assert ops["f32"] == 2 * 2001 + 3 * 1000 + 7 * 1000 + 18
    # n = 100: 25 + 26 blocks
    assert bench.step_ops("sphere", 100, 1)["mad_u64_u32"] == 20 * 51


def test_roofline_objects_and_counter_gate():
    r = bench.roofline_alu("sphere", "sphere", 3, 1, 2_919_235_584, 10.0, {"persistent": 0})
    assert r["bound"] == "alu" and r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    slots = sum(bench.step_ops("sphere", 3, 1)[k] * bench.SLOT_WEIGHTS[k] for k in bench.SLOT_WEIGHTS)
    assert r["achieved"] == pytest.approx(slots * 2_919_235_584 / 0.010 / 1e12)
    assert 0 < r["fp32_flop_frac"] < r["frac"]
    c = bench.roofline_cloud("cloud", 8192, 1024, 8192 * 1024 * 16, 1000.0, {"persistent": 1})
    assert c["bound"] == "hbm" and c["unit"] == "GB/s" and c["frac"] == pytest.approx(c["achieved"] * 1e9 / 8e12)
    # counter figures apply only to the kernel sources they were taken on
    saved = {k: v for k, v in bench.PROFILED.items()}
    try:
        bench.PROFILED["kernel_sha256"] = "0" * 64
        bench.PROFILED["kernels"] = {"sphere": {"valu_per_walk_step": 161.0, "walk_steps": 2_919_235_584,
                                                "fetch_kib": 456.0, "write_kib": 196608.0,
                                                "launch": {"persistent": 0, "block_size": 256}}}
        plain = {"persistent": 0, "block_size": 256, "lanes_per_walk": 1}
        r = bench.roofline_alu("sphere", "sphere", 3, 1, 2_919_235_584, 10.0, plain)
        assert r["traffic"] is None and "valu_issue_frac" not in r
        bench.PROFILED["kernel_sha256"] = bench.kernel_sha256()
        r = bench.roofline_alu("sphere", "sphere", 3, 1, 2_919_235_584, 10.0, plain)
        assert r["traffic"] == pytest.approx(1024 * (456.0 * 2.0 + 196608.0))
        assert r["valu_issue_frac"] == pytest.approx(161.0 * 2_919_235_584 / 0.010 / bench.PEAK_SLOTS)
        # ... and to the launch shape they were taken in
        r = bench.roofline_alu("sphere", "sphere", 3, 1, 2_919_235_584, 10.0, {"persistent": 1, "block_size": 256})
        assert r["traffic"] is None and "valu_issue_frac" not in r
    finally:
        bench.PROFILED.clear()
        bench.PROFILED.update(saved)


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True)
    assert p.returncode != 0 and "one GPU" in p.stderr


def test_backlog_growth_reads_a_growing_queue():
    # latency relative to each manifold's median, last third of the arrivals
    # over the first: steady latencies read 1 whatever the manifolds' own
    # levels, a queue whose latency grows with time reads the growth
    t = [i * 0.01 for i in range(300)]
    reqs = [(ti, "sphere" if i % 2 else "cap", None, 0, 0) for i, ti in enumerate(t)]
    steady = [0.05 if r[1] == "sphere" else 2.0 for r in reqs]
    assert bench.backlog_growth(reqs, np.array(steady)) == pytest.approx(1.0)
    growing = [(0.05 if r[1] == "sphere" else 2.0) * (1 + ti) for ti, r in zip(t, reqs)]
    g = bench.backlog_growth(reqs, np.array(growing))
    # medians of (1 + t) over the thirds: about 1.5 and 3.5
    assert 2.0 < g < 2.6
