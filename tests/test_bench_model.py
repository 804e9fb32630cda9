"""The benchmark's cost model and contract pieces that need no GPU: the
algorithmic operation counts of a walk-step (the roofline's numerator), the
traffic gate on the kernel sources' hash, and the single-GPU exit."""
import subprocess
import sys

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
    # the cap adds the boundary distance, two-slice table and the per-step weights
    cap = bench.step_ops("cap", 3, 1)
    assert cap["f64"] > ops["f64"] and cap["f32"] > ops["f32"]


def test_traffic_constants_follow_the_kernel_sources():
    # the counters are used only for the sources they were taken on
    assert len(bench.kernel_sha256()) == 64
    fake = {"sphere": {"walk_steps": 4096 * 4096 * 174, "kernel_ms": 10.0, "launch": {"persistent": 0}}}
    saved = dict(bench.TRAFFIC)
    try:
        bench.TRAFFIC["kernel_sha256"] = "0" * 64
        bench.valu_weights = lambda: ({k: 1.0 for k in ("f32", "bitop3_b32", "f64", "trans", "mad_u64_u32")}, {})
        r = bench.roofline({"per": fake, "form": "graph replay"}, "sphere", "sphere", 3, 1, "fp32")
        assert r["traffic"] is None and r["bound"] == "alu"
        assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
        bench.TRAFFIC["kernel_sha256"] = bench.kernel_sha256()
        r = bench.roofline({"per": fake, "form": "graph replay"}, "sphere", "sphere", 3, 1, "fp32")
        assert r["traffic"] == pytest.approx(1024 * (saved["fetch_kib"] * saved["fetch_factor"] +
                                                     saved["write_kib"] * saved["write_factor"]))
    finally:
        bench.TRAFFIC.clear()
        bench.TRAFFIC.update(saved)
        import importlib
        importlib.reload(bench)


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True)
    assert p.returncode != 0 and "one GPU" in p.stderr
