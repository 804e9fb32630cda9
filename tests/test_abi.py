"""C ABI checks that need no GPU: the library loads, exports every entry point
declared in include/mpwos.h, and the ctypes binding's struct layouts match the
header (sizes and field offsets measured by a small C program built with gcc)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2606_21883_amd import mpwos

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpwos.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mpwos_[a-z_0-9]+)\s*\(", txt)))


def test_library_loads_and_exports_every_declared_symbol():
    L = mpwos.lib()
    names = declared_functions()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(mpwos.EXPORTS)


def test_library_has_gfx950_code_object():
    # the library built here embeds its device code object for gfx950
    data = open(mpwos.LIBPATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_options_default_values():
    o = mpwos.options_default()
    assert o.theta == 0.95 and o.c_kappa == 1.2 and o.c_h == 2.4 and o.tau_w == 1e-8
    assert o.n_v == 1 and o.precision == 0 and o.compensation == 1 and o.max_steps == 10_000_000


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "mpwos.h"
#define P(T) printf(#T " %zu\n", sizeof(T));
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  P(mpwos_manifold_desc) P(mpwos_fn) P(mpwos_options) P(mpwos_stats) P(mpwos_request) P(mpwos_server_stats)
  O(mpwos_options, max_steps) O(mpwos_options, stream) O(mpwos_options, walk_S) O(mpwos_options, walk_K)
  O(mpwos_fn, values) O(mpwos_fn, n_values) O(mpwos_manifold_desc, points) O(mpwos_manifold_desc, k_nn)
  O(mpwos_manifold_desc, fit_scale)
  O(mpwos_request, opt) O(mpwos_request, u_out) O(mpwos_request, seed) O(mpwos_stats, kernel_ms)
  O(mpwos_stats, k_p50) O(mpwos_stats, k_p99)
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    got = {k: int(v) for k, v in got.items()}
    m = mpwos
    assert got["mpwos_manifold_desc"] == ctypes.sizeof(m.ManifoldDesc)
    assert got["mpwos_fn"] == ctypes.sizeof(m.Fn)
    assert got["mpwos_options"] == ctypes.sizeof(m.Options)
    assert got["mpwos_stats"] == ctypes.sizeof(m.Stats)
    assert got["mpwos_request"] == ctypes.sizeof(m.Request)
    assert got["mpwos_server_stats"] == ctypes.sizeof(m.ServerStats)
    for key, (cls, field) in {
        "mpwos_options.max_steps": (m.Options, "max_steps"), "mpwos_options.stream": (m.Options, "stream"),
        "mpwos_options.walk_S": (m.Options, "walk_S"), "mpwos_options.walk_K": (m.Options, "walk_K"),
        "mpwos_fn.values": (m.Fn, "values"), "mpwos_fn.n_values": (m.Fn, "n_values"),
        "mpwos_manifold_desc.points": (m.ManifoldDesc, "points"),
        "mpwos_manifold_desc.k_nn": (m.ManifoldDesc, "k_nn"), "mpwos_request.opt": (m.Request, "opt"),
        "mpwos_manifold_desc.fit_scale": (m.ManifoldDesc, "fit_scale"),
        "mpwos_request.u_out": (m.Request, "u_out"), "mpwos_request.seed": (m.Request, "seed"),
        "mpwos_stats.kernel_ms": (m.Stats, "kernel_ms"), "mpwos_stats.k_p50": (m.Stats, "k_p50"),
        "mpwos_stats.k_p99": (m.Stats, "k_p99"),
    }.items():
        assert got[key] == getattr(cls, field).offset, key


def test_enum_values_match_header():
    txt = open(HEADER).read()
    for name, val in [("MPWOS_SPHERE", 0), ("MPWOS_SPHERE_CAP", 1), ("MPWOS_TORUS_IMPLICIT", 2),
                      ("MPWOS_POINT_CLOUD", 3), ("MPWOS_DUMBBELL", 4), ("MPWOS_FN_SPH_PAIR", 2),
                      ("MPWOS_FN_TABLE_S1", 6), ("MPWOS_FN_DUMBBELL_POLY", 7),
                      ("MPWOS_FP32_MIXED", 1), ("MPWOS_EOFFMANIFOLD", -2), ("MPWOS_WTRUNC", 1),
                      ("MPWOS_PRODUCT", 5), ("MPWOS_CUT_TORUS", 6), ("MPWOS_FN_TORUS_SINE", 9),
                      ("MPWOS_COMP_SECOND_ORDER", 2)]:
        assert re.search(rf"\b{name}\s*=\s*{val}\b", txt), name
    assert mpwos.KINDS == {"sphere": 0, "sphere_cap": 1, "torus": 2, "point_cloud": 3, "dumbbell": 4, "product": 5,
                           "cut_torus": 6}
    assert mpwos.FN_KINDS["torus_sine"] == 9 and mpwos.COMP["second_order"] == 2
    assert mpwos.FN_KINDS["table_s1"] == 6 and mpwos.FN_KINDS["torus_mode"] == 5
    assert mpwos.FN_KINDS["dumbbell_poly"] == 7 and mpwos.FN_KINDS["product_modes"] == 8


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(mpwos, "_lib", None)
    monkeypatch.setattr(mpwos, "LIBPATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        mpwos.lib()
