"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np


def announce(msg):
    """Names the case on the real stderr before a GPU step (survives a crash)."""
    sys.__stderr__.write(f"[gpu-case] {msg}\n")
    sys.__stderr__.flush()


def score_scale(prob):
    """Bound of sum_k W_k omega_k |F_k| (<= max|f + m| / sigma) plus the boundary term."""
    f = prob.get("f", {})
    s = 1.0 + sum(abs(c) for c in f.get("coef", [0.0])) / prob["sigma"]
    if f.get("kind") == "torus_mode":
        R, a = prob["p"][:2]
        fmax = 4 / a ** 2 + 1 / (R - a) ** 2 + 2 / (a * (R - a)) + prob["sigma"]
        s = 1.0 + abs(f["coef"][0]) * 2 * fmax / prob["sigma"]
    if "values" in prob.get("f", {}):
        s += float(np.max(np.abs(prob["f"]["values"]))) * 2 / prob["sigma"]
    if prob["manifold"] in ("sphere_cap", "cut_torus"):
        s += sum(abs(c) for c in prob.get("g", {}).get("coef", [0.0]))
    return s


def compare_walks(gpu, orc, prob, tol=1e-12, min_frac=0.999):
    """Walk agreement (same K, |dS| <= tol * scale) on >= min_frac of the walks,
    and per-query means over agreeing walks within 1e-10 relative."""
    gS, gK = gpu["walk_S"], gpu["walk_K"]
    oS, oK = orc["walk_S"], orc["walk_K"]
    scale = score_scale(prob)
    agree = (gK == oK) & (np.abs(gS - oS) <= tol * scale)
    frac = float(agree.mean())
    assert frac >= min_frac, (frac, np.argwhere(~agree)[:5], np.max(np.abs(gS - oS)))
    for q in range(gS.shape[0]):
        m = agree[q]
        if not m.any():
            continue
        mg, mo = gS[q, m].mean(), oS[q, m].mean()
        ref = max(abs(mo), np.abs(oS[q]).mean(), 1e-300)
        assert abs(mg - mo) <= 1e-10 * ref, (q, mg, mo)
    return frac
