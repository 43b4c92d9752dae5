"""Comparison of one pair's GPU level records and multi-scale pick with the
FP64 oracle, shared by the GPU parity tests of the batched plan and of the
serving loop.  Bounds: tests/tolerance.py."""
import math

import numpy as np
import torch

import oracle as O
from tolerance import TAU_SUM, abs_sums, resid_bound, solution_bounds

WORST = {"sum": 0.0, "C": 0.0, "foe": 0.0, "resid": 0.0}


def _frames_np(frames):
    return frames.cpu().numpy() if isinstance(frames, torch.Tensor) else np.asarray(frames)


def check_pair(rec, pick, P0, P1, levels, tag=""):
    """Compare one pair's GPU level records and pick with the oracle."""
    H0, W0 = P0.shape
    ref = O.ttc_pair(P0, P1, levels)
    p0 = O.pyramid(P0, levels)
    p1 = O.pyramid(P1, levels)
    for l in range(levels):
        r, g = ref[l], rec[l]
        assert g["level"] == l
        assert g["n"] == r["n"]
        assert g["status"] == r["status"], (tag, l, g["status"], r["status"])
        a = abs_sums(p0[l], p1[l], l, H0, W0)
        err = np.abs(g["sums"] - r["sums"])
        rel = float(np.max(err / np.maximum(a, 1e-300)))
        WORST["sum"] = max(WORST["sum"], rel)
        assert np.all(err <= TAU_SUM * a + 1e-300), (tag, l, rel)
        if r["status"] != O.STATUS_OK:
            assert math.isnan(g["ttc"])
            continue
        b = solution_bounds(r["sums"], a)
        for key in ("A", "B", "C", "ttc", "x0", "y0"):
            assert abs(g[key] - r[key]) <= b[key], (tag, l, key, g[key], r[key], b[key])
        WORST["C"] = max(WORST["C"], abs(g["C"] - r["C"]) / abs(r["C"]))
        WORST["foe"] = max(WORST["foe"], abs(g["x0"] - r["x0"]), abs(g["y0"] - r["y0"]))
        rb = resid_bound(r["sums"], a)
        WORST["resid"] = max(WORST["resid"], abs(g["resid"] - r["resid"]) / rb)
        assert abs(g["resid"] - r["resid"]) <= rb, (tag, l, g["resid"], r["resid"], rb)
    sel = O.select_level(ref)
    ttcs = [r["ttc"] for r in ref]
    near_tie = any(abs(ttcs[i + 1] - ttcs[i]) <= solution_bounds(ref[i]["sums"], abs_sums(p0[i], p1[i], i, H0, W0))["ttc"]
                   + solution_bounds(ref[i + 1]["sums"], abs_sums(p0[i + 1], p1[i + 1], i + 1, H0, W0))["ttc"]
                   for i in range(levels - 1) if ref[i]["status"] == 0 and ref[i + 1]["status"] == 0)
    if not near_tie:
        assert pick["level"] == sel, (tag, pick["level"], sel, ttcs)
        assert pick["ttc"] == rec[sel]["ttc"]
