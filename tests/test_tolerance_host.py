"""CPU checks of the parity tolerances themselves (tests/tolerance.py): the
first-order bounds on (A, B, C), TTC, FOE and the residual must cover what the
oracle's own solve gives when every sum moves by up to its stated bound
TAU_SUM * sum|terms|, including the worst sign pattern of each sensitivity."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_1612_08825_amd import synth
from tolerance import TAU_SUM, abs_sums, resid_bound, solution_bounds


def _levels():
    v = synth.multiscale_video(case=3, H=96, W=128, F=3, foe=(12.0, -8.0), ttc_start=40, ttc_end=38)
    P0, P1 = v.frames[0], v.frames[1]
    H0, W0 = P0.shape
    p0, p1 = O.pyramid(P0, 3), O.pyramid(P1, 3)
    out = []
    for l in range(3):
        s, _ = O.level_sums(p0[l], p1[l], l, H0, W0)
        a = abs_sums(p0[l], p1[l], l, H0, W0)
        out.append((np.asarray(s, dtype=np.float64), a))
    return out


@pytest.mark.parametrize("level", [0, 1, 2])
def test_bounds_cover_perturbed_solves(level):
    s, a = _levels()[level]
    ref = O.solve_level(s)
    assert ref["status"] == O.STATUS_OK
    b = solution_bounds(s, a)
    rb = resid_bound(s, a)
    rng = np.random.default_rng(level)
    # random perturbations within the bound, and the sign patterns that push
    # each output furthest (+/- on every sum, 2^10 of them)
    deltas = [rng.uniform(-1, 1, 10) for _ in range(200)]
    deltas += [np.array(sg, dtype=np.float64) for sg in itertools.product((-1.0, 1.0), repeat=10)]
    worst = dict(A=0.0, B=0.0, C=0.0, ttc=0.0, x0=0.0, y0=0.0, resid=0.0)
    for d in deltas:
        sp = s + d * TAU_SUM * a
        r = O.solve_level(sp)
        assert r["status"] == O.STATUS_OK
        for key in ("A", "B", "C", "ttc", "x0", "y0"):
            worst[key] = max(worst[key], abs(r[key] - ref[key]) / b[key])
        worst["resid"] = max(worst["resid"], abs(r["resid"] - ref["resid"]) / rb)
    # the bounds carry a safety factor of 2 over first order: the worst
    # perturbed solve stays inside, and the bound is not vacuous (within 10x)
    for key, w in worst.items():
        assert w <= 1.0, (key, w)
        assert w >= 0.05, (key, w)


def test_resid_bound_catches_a_wrong_residual():
    """A residual computed without one of its terms (C s8 dropped) is far
    outside the bound."""
    s, a = _levels()[0]
    ref = O.solve_level(s)
    wrong = ref["resid"] - ref["C"] * s[8]
    assert abs(wrong - ref["resid"]) > 100 * resid_bound(s, a)
    assert math.isfinite(ref["resid"])
