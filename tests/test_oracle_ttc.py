"""Pins of the least-squares TTC/FOE oracle: a hand-worked system, LAPACK and
exact-rational Cramer's rule for the solve, exact rational sums, symmetry
invariants of the sums, the point-symmetric video (A = B = 0 exactly), the
singular ramp video, and the analytic ground truth of approaching-plane videos.
The last group also plants mistakes in a copy of the oracle and checks that the
pins catch them."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle import ttc as T
from paper_1612_08825_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_normal_equations():
    g = json.load(open(os.path.join(GOLDEN, "normal_equations_worked.json")))
    r = O.solve_level(g["sums"])
    assert r["status"] == O.STATUS_OK
    for key, val in g["expected"].items():
        assert r[key] == pytest.approx(val, rel=1e-14, abs=1e-14), key


def _cramer(M, r):
    M = [[Fraction(v) for v in row] for row in M]
    r = [Fraction(v) for v in r]

    def det(a):
        return (a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1])
                - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
                + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]))

    d = det(M)
    out = []
    for c in range(3):
        a = [row[:] for row in M]
        for i in range(3):
            a[i][c] = r[i]
        out.append(det(a) / d)
    return out


def test_solve3_vs_lapack_and_cramer():
    rng = np.random.default_rng(11)
    for _ in range(50):
        X = rng.standard_normal((20, 3)) * rng.uniform(0.1, 100, 3)
        M = X.T @ X
        r = rng.standard_normal(3)
        v, piv = O.solve3(M, r)
        np.testing.assert_allclose(v, np.linalg.solve(M, r), rtol=1e-9, atol=1e-12)
        exact = [float(q) for q in _cramer(M, r)]
        np.testing.assert_allclose(v, exact, rtol=1e-9, atol=1e-12)
    # a permutation that needs pivoting
    v, _ = O.solve3([[0, 1, 0], [1, 0, 0], [0, 0, 2]], [3, 4, 8])
    assert v == [4.0, 3.0, 4.0]


def _small_video(levels_ok=3, dtype="u8"):
    return synth.multiscale_video(H=48, W=64, F=2, foe=(6.0, -4.0), ttc_start=30, ttc_end=29, dtype=dtype)


@pytest.mark.parametrize("dtype", ["u8", "f16"])
def test_sums_match_exact_rationals(dtype):
    v = _small_video(dtype=dtype)
    p0 = O.pyramid(v.frames[0], 3)
    p1 = O.pyramid(v.frames[1], 3)
    for l in range(3):
        s, n = O.level_sums(p0[l], p1[l], l, 48, 64)
        ex, ne = O.level_sums_exact(p0[l], p1[l], l, 48, 64)
        assert n == ne == (p0[l].shape[0] - 1) * (p0[l].shape[1] - 1)
        for a, b in zip(s, ex):
            # products of levels <= 2 are exact in FP64, so the fsum result is the correctly rounded exact sum
            assert a == float(b)


def test_solution_vs_exact_cramer():
    v = _small_video()
    p0 = O.pyramid(v.frames[0], 2)
    p1 = O.pyramid(v.frames[1], 2)
    for l in range(2):
        ex, _ = O.level_sums_exact(p0[l], p1[l], l, 48, 64)
        M = [[ex[0], ex[1], ex[3]], [ex[1], ex[2], ex[4]], [ex[3], ex[4], ex[5]]]
        abc = _cramer(M, [-ex[6], -ex[7], -ex[8]])
        r = O.solve_level([float(q) for q in ex])
        np.testing.assert_allclose([r["A"], r["B"], r["C"]], [float(q) for q in abc], rtol=1e-10)
        resid = float(ex[9] + abc[0] * ex[6] + abc[1] * ex[7] + abc[2] * ex[8])
        assert r["resid"] == pytest.approx(resid, rel=1e-8)
        # the residual identity against a direct evaluation of sum (A Ex + B Ey + C G + Et)^2
        exx, eyy, ett, gg = O.level_terms(p0[l], p1[l], l, 48, 64)
        direct = math.fsum(((r["A"] * exx + r["B"] * eyy + r["C"] * gg + ett) ** 2).ravel().tolist())
        assert r["resid"] == pytest.approx(direct, rel=1e-7)


def _sums(P0, P1, level=0):
    H0, W0 = P0.shape
    p0 = O.pyramid(P0, level + 1)
    p1 = O.pyramid(P1, level + 1)
    return O.level_sums(p0[level], p1[level], level, H0, W0)[0]


@pytest.mark.parametrize("level", [0, 1, 2])
def test_mirror_invariants(level):
    v = synth.plain_ttc_video(H=64, W=64, F=2)
    a = _sums(v.frames[0], v.frames[1], level)
    m = _sums(v.frames[0][:, ::-1], v.frames[1][:, ::-1], level)
    sign = np.array([1, -1, 1, -1, 1, 1, -1, 1, 1, 1])  # odd in E_x: ExEy, GEx, ExEt
    np.testing.assert_array_equal(m, sign * a)
    t = _sums(v.frames[0].T, v.frames[1].T, level)
    perm = [2, 1, 0, 4, 3, 5, 7, 6, 8, 9]  # x <-> y
    np.testing.assert_array_equal(t, a[perm])
    r = _sums(v.frames[1], v.frames[0], level)
    tsign = np.array([1, 1, 1, 1, 1, 1, -1, -1, -1, 1])  # time reversal flips E_t
    np.testing.assert_array_equal(r, tsign * a)
    o = _sums(v.frames[0].astype(np.float64) + 9, v.frames[1].astype(np.float64) + 9, level)
    np.testing.assert_array_equal(o, a)


def test_symmetric_video_closed_form():
    v = synth.plain_ttc_video(H=64, W=80, F=2, symmetric=True)
    f0 = v.frames[0]
    np.testing.assert_array_equal(f0, f0[::-1, ::-1])  # rendered bit-symmetric
    for l in range(3):
        s = _sums(v.frames[0], v.frames[1], l)
        assert s[6] == 0 and s[7] == 0 and s[3] == 0 and s[4] == 0
        r = O.solve_level(s)
        assert r["A"] == 0.0 and r["B"] == 0.0
        assert r["C"] == pytest.approx(-s[8] / s[5], rel=1e-14)


def test_ramp_video_is_singular():
    i, j = np.meshgrid(np.arange(32), np.arange(40), indexing="ij")
    P0 = (2 * j + i + 20).astype(np.uint8)
    P1 = (2 * j + i + 23).astype(np.uint8)
    for r in O.ttc_pair(P0, P1, 3):
        assert r["status"] == O.STATUS_SINGULAR
        assert math.isnan(r["ttc"])


def test_nonfinite_status():
    r = O.solve_level([1, 0, 1, 0, 0, 1, math.nan, 0, 0, 1])
    assert r["status"] == O.STATUS_NONFINITE


def test_selection_rule():
    def mk(ts):
        return [dict(ttc=t, status=O.STATUS_OK if not math.isnan(t) else O.STATUS_SINGULAR) for t in ts]

    assert O.select_level(mk([50, 45, 47, 30])) == 1
    assert O.select_level(mk([50, 45, 40, 30])) == 3
    assert O.select_level(mk([60, -5, 40])) == 0
    assert O.select_level(mk([math.nan, 30, 20])) == 2
    assert O.select_level(mk([30])) == 0
    assert O.select_level(mk([30, 30])) == 0


# ---------------------------------------------------------------------------
# Ground truth of approaching-plane videos, and planted mistakes
# ---------------------------------------------------------------------------
def _gt_checks(module):
    """True when the chain recovers the analytic TTC and FOE of two videos."""
    v = synth.plain_ttc_video(H=96, W=96, F=3)
    ok = True
    for res in module.ttc_sequence(v.frames, 1):
        r = res[0][0]
        ok &= abs(r["ttc"] - 40.0) < 0.05 * 40.0 and abs(r["x0"]) < 0.5 and abs(r["y0"]) < 0.5
    w = synth.multiscale_video(H=120, W=160, F=2, foe=(20.0, -10.0), ttc_start=60, ttc_end=50)
    gt = w.ttc_gt()[0]
    for r in module.ttc_pair(w.frames[0], w.frames[1], 3):
        ok &= abs(r["ttc"] - gt) < 0.15 * gt and abs(r["x0"] - 20.0) < 1.5 and abs(r["y0"] + 10.0) < 2.0
    return bool(ok)


def test_ground_truth_recovered():
    assert _gt_checks(T)


@pytest.mark.parametrize("mutation", ["et_sign", "swap_xy", "no_level_scale", "g_sign", "rhs_sign"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    """Each mistake is planted in the oracle (CPU only) and must break a pin."""
    if mutation == "et_sign":
        orig = T.horn
        monkeypatch.setattr(T, "horn", lambda a, b: (lambda e: (e[0], e[1], -e[2]))(orig(a, b)))
    elif mutation == "swap_xy":
        orig_terms = T.level_terms

        def terms(P0, P1, level, H0, W0):
            ex, ey, et, _ = orig_terms(P0, P1, level, H0, W0)
            x, y = T.cube_coords(level, P0.shape[0], P0.shape[1], H0, W0)
            return ex, ey, et, y[:, None] * ex + x[None, :] * ey  # G with the coordinates exchanged

        monkeypatch.setattr(T, "level_terms", terms)
    elif mutation == "no_level_scale":
        orig_terms = T.level_terms

        def terms(P0, P1, level, H0, W0):
            ex, ey, et, g = orig_terms(P0, P1, level, H0, W0)
            s = float(2 ** level)
            ex, ey = ex * s, ey * s
            x, y = T.cube_coords(level, P0.shape[0], P0.shape[1], H0, W0)
            return ex, ey, et, x[None, :] * ex + y[:, None] * ey

        monkeypatch.setattr(T, "level_terms", terms)
    elif mutation == "g_sign":
        orig_terms = T.level_terms
        monkeypatch.setattr(T, "level_terms", lambda *a: (lambda q: (q[0], q[1], q[2], -q[3]))(orig_terms(*a)))
    elif mutation == "rhs_sign":
        orig_nm = T.normal_matrix
        monkeypatch.setattr(T, "normal_matrix", lambda s: (lambda m: (m[0], [-v for v in m[1]]))(orig_nm(s)))
    assert not _gt_checks(T)
