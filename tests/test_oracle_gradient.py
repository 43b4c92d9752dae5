"""Pins of the gradient oracle (magnitude / direction with the 2x2 and 3x3
masks) and of the residual-based multi-scale rule."""
import math

import numpy as np
import pytest
import scipy.signal

import oracle as O


def ramp(H, W, a, b):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    return a * x + b * y


def test_worked_2x2():
    # E = [[1, 3], [5, 9]]: E_x = ((3-1) + (9-5)) / 2 = 3, E_y = ((5-1) + (9-3)) / 2 = 5
    g = O.gradient(np.array([[1.0, 3.0], [5.0, 9.0]]), "fd2")
    assert g["ex"][0, 0] == 3.0 and g["ey"][0, 0] == 5.0
    assert g["mag"][0, 0] == math.sqrt(34.0)
    assert g["dir"][0, 0] == math.atan2(5.0, 3.0)


RAMPS = [(1.0, 0.0), (0.0, 1.0), (2.0, -3.0), (-1.5, -0.5)]


def ramp_pin_holds(stencil, a, b):
    """The ramp E = a x + b y has gradient (a, b): magnitude hypot(a, b) and
    direction atan2(b, a) (turned by -45 degrees for the diagonal Roberts axes)."""
    g = O.gradient(ramp(9, 11, a, b), stencil)
    ok = np.allclose(g["mag"], math.hypot(a, b), rtol=0, atol=1e-12)
    want = math.atan2(b, a)
    if stencil == "roberts":
        want = math.atan2(math.sin(want - math.pi / 4), math.cos(want - math.pi / 4))
    else:
        ok &= np.allclose(g["ex"], a, atol=1e-12) and np.allclose(g["ey"], b, atol=1e-12)
    return ok and np.allclose(g["dir"], want, atol=1e-12)


@pytest.mark.parametrize("stencil", O.STENCILS)
@pytest.mark.parametrize("a,b", RAMPS)
def test_ramps(stencil, a, b):
    assert ramp_pin_holds(stencil, a, b)


def _transposed(masks):
    return lambda st: tuple(reversed(masks(st)))


def _sobel_center_1(masks):
    def f(st):
        mx, my = masks(st)
        if st == "sobel3":
            mx = mx.copy()
            mx[1] /= 2.0
            my = mx.T.copy()
        return mx, my
    return f


def _roberts_unscaled(masks):
    def f(st):
        mx, my = masks(st)
        return (mx * math.sqrt(2.0), my * math.sqrt(2.0)) if st == "roberts" else (mx, my)
    return f


@pytest.mark.parametrize("mutation", ["swapped_atan2", "transposed_masks", "sobel_center_1", "roberts_unscaled"])
def test_ramp_pins_catch_planted_mistakes(monkeypatch, mutation):
    """Each plausible mistake planted in the oracle fails at least one ramp pin."""
    import sys

    G = sys.modules["oracle.gradient"]  # the package re-exports a function of the same name

    if mutation == "swapped_atan2":
        real = np.arctan2
        monkeypatch.setattr(G, "np", type("np_swapped", (), {"__getattr__": lambda self, n: getattr(np, n),
                                                             "arctan2": staticmethod(lambda y, x: real(x, y))})())
    elif mutation == "transposed_masks":
        monkeypatch.setattr(G, "masks", _transposed(G.masks))
    elif mutation == "sobel_center_1":
        monkeypatch.setattr(G, "masks", _sobel_center_1(G.masks))
    else:
        monkeypatch.setattr(G, "masks", _roberts_unscaled(G.masks))
    assert not all(ramp_pin_holds(st, a, b) for st in O.STENCILS for a, b in RAMPS)


@pytest.mark.parametrize("stencil", O.STENCILS)
def test_masks_are_correlations(stencil):
    rng = np.random.default_rng(5)
    img = rng.uniform(0, 255, (13, 17))
    mx, my = O.masks(stencil)
    g = O.gradient(img, stencil)
    assert np.allclose(g["ex"], scipy.signal.correlate2d(img, mx, mode="valid"), atol=1e-9)
    assert np.allclose(g["ey"], scipy.signal.correlate2d(img, my, mode="valid"), atol=1e-9)
    assert np.all(np.abs(g["dir"]) <= math.pi)


def test_fd2_is_the_cube_of_a_still_pair():
    # with both frames equal, the 2x2x2 cube's spatial derivatives are the 2x2 mask's
    rng = np.random.default_rng(6)
    img = rng.integers(0, 256, (10, 12)).astype(np.float64)
    ex, ey, et = O.horn(img, img)
    g = O.gradient(img, "fd2")
    assert np.array_equal(ex, g["ex"]) and np.array_equal(ey, g["ey"]) and not et.any()


def test_sobel_is_separable_smoothing_times_difference():
    rng = np.random.default_rng(7)
    img = rng.uniform(0, 1, (12, 14))
    g = O.gradient(img, "sobel3")
    rows = scipy.signal.correlate2d(img, np.array([[-1.0, 0.0, 1.0]]) / 2.0, mode="valid")
    smooth = scipy.signal.correlate2d(rows, np.array([[1.0], [2.0], [1.0]]) / 4.0, mode="valid")
    assert np.allclose(g["ex"], smooth, atol=1e-12)


def _rec(ttc, status, resid, n):
    return {"ttc": ttc, "status": status, "resid": resid, "n": n}


def test_residual_rule():
    recs = [_rec(10.0, 0, 100.0, 100), _rec(8.0, 0, 30.0, 20), _rec(12.0, 0, 1.0, 5)]
    assert O.select_level_residual(recs) == 2      # 1.0, 1.5, 0.2 per cube
    assert O.select_level(recs) == 1               # the decreasing-TTC rule differs
    recs[2]["status"] = O.STATUS_SINGULAR
    assert O.select_level_residual(recs) == 0
    recs[0]["ttc"] = -3.0                          # a non-positive TTC is not valid
    assert O.select_level_residual(recs) == 1
    assert O.select_level_residual([_rec(math.nan, 1, math.nan, 4)] * 3) == 0
    tie = [_rec(5.0, 0, 2.0, 2), _rec(4.0, 0, 4.0, 4)]
    assert O.select_level_residual(tie) == 0       # the lower level on a tie
