"""Pins of the TTC oracle with the 3x3 derivative stencils and the pyramid
low-pass filter (oracle/variant.py)."""
import math
import sys

import numpy as np
import pytest
import scipy.ndimage

import oracle as O
from oracle import variant as V
from paper_1612_08825_amd import synth

VM = sys.modules["oracle.variant"]


def test_lowpass_worked_corner():
    # a unit impulse in the corner of a 3x3 image: the clamped border repeats
    # it under the four taps (-1,-1), (-1,0), (0,-1), (0,0)
    img = np.zeros((3, 3))
    img[0, 0] = 1.0
    out = V.lowpass_binomial3(img)
    assert out[0, 0] == 0.0625 + 0.125 + 0.125 + 0.25
    assert out[1, 1] == 0.0625 and out[0, 1] == 0.125 + 0.0625 and out[2, 2] == 0.0


def lowpass_pins_hold():
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 255, (11, 14))
    w = np.array([1.0, 2.0, 1.0]) / 4.0
    ref = scipy.ndimage.correlate(img, np.outer(w, w), mode="nearest")
    ok = np.allclose(V.lowpass_binomial3(img), ref, rtol=0, atol=1e-12)
    ok &= np.array_equal(V.lowpass_binomial3(np.full((5, 7), 9.5)), np.full((5, 7), 9.5))
    return bool(ok)


def test_lowpass_is_clamped_binomial():
    assert lowpass_pins_hold()


def test_pyramid_without_lowpass_is_block_mean():
    rng = np.random.default_rng(4)
    P = rng.integers(0, 256, (37, 50)).astype(np.uint8)
    for a, b in zip(V.pyramid_variant(P, 4, "none"), O.pyramid(P, 4)):
        assert np.array_equal(a, b)
    lp = V.pyramid_variant(P, 3, "binomial3")
    assert np.array_equal(lp[0], P.astype(np.float64))
    assert np.allclose(lp[1], V.lowpass_binomial3(O.reduce2(P)), rtol=0, atol=0)
    assert [x.shape for x in lp] == [(37, 50), (18, 25), (9, 12)]


def stencil_pins_hold(stencil):
    """E_x, E_y, E_t against scipy's correlation with the 3x3 masks."""
    rng = np.random.default_rng(5)
    P0 = rng.uniform(0, 255, (12, 15))
    P1 = rng.uniform(0, 255, (12, 15))
    ok = True
    for level in (0, 2):
        ex, ey, et, _ = VM.level_terms_variant(P0, P1, level, 48, 60, stencil)
        smooth = {"prewitt3": np.array([1.0, 1.0, 1.0]) / 3, "sobel3": np.array([1.0, 2.0, 1.0]) / 4}[stencil]
        mx = np.outer(smooth, [-0.5, 0.0, 0.5])
        c = lambda a, m: scipy.ndimage.correlate(a, m, mode="constant")[1:-1, 1:-1]
        s = 2.0 ** level
        ok &= np.allclose(ex, 0.5 * (c(P0, mx) + c(P1, mx)) / s, rtol=0, atol=1e-9)
        ok &= np.allclose(ey, 0.5 * (c(P0, mx.T) + c(P1, mx.T)) / s, rtol=0, atol=1e-9)
        ok &= np.allclose(et, c(P1 - P0, np.outer(smooth, smooth)), rtol=0, atol=1e-9)
    return bool(ok)


@pytest.mark.parametrize("stencil", ["prewitt3", "sobel3"])
def test_stencil_terms_are_the_masks(stencil):
    assert stencil_pins_hold(stencil)


def linear_pins_hold(stencil):
    """E = a x + b y + c t has E_x = a, E_y = b (per base pixel) and E_t = c at
    every position of every level without the low-pass, and with it outside
    the l outer rings of level l (the clamped border reaches one ring further
    per level through the block mean)."""
    a, b, c = 1.25, -0.75, 3.0
    H, W = 40, 56
    i, j = np.mgrid[0:H, 0:W].astype(np.float64)
    P0 = a * j + b * i + 100.0
    P1 = P0 + c
    ok = True
    for lowpass in ("none", "binomial3"):
        p0 = V.pyramid_variant(P0, 3, lowpass)
        p1 = V.pyramid_variant(P1, 3, lowpass)
        for l in range(3):
            ex, ey, et, _ = VM.level_terms_variant(p0[l], p1[l], l, H, W, stencil)
            cut = (slice(None), slice(None)) if lowpass == "none" or l == 0 else (slice(l, -l), slice(l, -l))
            ok &= np.allclose(ex[cut], a, atol=1e-12) and np.allclose(ey[cut], b, atol=1e-12)
            ok &= np.allclose(et[cut], c, atol=1e-12)
    return bool(ok)


@pytest.mark.parametrize("stencil", ["prewitt3", "sobel3"])
def test_linear_video_derivatives_exact(stencil):
    assert linear_pins_hold(stencil)


def symmetric_pins_hold(stencil, lowpass):
    """A video symmetric under the half-turn about the image centre has zero
    first-order sums and A = B = 0 (FOE at the centre), which fixes where the
    positions are taken."""
    v = synth.plain_ttc_video(H=64, W=80, F=2, symmetric=True)
    res = V.ttc_pair_variant(v.frames[0], v.frames[1], 3, stencil, lowpass)
    ok = True
    for r in res:
        a = np.abs(r["sums"]).max()
        ok &= all(abs(r["sums"][q]) <= 1e-12 * a for q in (3, 4, 6, 7))
        ok &= abs(r["x0"]) < 1e-6 and abs(r["y0"]) < 1e-6
    return bool(ok)


@pytest.mark.parametrize("stencil", ["cube", "prewitt3", "sobel3"])
@pytest.mark.parametrize("lowpass", ["none", "binomial3"])
def test_symmetric_video_foe_at_centre(stencil, lowpass):
    assert symmetric_pins_hold(stencil, lowpass)


def gt_pins_hold(stencil, lowpass):
    """The analytic TTC and FOE of approaching-plane videos (bounds of the cube's pin)."""
    v = synth.plain_ttc_video(H=96, W=96, F=3)
    ok = True
    for t in range(2):
        r = V.ttc_pair_variant(v.frames[t], v.frames[t + 1], 1, stencil, lowpass)[0]
        ok &= abs(r["ttc"] - 40.0) < 0.05 * 40.0 and abs(r["x0"]) < 0.5 and abs(r["y0"]) < 0.5
    w = synth.multiscale_video(H=120, W=160, F=2, foe=(20.0, -10.0), ttc_start=60, ttc_end=50)
    gt = w.ttc_gt()[0]
    for r in V.ttc_pair_variant(w.frames[0], w.frames[1], 3, stencil, lowpass):
        ok &= abs(r["ttc"] - gt) < 0.15 * gt and abs(r["x0"] - 20.0) < 1.5 and abs(r["y0"] + 10.0) < 2.0
    return bool(ok)


@pytest.mark.parametrize("stencil", ["cube", "prewitt3", "sobel3"])
@pytest.mark.parametrize("lowpass", ["none", "binomial3"])
def test_ground_truth_recovered(stencil, lowpass):
    assert gt_pins_hold(stencil, lowpass)


def test_cube_without_lowpass_is_the_plain_oracle():
    v = synth.multiscale_video(H=60, W=84, F=2, foe=(5.0, 3.0), ttc_start=40, ttc_end=38)
    a = V.ttc_pair_variant(v.frames[0], v.frames[1], 3, "cube", "none")
    b = O.ttc_pair(v.frames[0], v.frames[1], 3)
    for x, y in zip(a, b):
        assert np.array_equal(x["sums"], y["sums"]) and x["n"] == y["n"]
    assert a[1]["n"] == 29 * 41
    c = V.ttc_pair_variant(v.frames[0], v.frames[1], 3, "sobel3", "none")
    assert [r["n"] for r in c] == [58 * 82, 28 * 40, 13 * 19]


def _all_pins():
    return (lowpass_pins_hold() and all(stencil_pins_hold(s) and linear_pins_hold(s) for s in ("prewitt3", "sobel3"))
            and all(symmetric_pins_hold(s, lp) for s in ("prewitt3", "sobel3") for lp in ("none", "binomial3")))


@pytest.mark.parametrize("mutation", ["et_unsmoothed", "centre_offset", "lowpass_box", "no_level_scale",
                                      "transposed_mask"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    """Each mistake is planted in the oracle (CPU only) and must break a pin."""
    orig_terms = VM.level_terms_variant
    if mutation == "et_unsmoothed":
        def terms(P0, P1, level, H0, W0, stencil):
            ex, ey, et, g = orig_terms(P0, P1, level, H0, W0, stencil)
            if stencil != "cube":
                et = (np.asarray(P1, float) - np.asarray(P0, float))[1:-1, 1:-1]
            return ex, ey, et, g
        monkeypatch.setattr(VM, "level_terms_variant", terms)
    elif mutation == "centre_offset":
        def terms(P0, P1, level, H0, W0, stencil):
            ex, ey, et, g = orig_terms(P0, P1, level, H0, W0, stencil)
            if stencil != "cube":
                g = g + (2.0 ** level) * 0.5 * (ex + ey)  # positions at the pixel corner
            return ex, ey, et, g
        monkeypatch.setattr(VM, "level_terms_variant", terms)
    elif mutation == "lowpass_box":
        monkeypatch.setattr(VM, "lowpass_binomial3",
                            lambda img: scipy.ndimage.uniform_filter(np.asarray(img, float), 3, mode="nearest"))
    elif mutation == "no_level_scale":
        def terms(P0, P1, level, H0, W0, stencil):
            ex, ey, et, g = orig_terms(P0, P1, level, H0, W0, stencil)
            s = 2.0 ** level
            return ex * s, ey * s, et, g * s
        monkeypatch.setattr(VM, "level_terms_variant", terms)
    else:
        orig_masks = VM.stencil_masks
        monkeypatch.setattr(VM, "stencil_masks", lambda st: (lambda m: (m[0].T.copy(), m[1]))(orig_masks(st)))
    assert not _all_pins()
