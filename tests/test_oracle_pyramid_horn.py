"""Pins of the pyramid and derivative-cube oracles: hand-worked values, exact
identities of block averaging, linear-ramp videos (first differences are exact
for linear functions), and the tie to the (scipy-pinned) convolution oracle."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1612_08825_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_2x2_derivative():
    g = json.load(open(os.path.join(GOLDEN, "derivative_2x2_worked.json")))
    E = np.array(g["frame"], dtype=np.float64)
    ex, ey, et = O.horn(E, E)
    np.testing.assert_array_equal(ex, g["expected_Ex"])
    np.testing.assert_array_equal(ey, g["expected_Ey"])
    np.testing.assert_array_equal(et, np.zeros((2, 2)))
    ex, ey, et = O.horn(E, E + g["brighten"])
    np.testing.assert_array_equal(ex, g["expected_Ex"])
    np.testing.assert_array_equal(ey, g["expected_Ey"])
    np.testing.assert_array_equal(et, np.full((2, 2), g["expected_Et_after_brighten"]))


def test_pyramid_constant_and_sum():
    P = np.full((12, 18), 77, np.uint8)
    for lv in O.pyramid(P, 3):
        np.testing.assert_array_equal(lv, np.full(lv.shape, 77.0))
    R = synth.conv_image((32, 48), dtype="u8")
    levels = O.pyramid(R, 4)
    for a, b in zip(levels[:-1], levels[1:]):
        assert b.sum() == a.sum() / 4  # exact: all values are dyadic


def test_pyramid_reshape_mean_and_loops():
    R = synth.conv_image((27, 33), dtype="u8", case=3)
    h, w = 13, 16
    ref = R[: 2 * h, : 2 * w].astype(np.float64).reshape(h, 2, w, 2).mean(axis=(1, 3))
    np.testing.assert_array_equal(O.reduce2(R), ref)
    from oracle.pyramid import reduce2_loops

    np.testing.assert_array_equal(O.reduce2(R), reduce2_loops(R))
    assert O.pyramid(R, 3)[2].shape == (6, 8)  # floor(floor(27/2)/2), floor(floor(33/2)/2)


def test_pyramid_ramp_slope_doubles():
    a = 3.0
    P = np.tile(a * np.arange(64, dtype=np.float64), (8, 1))
    levels = O.pyramid(P, 4)
    for l, lv in enumerate(levels):
        d = np.diff(lv, axis=1)
        np.testing.assert_array_equal(d, np.full(d.shape, a * 2 ** l))


@pytest.mark.parametrize("a,b,c,d", [(2, -1, 3, 50), (0.5, 0.25, -1.5, 100), (0, 0, 0, 10)])
def test_ramp_video_exact(a, b, c, d):
    i, j = np.meshgrid(np.arange(9), np.arange(11), indexing="ij")
    P0 = a * j + b * i + d
    P1 = P0 + c
    ex, ey, et = O.horn(P0, P1)
    assert ex.shape == (8, 10)
    np.testing.assert_array_equal(ex, np.full(ex.shape, float(a)))
    np.testing.assert_array_equal(ey, np.full(ex.shape, float(b)))
    np.testing.assert_array_equal(et, np.full(ex.shape, float(c)))


def _cube_masks():
    # correlation masks indexed [frame c][row a][col b]
    kx = np.zeros((2, 2, 2))
    kx[:, :, 1] = 1
    kx[:, :, 0] = -1
    ky = np.zeros((2, 2, 2))
    ky[:, 1, :] = 1
    ky[:, 0, :] = -1
    kt = np.zeros((2, 2, 2))
    kt[1] = 1
    kt[0] = -1
    return kx, ky, kt


def test_horn_equals_valid_conv_of_stacked_pair():
    v = synth.plain_ttc_video(H=20, W=24, F=2)
    stack = v.frames.astype(np.int64)
    nx, ny, nt = O.horn_numerators(v.frames[0], v.frames[1])
    for mask, num in zip(_cube_masks(), (nx, ny, nt)):
        y = O.conv(stack, mask[::-1, ::-1, ::-1].astype(np.int64), "valid")
        assert y.shape == (1,) + num.shape
        np.testing.assert_array_equal(y[0], num)
    ex, ey, et = O.horn(v.frames[0], v.frames[1])
    np.testing.assert_array_equal(4 * ex, nx)
    np.testing.assert_array_equal(4 * ey, ny)
    np.testing.assert_array_equal(4 * et, nt)


def test_horn_f16_rendered_is_exact():
    v = synth.plain_ttc_video(H=16, W=16, F=2, dtype="f16")
    f = v.frames.astype(np.float64)
    # rendered f16 values in [16, 240] all lie on the 2^-6 grid, so the FP64 cube is exact
    assert np.all(f * 64 == np.rint(f * 64))
    ex, _, _ = O.horn(f[0], f[1])
    assert np.all(ex * 256 == np.rint(ex * 256))
